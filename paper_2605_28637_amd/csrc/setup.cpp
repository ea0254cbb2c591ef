// Host-side problem setup: validation, occupation shells, the plane-wave
// sphere in column order, FFT plans and the projector list.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "roks_internal.h"

namespace roks {

// The sphere keeps |G|^2/2 <= ecut (1 + kCutTol): points that sit on the
// cutoff within rounding are included, whatever the order of the sums.
static constexpr double kCutTol = 1e-10;

FftPlan1D make_plan(int n) {
  FftPlan1D p;
  p.n = n;
  int m = n;
  auto push = [&](int r) {
    ROKS_CHECK(p.nstages < kMaxStages, ROKS_ERR_SHAPE, "FFT size has too many factors");
    p.radix[p.nstages++] = r;
    m /= r;
  };
  while (m % 8 == 0) push(8);
  while (m % 4 == 0) push(4);
  while (m % 2 == 0) push(2);
  while (m % 3 == 0) push(3);
  while (m % 5 == 0) push(5);
  ROKS_CHECK(m == 1, ROKS_ERR_SHAPE, "FFT grid sizes must have only the prime factors 2, 3, 5");
  return p;
}

static void invert3(const double a[3][3], double inv[3][3]) {
  double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
               a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
               a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
  ROKS_CHECK(std::fabs(det) > 1e-12, ROKS_ERR_ARG, "cell is singular");
  inv[0][0] = (a[1][1] * a[2][2] - a[1][2] * a[2][1]) / det;
  inv[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / det;
  inv[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / det;
  inv[1][0] = (a[1][2] * a[2][0] - a[1][0] * a[2][2]) / det;
  inv[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / det;
  inv[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / det;
  inv[2][0] = (a[1][0] * a[2][1] - a[1][1] * a[2][0]) / det;
  inv[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / det;
  inv[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / det;
}

void grid_rule(const double cell[3][3], double ecut, int grid[3]) {
  // G_cut = pi N / (2 |a_d|), i.e. N >= 2 G_cut |a_d| / pi, rounded up to the
  // next size with factors 2, 3, 5 only (relative slack 1e-12 for the
  // rounding of an exact product)
  auto smooth = [](int v) {
    for (int f : {2, 3, 5})
      while (v % f == 0) v /= f;
    return v == 1;
  };
  for (int d = 0; d < 3; ++d) {
    const double ad = std::sqrt(cell[d][0] * cell[d][0] + cell[d][1] * cell[d][1] + cell[d][2] * cell[d][2]);
    const double need = 2.0 * std::sqrt(2.0 * ecut) * ad / M_PI;
    int n = need < 1e9 ? std::max(4, (int)std::ceil(need * (1.0 - 1e-12))) : (1 << 30);
    while (n < (1 << 30) && !smooth(n)) ++n;
    grid[d] = n;
  }
}

void build_problem(Ctx& c, const roks_system* s) {
  ROKS_CHECK(s != nullptr, ROKS_ERR_ARG, "system is NULL");
  std::memcpy(c.cell, s->cell, sizeof(c.cell));
  double inv[3][3];
  invert3(c.cell, inv);
  // b_i = 2 pi (a^-1)^T rows
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c.recip[i][j] = 2.0 * M_PI * inv[j][i];
  double det = c.cell[0][0] * (c.cell[1][1] * c.cell[2][2] - c.cell[1][2] * c.cell[2][1]) -
               c.cell[0][1] * (c.cell[1][0] * c.cell[2][2] - c.cell[1][2] * c.cell[2][0]) +
               c.cell[0][2] * (c.cell[1][0] * c.cell[2][1] - c.cell[1][1] * c.cell[2][0]);
  c.omega = std::fabs(det);
  ROKS_CHECK(s->ecut > 0 && std::isfinite(s->ecut), ROKS_ERR_ARG, "ecut must be > 0");
  c.ecut = s->ecut;
  const bool auto_grid = s->grid[0] == 0 && s->grid[1] == 0 && s->grid[2] == 0;
  int rule[3] = {0, 0, 0};
  if (auto_grid) grid_rule(c.cell, c.ecut, rule);
  for (int d = 0; d < 3; ++d) {
    const int n = auto_grid ? rule[d] : s->grid[d];
    ROKS_CHECK(n >= 4 && n <= 128, ROKS_ERR_SHAPE,
               "grid sizes must be in [4, 128] (or all 0 for the grid rule)");
    c.N[d] = n;
    c.plan[d] = make_plan(c.N[d]);
  }
  c.ntot = c.N[0] * c.N[1] * c.N[2];
  ROKS_CHECK(s->natoms >= 0, ROKS_ERR_ARG, "natoms < 0");
  c.natoms = s->natoms;
  ROKS_CHECK(s->nspecies >= 0 && (s->nspecies > 0 || s->natoms == 0), ROKS_ERR_ARG,
             "atoms need species");
  c.species.clear();
  for (int i = 0; i < s->nspecies; ++i) {
    const roks_species& sp = s->spec[i];
    Ctx::Species o;
    ROKS_CHECK(std::isfinite(sp.A) && sp.sigma > 0, ROKS_ERR_ARG, "species needs sigma > 0");
    o.A = sp.A;
    o.sigma = sp.sigma;
    ROKS_CHECK(sp.nproj >= 0 && sp.nproj <= 16, ROKS_ERR_ARG, "species nproj out of range");
    ROKS_CHECK(sp.nproj == 0 || (sp.proj && sp.D), ROKS_ERR_ARG, "projector arrays are NULL");
    for (int p = 0; p < sp.nproj; ++p) {
      ROKS_CHECK(sp.proj[p].l == 0 || sp.proj[p].l == 1, ROKS_ERR_ARG, "projector l must be 0 or 1");
      ROKS_CHECK(sp.proj[p].rp > 0, ROKS_ERR_ARG, "projector radius must be > 0");
      o.l.push_back(sp.proj[p].l);
      o.rp.push_back(sp.proj[p].rp);
    }
    o.D.assign(sp.D, sp.D + (size_t)sp.nproj * sp.nproj);
    for (int p = 0; p < sp.nproj; ++p)
      for (int q = 0; q < sp.nproj; ++q) {
        double a = o.D[p * sp.nproj + q], b = o.D[q * sp.nproj + p];
        ROKS_CHECK(std::fabs(a - b) <= 1e-14 * (std::fabs(a) + std::fabs(b)) + 0.0, ROKS_ERR_ARG,
                   "D must be symmetric");
        ROKS_CHECK(o.l[p] == o.l[q] || a == 0.0, ROKS_ERR_ARG, "D couples different l");
      }
    // overlap coefficients (NULL: S = 1), checked like D
    o.q.assign((size_t)sp.nproj * sp.nproj, 0.0);
    if (sp.q && sp.nproj > 0) o.q.assign(sp.q, sp.q + (size_t)sp.nproj * sp.nproj);
    for (int p = 0; p < sp.nproj; ++p)
      for (int q = 0; q < sp.nproj; ++q) {
        double a = o.q[p * sp.nproj + q], b = o.q[q * sp.nproj + p];
        ROKS_CHECK(std::isfinite(a), ROKS_ERR_ARG, "non-finite q");
        ROKS_CHECK(std::fabs(a - b) <= 1e-14 * (std::fabs(a) + std::fabs(b)), ROKS_ERR_ARG,
                   "q must be symmetric");
        ROKS_CHECK(o.l[p] == o.l[q] || a == 0.0, ROKS_ERR_ARG, "q couples different l");
      }
    c.species.push_back(o);
  }
  c.spec_of.assign(s->species, s->species + c.natoms);
  for (int a = 0; a < c.natoms; ++a)
    ROKS_CHECK(c.spec_of[a] >= 0 && c.spec_of[a] < s->nspecies, ROKS_ERR_ARG, "bad species index");
  c.pos.assign(s->pos, s->pos + 3 * (size_t)c.natoms);
  for (double v : c.pos) ROKS_CHECK(std::isfinite(v), ROKS_ERR_ARG, "non-finite position");

  ROKS_CHECK(s->nbands >= 1 && s->nbands <= 4096, ROKS_ERR_ARG, "nbands out of range");
  ROKS_CHECK(s->nconfig == 1 || s->nconfig == 2, ROKS_ERR_ARG, "nconfig must be 1 or 2");
  c.nb = s->nbands;
  c.nconf = s->nconfig;
  c.occ.assign(s->occ, s->occ + (size_t)c.nconf * 2 * c.nb);
  for (uint8_t v : c.occ) ROKS_CHECK(v <= 1, ROKS_ERR_ARG, "occupations must be 0 or 1");
  for (int L = 0; L < c.nconf; ++L) {
    ROKS_CHECK(std::isfinite(s->cL[L]), ROKS_ERR_ARG, "non-finite c_L");
    c.cL[L] = s->cL[L];
  }
  ROKS_CHECK(s->xc == ROKS_XC_PW92 || s->xc == ROKS_XC_X || s->xc == ROKS_XC_PBE, ROKS_ERR_ARG,
             "unknown xc");
  c.xc = s->xc;
  ROKS_CHECK(std::isfinite(s->exx) && s->exx >= 0.0 && s->exx <= 1.0, ROKS_ERR_ARG,
             "exact-exchange fraction outside [0, 1]");
  ROKS_CHECK(s->exx == 0.0 || s->xc == ROKS_XC_PBE, ROKS_ERR_ARG, "exact exchange is mixed with PBE only");
  c.exx = s->exx;
  ROKS_CHECK(s->precision == ROKS_FP64 || s->precision == ROKS_FP32 || s->precision == ROKS_FP32_BF16X3,
             ROKS_ERR_ARG, "precision tier not available");
  // the FFT tier; the projector products follow the BF16x3 flag
  c.prec = s->precision == ROKS_FP64 ? ROKS_FP64 : ROKS_FP32;
  c.bf3 = s->precision == ROKS_FP32_BF16X3;
  ROKS_CHECK((s->flags & ~31u) == 0, ROKS_ERR_ARG, "unknown flag bits");
  c.flags = s->flags;

  // shells: closed (all ones), open patterns by first appearance, virtual (all zeros)
  const int np = 2 * c.nconf;
  auto pattern = [&](int n) {
    uint32_t p = 0;
    for (int L = 0; L < c.nconf; ++L)
      for (int sp = 0; sp < 2; ++sp) p |= (uint32_t)c.occ[(L * 2 + sp) * c.nb + n] << (L * 2 + sp);
    return p;
  };
  const uint32_t full = (1u << np) - 1u;
  std::vector<uint32_t> order;
  bool has_full = false, has_empty = false;
  for (int n = 0; n < c.nb; ++n) {
    uint32_t p = pattern(n);
    if (p == full) has_full = true;
    if (p == 0) has_empty = true;
  }
  if (has_full) order.push_back(full);
  for (int n = 0; n < c.nb; ++n) {
    uint32_t p = pattern(n);
    if (p != full && p != 0 && std::find(order.begin(), order.end(), p) == order.end())
      order.push_back(p);
  }
  if (has_empty) order.push_back(0u);
  ROKS_CHECK((int)order.size() <= kMaxShell, ROKS_ERR_ARG, "at most 4 occupation shells");
  c.nshell = (int)order.size();
  c.nsocc = has_empty ? c.nshell - 1 : c.nshell;
  ROKS_CHECK(c.nsocc >= 1, ROKS_ERR_ARG, "no occupied band");
  ROKS_CHECK(c.nsocc <= 3, ROKS_ERR_ARG, "at most 3 occupied shells (closed and two open)");
  c.band_shell.resize(c.nb);
  for (int n = 0; n < c.nb; ++n) {
    uint32_t p = pattern(n);
    c.band_shell[n] = (int)(std::find(order.begin(), order.end(), p) - order.begin());
    if (n > 0)
      ROKS_CHECK(c.band_shell[n] >= c.band_shell[n - 1], ROKS_ERR_ARG,
                 "bands must be ordered closed, open shells, virtual");
  }
  for (int X = 0; X < c.nshell; ++X) {
    double w = 0;
    for (int L = 0; L < c.nconf; ++L)
      for (int sp = 0; sp < 2; ++sp) {
        double f = (order[X] >> (L * 2 + sp)) & 1u;
        c.shell_f[X][L][sp] = f;
        w += c.cL[L] * f;
      }
    c.shell_w[X] = w;
    c.shell_closed[X] = order[X] == full;
    c.shell_virtual[X] = order[X] == 0u;
  }
}

void build_sphere(Ctx& c) {
  const double two_e = 2.0 * c.ecut * (1.0 + kCutTol);
  const double gcut = std::sqrt(two_e);
  int hm[3];
  for (int d = 0; d < 3; ++d) {
    double len = std::sqrt(c.cell[d][0] * c.cell[d][0] + c.cell[d][1] * c.cell[d][1] +
                           c.cell[d][2] * c.cell[d][2]);
    hm[d] = (int)std::floor(gcut * len / (2.0 * M_PI)) + 1;
  }
  auto g2of = [&](int h, int k, int l) {
    double g[3];
    for (int i = 0; i < 3; ++i)
      g[i] = (double)h * c.recip[0][i] + (double)k * c.recip[1][i] + (double)l * c.recip[2][i];
    return g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  };
  c.cols.clear();
  c.miller.clear();
  c.g2half.clear();
  c.hmax = 0;
  int maxabs[3] = {0, 0, 0};
  auto add_column = [&](int h, int k, bool only_nonneg) {
    int lmin = 1 << 30, lmax = -(1 << 30);
    for (int l = -hm[2]; l <= hm[2]; ++l) {
      if (only_nonneg && l < 0) continue;
      if (g2of(h, k, l) <= two_e) {
        lmin = std::min(lmin, l);
        lmax = std::max(lmax, l);
      }
    }
    if (lmax < lmin) return;
    ColDesc d;
    d.h = h;
    d.k = k;
    d.lmin = lmin;
    d.lmax = lmax;
    d.base = (int32_t)(c.miller.size() / 3);
    for (int l = lmin; l <= lmax; ++l) {
      ROKS_CHECK(g2of(h, k, l) <= two_e, ROKS_ERR_SHAPE, "sphere column is not contiguous");
      c.miller.push_back(h);
      c.miller.push_back(k);
      c.miller.push_back(l);
      c.g2half.push_back(0.5 * g2of(h, k, l));
      maxabs[2] = std::max(maxabs[2], std::abs(l));
    }
    maxabs[0] = std::max(maxabs[0], std::abs(h));
    maxabs[1] = std::max(maxabs[1], std::abs(k));
    c.cols.push_back(d);
  };
  add_column(0, 0, true);
  ROKS_CHECK(!c.cols.empty(), ROKS_ERR_ARG, "empty sphere");
  for (int h = -hm[0]; h <= hm[0]; ++h)
    for (int k = -hm[1]; k <= hm[1]; ++k)
      if (k > 0 || (k == 0 && h > 0)) add_column(h, k, false);
  c.npw = (int)(c.miller.size() / 3);
  c.nH = (int)c.cols.size() - 1;
  c.ncol = 2 * c.nH + 1;
  for (int d = 0; d < 3; ++d)
    ROKS_CHECK(2 * maxabs[d] < c.N[d], ROKS_ERR_SHAPE,
               "the plane-wave sphere does not fit the FFT grid (need N > 2 max|m|)");
  c.hmax = maxabs[0];
  ROKS_CHECK(c.miller[0] == 0 && c.miller[1] == 0 && c.miller[2] == 0, ROKS_ERR_SHAPE,
             "G = 0 must be the first plane wave");
}

void build_projectors(Ctx& c) {
  c.proj_atom.clear();
  c.proj_l.clear();
  c.proj_m.clear();
  c.proj_rp.clear();
  c.atom_proj_off.assign(c.natoms, 0);
  c.atom_proj_cnt.assign(c.natoms, 0);
  c.Dblk.clear();
  c.Qblk.clear();
  c.has_q = false;
  c.Dblk_off.assign(c.natoms, 0);
  for (int a = 0; a < c.natoms; ++a) {
    const Ctx::Species& sp = c.species[c.spec_of[a]];
    c.atom_proj_off[a] = (int)c.proj_atom.size();
    std::vector<int> chan, mm;
    for (size_t p = 0; p < sp.l.size(); ++p) {
      int nm = sp.l[p] == 0 ? 1 : 3;
      for (int m = 0; m < nm; ++m) {
        c.proj_atom.push_back(a);
        c.proj_l.push_back(sp.l[p]);
        c.proj_m.push_back(m);
        c.proj_rp.push_back(sp.rp[p]);
        chan.push_back((int)p);
        mm.push_back(m);
      }
    }
    int na = (int)chan.size();
    c.atom_proj_cnt[a] = na;
    c.Dblk_off[a] = (int)c.Dblk.size();
    const int np = (int)sp.l.size();
    for (int i = 0; i < na; ++i)
      for (int j = 0; j < na; ++j) {
        double v = 0, w = 0;
        if (sp.l[chan[i]] == sp.l[chan[j]] && mm[i] == mm[j]) {
          v = sp.D[chan[i] * np + chan[j]];
          w = sp.q[chan[i] * np + chan[j]];
        }
        c.Dblk.push_back(v);
        c.Qblk.push_back(w);
        c.has_q = c.has_q || w != 0.0;
      }
  }
  c.nproj = (int)c.proj_atom.size();
}

}  // namespace roks
