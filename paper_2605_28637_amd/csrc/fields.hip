// Pointwise and reduction kernels: external potential, projector tables,
// shell densities, Hartree and spin-LDA exchange-correlation potentials,
// energy terms and forces.  All reductions use a fixed block count and a
// fixed order (partials, then an ordered sum), so results are reproducible.
#include <cmath>

#include "roks_internal.h"

namespace roks {

namespace {

constexpr int kRedBlocks = 1024;

struct Lattice {
  double b[3][3];  // reciprocal vectors (rows)
  int N[3];
  double omega;
};

Lattice lattice(const Ctx& c) {
  Lattice L;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) L.b[i][j] = c.recip[i][j];
  for (int d = 0; d < 3; ++d) L.N[d] = c.N[d];
  L.omega = c.omega;
  return L;
}

// grid index [z][x][y] -> signed frequencies (h, k, l); returns true on a
// Nyquist plane of an even grid
__device__ __forceinline__ bool grid_freq(const Lattice& L, size_t i, int* m) {
  const int np2 = L.N[0] * L.N[1];
  const int z = (int)(i / np2);
  const int r = (int)(i - (size_t)z * np2);
  const int x = r / L.N[1], y = r - x * L.N[1];
  const int idx[3] = {x, y, z};
  bool nyq = false;
  for (int d = 0; d < 3; ++d) {
    int v = idx[d];
    if (2 * v >= L.N[d]) v -= L.N[d];
    if ((L.N[d] & 1) == 0 && 2 * v == -L.N[d]) nyq = true;
    m[d] = v;
  }
  return nyq;
}

__device__ __forceinline__ void gvec(const Lattice& L, const int* m, double* G) {
  for (int a = 0; a < 3; ++a) G[a] = m[0] * L.b[0][a] + m[1] * L.b[1][a] + m[2] * L.b[2][a];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block sum of k values per thread (k <= 8); result valid in thread 0
template <int K>
__device__ void block_sum(double (&v)[K], double* red) {
  const int tid = threadIdx.x, nw = blockDim.x >> 6, wid = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double s = wave_sum(v[j]);
    if (lane == 0) red[j * 16 + wid] = s;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double s = 0;
      for (int w = 0; w < nw; ++w) s += red[j * 16 + w];
      v[j] = s;
    }
  }
  __syncthreads();
}

struct AtomP {
  double x, y, z, A, sigma;
};

// ---------------------------------------------------------------------------
// V_ext(G) on the grid: Omega^-1 sum_I v_s(G) e^{-iG.R_I}; Nyquist planes zero
// ---------------------------------------------------------------------------
__global__ void k_vext_G(Lattice L, const AtomP* __restrict__ atoms, int natoms,
                         double2* __restrict__ out, size_t ntot) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    int m[3];
    const bool nyq = grid_freq(L, i, m);
    double G[3];
    gvec(L, m, G);
    const double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
    double re = 0, im = 0;
    if (!nyq) {
      for (int a = 0; a < natoms; ++a) {
        const AtomP p = atoms[a];
        const double s2 = p.sigma * p.sigma;
        const double vs = -p.A * pow(2.0 * M_PI * s2, 1.5) * exp(-0.5 * g2 * s2);
        const double th = G[0] * p.x + G[1] * p.y + G[2] * p.z;
        double sn, cs;
        sincos(th, &sn, &cs);
        re += vs * cs;
        im -= vs * sn;
      }
    }
    out[i] = make_double2(re / L.omega, im / L.omega);
  }
}

__global__ void k_to_float(const double* __restrict__ in, float* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

__global__ void k_take_real(const double2* __restrict__ in, double* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = in[i].x;
}

// ---------------------------------------------------------------------------
// projector table beta_i(G) = Omega^-1/2 f_i(G) e^{-iG.R} (optionally times -iG_a)
// ---------------------------------------------------------------------------
struct ProjP {
  int atom, l, m;
  double rp;
};

// the table of projectors (axis = -1) or of their derivative along `axis`
__global__ void k_projectors(Lattice L, const int32_t* __restrict__ miller, int npw,
                             const ProjP* __restrict__ proj, int nproj,
                             const AtomP* __restrict__ atoms, int axis, double2* __restrict__ B) {
  const size_t total = (size_t)nproj * npw;
  const double inv_sqrt_omega = 1.0 / sqrt(L.omega);
  const double c0 = 4.0 * M_PI;
  const double c1 = 4.0 * pow(M_PI, 0.75);
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(t / npw), g = (int)(t - (size_t)i * npw);
    const int m[3] = {miller[3 * g], miller[3 * g + 1], miller[3 * g + 2]};
    double G[3];
    gvec(L, m, G);
    const double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
    const ProjP p = proj[i];
    const AtomP a = atoms[p.atom];
    const double e = exp(-0.5 * g2 * p.rp * p.rp) * inv_sqrt_omega;
    const double th = G[0] * a.x + G[1] * a.y + G[2] * a.z;
    double sn, cs;
    sincos(th, &sn, &cs);
    double2 v;
    if (p.l == 0) {
      const double f = pow(c0 * p.rp * p.rp, 0.75) * e;
      v = make_double2(f * cs, -f * sn);
    } else {
      const double f = c1 * pow(p.rp, 2.5) * e * G[p.m];
      // -i f (cos - i sin) = f (-sin, -cos)
      v = make_double2(-f * sn, -f * cs);
    }
    if (axis >= 0) {
      const double ga = G[axis];
      v = make_double2(ga * v.y, -ga * v.x);  // times -i G_a
    }
    B[t] = v;
  }
}

// Cartesian G of every stored coefficient, [3][npw] (the derivative of a
// projector's table is -i G_a times the table)
__global__ void k_gcart(Lattice L, const int32_t* __restrict__ miller, int npw, double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npw) return;
  const int m[3] = {miller[3 * g], miller[3 * g + 1], miller[3 * g + 2]};
  double G[3];
  gvec(L, m, G);
  for (int a = 0; a < 3; ++a) out[(size_t)a * npw + g] = G[a];
}

// ---------------------------------------------------------------------------
// densities
// ---------------------------------------------------------------------------
struct ShellArgs {
  int nconf, nsocc, xc;
  int same_rho;  // every configuration has the same total occupation of each shell
  double f[3][kMaxConf][2];
  double cL[kMaxConf];
};

// configuration densities rho_L = sum_X (f_X^up + f_X^dn) rho_X packed as rho_0 + i rho_1
__global__ void k_pack_rho(ShellArgs a, const double* __restrict__ rho, size_t ntot,
                           double2* __restrict__ out, int weighted) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    double r[kMaxConf] = {0, 0};
    for (int X = 0; X < a.nsocc; ++X) {
      const double v = rho[(size_t)X * ntot + i];
      for (int L = 0; L < a.nconf; ++L) r[L] += (a.f[X][L][0] + a.f[X][L][1]) * v;
    }
    if (weighted) {
      double s = 0;
      for (int L = 0; L < a.nconf; ++L) s += a.cL[L] * r[L];
      out[i] = make_double2(s, 0.0);
    } else {
      out[i] = make_double2(r[0], a.nconf > 1 ? r[1] : 0.0);
    }
  }
}

// the shell densities from the plane passes' chunk partials (summed in chunk
// order, / Omega), and the same pass packs the configuration densities for
// the Hartree transform as k_pack_rho (weighted = 0) does
__global__ void k_density_reduce(ShellArgs a, const double* __restrict__ part, int nchunk,
                                 size_t ntot, double inv_omega, double* __restrict__ rho,
                                 double2* __restrict__ packed) {
  const size_t total = (size_t)a.nsocc * ntot;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    double r[kMaxConf] = {0, 0};
    for (int X = 0; X < a.nsocc; ++X) {
      const size_t t = (size_t)X * ntot + i;
      double s = 0;
      for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * total + t];
      const double v = s * inv_omega;
      rho[t] = v;
      for (int L = 0; L < a.nconf; ++L) r[L] += (a.f[X][L][0] + a.f[X][L][1]) * v;
    }
    packed[i] = make_double2(r[0], a.nconf > 1 ? r[1] : 0.0);
  }
}

// Hartree integrals sum_r V_H,L(r) rho_L(r) = sum_{G != 0} 4 pi |F_L(G)|^2 / (G^2 N^3)
// straight from the packed transform F = FFT(rho_0 + i rho_1) (no inverse
// transform): F_0 = (F(G) + F(-G)*)/2, F_1 = (F(G) - F(-G)*)/(2i); per-block
// partials [block][2], fixed order
__global__ void __launch_bounds__(256) k_hartree_energy(Lattice L, const double2* __restrict__ f,
                                                        size_t ntot, int nconf,
                                                        double* __restrict__ part) {
  __shared__ double red[8 * 16];
  double acc[2] = {0.0, 0.0};
  const double inv = 1.0 / (double)ntot;
  const int np2 = L.N[0] * L.N[1];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    int m[3];
    grid_freq(L, i, m);
    double G[3];
    gvec(L, m, G);
    const double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
    if (g2 > 0.0) {
      const int z = (int)(i / np2);
      const int r = (int)(i - (size_t)z * np2);
      const int x = r / L.N[1], y = r - x * L.N[1];
      const int xm = x ? L.N[0] - x : 0, ym = y ? L.N[1] - y : 0, zm = z ? L.N[2] - z : 0;
      const double2 a = f[i];
      const double2 b = f[(size_t)zm * np2 + (size_t)xm * L.N[1] + ym];
      const double w = 4.0 * M_PI * inv / g2;
      const double mx = 0.5 * (a.x + b.x), my = 0.5 * (a.y - b.y);
      acc[0] += w * (mx * mx + my * my);
      if (nconf > 1) {
        const double tx = 0.5 * (a.y + b.y), ty = -0.5 * (a.x - b.x);
        acc[1] += w * (tx * tx + ty * ty);
      }
    }
  }
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    part[(size_t)blockIdx.x * 2] = acc[0];
    part[(size_t)blockIdx.x * 2 + 1] = acc[1];
  }
}

// ---------------------------------------------------------------------------
// spin LDA: Slater exchange + Perdew-Wang 1992 correlation
// ---------------------------------------------------------------------------
template <bool DERIV>
__device__ void pw92_G(double rs, double srs, double isrs, double A, double a1, double b1, double b2,
                       double b3, double b4, double* G, double* dG) {
  const double Q = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs);
  const double lg = log1p(1.0 / Q);
  *G = -2.0 * A * (1.0 + a1 * rs) * lg;
  if (DERIV) {
    const double dQ = 2.0 * A * (0.5 * b1 * isrs + b2 + 1.5 * b3 * srs + 2.0 * b4 * rs);
    *dG = -2.0 * A * a1 * lg + 2.0 * A * (1.0 + a1 * rs) * dQ / (Q * Q + Q);
  }
}

// The parts of a spin-LDA point that depend on the total density only: rho^(1/3)
// and the three PW92 G functions of r_s (with their r_s derivatives for the
// potentials).  Configurations with the same total density share them.
struct LdaRho {
  double rho, crho, rs, ec0, dec0, ec1, dec1, ac, dac;
};

// (6/pi)^(1/3), 2^(-1/3), (3/(4 pi))^(1/3), 2^(4/3) - 2
constexpr double kCx = 1.2407009817988, kCbrtHalf = 0.7937005259840998;
constexpr double kRsCoef = 0.6203504908994, kFzDen = 0.5198420997897464;

template <bool DERIV>
__device__ void lda_rho(double rho, int kind, LdaRho* r) {
  r->rho = rho;
  if (rho < 1e-12) return;
  r->crho = cbrt(rho);
  if (kind == ROKS_XC_X) return;
  const double rs = kRsCoef / r->crho;
  const double srs = sqrt(rs), isrs = DERIV ? 1.0 / srs : 0.0;
  r->rs = rs;
  double mac, dmac = 0.0;
  pw92_G<DERIV>(rs, srs, isrs, 0.031091, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294, &r->ec0, &r->dec0);
  pw92_G<DERIV>(rs, srs, isrs, 0.015545, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517, &r->ec1, &r->dec1);
  pw92_G<DERIV>(rs, srs, isrs, 0.016887, 0.11125, 10.357, 3.6231, 0.88026, 0.49671, &mac, &dmac);
  r->ac = -mac;
  r->dac = -dmac;
}

// energy density e and (DERIV) potentials of spin densities (ru, rd) whose sum
// is r.rho: Slater exchange + PW92 correlation, spin interpolation f(zeta)
template <bool DERIV>
__device__ void lda_spin(double ru, double rd, const LdaRho& r, int kind, double* e, double* vu,
                         double* vd) {
  const double rho = r.rho;
  if (rho < 1e-12) {
    *e = 0.0;
    *vu = 0.0;
    *vd = 0.0;
    return;
  }
  const double third = 1.0 / 3.0;
  // rho_up,down = rho (1 +- z) / 2, so (rho_up,down)^(1/3) = rho^(1/3) 2^(-1/3) (1 +- z)^(1/3)
  double z = (ru - rd) / rho;
  z = fmin(1.0, fmax(-1.0, z));
  const double opz = 1.0 + z, omz = 1.0 - z;
  const double copz = cbrt(opz), comz = cbrt(omz);
  const double ch = r.crho * kCbrtHalf;
  const double cu = ch * copz, cd = ch * comz;
  const double ex = -0.75 * kCx * (ru * cu + rd * cd);
  const double vxu = -kCx * cu, vxd = -kCx * cd;
  if (kind == ROKS_XC_X) {
    *e = ex;
    *vu = vxu;
    *vd = vxd;
    return;
  }
  const double fz20 = 1.709921;
  const double f = (opz * copz + omz * comz - 2.0) / kFzDen;
  const double z3 = z * z * z, z4 = z3 * z;
  const double ec0 = r.ec0, ec1 = r.ec1, ac = r.ac;
  const double eps = ec0 + ac * f / fz20 * (1.0 - z4) + (ec1 - ec0) * f * z4;
  *e = ex + rho * eps;
  if (DERIV) {
    const double fp = (4.0 * third) * (copz - comz) / kFzDen;
    const double deps_rs = r.dec0 + r.dac * f / fz20 * (1.0 - z4) + (r.dec1 - r.dec0) * f * z4;
    const double deps_z =
        4.0 * z3 * f * (ec1 - ec0 - ac / fz20) + fp * (z4 * (ec1 - ec0) + (1.0 - z4) * ac / fz20);
    const double common = eps - r.rs * third * deps_rs;
    *vu = vxu + common + (1.0 - z) * deps_z;
    *vd = vxd + common - (1.0 + z) * deps_z;
  }
}

// per point: configuration spin densities, LDA, V_loc^{sigma L}, shell potentials
// V^X = sum c_L f_X V_loc^{sigma L}; partial sums of e_xc, V_ext rho, V_H rho per L.
// WRITE = false: energy sums only (xc and external; no V_H read, no potentials,
// no derivatives).  With a.same_rho every configuration has the total density
// of configuration 0 and shares its r_s part.  vh: the Hartree potentials as
// the inverse transform leaves them, V_H^0 + i V_H^1 per point.
template <bool WRITE>
__global__ void __launch_bounds__(256) k_xc(ShellArgs a, const double* __restrict__ rho,
                                            const double* __restrict__ vext,
                                            const double2* __restrict__ vh, size_t ntot,
                                            double* __restrict__ vloc, double* __restrict__ vsh,
                                            double* __restrict__ part) {
  __shared__ double red[8 * 16];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    double rX[3] = {0, 0, 0};
    for (int X = 0; X < a.nsocc; ++X) rX[X] = rho[(size_t)X * ntot + i];
    const double ve = vext[i];
    const double2 vhp = WRITE ? vh[i] : make_double2(0.0, 0.0);
    double vl[kMaxConf][2];
    LdaRho lr;
    for (int L = 0; L < a.nconf; ++L) {
      double ru = 0, rd = 0;
      for (int X = 0; X < a.nsocc; ++X) {
        ru += a.f[X][L][0] * rX[X];
        rd += a.f[X][L][1] * rX[X];
      }
      ru = fmax(ru, 0.0);
      rd = fmax(rd, 0.0);
      if (L == 0 || !a.same_rho) lda_rho<WRITE>(ru + rd, a.xc, &lr);
      double e, vu, vd;
      lda_spin<WRITE>(ru, rd, lr, a.xc, &e, &vu, &vd);
      acc[3 * L + 0] += e;
      acc[3 * L + 1] += ve * (ru + rd);
      if (!WRITE) continue;
      const double h = L == 0 ? vhp.x : vhp.y;
      vl[L][0] = ve + h + vu;
      vl[L][1] = ve + h + vd;
      vloc[(size_t)(2 * L) * ntot + i] = vl[L][0];
      vloc[(size_t)(2 * L + 1) * ntot + i] = vl[L][1];
      acc[3 * L + 2] += h * (ru + rd);
    }
    if (!WRITE) continue;
    for (int X = 0; X < a.nsocc; ++X) {
      double s = 0;
      for (int L = 0; L < a.nconf; ++L)
        s += a.cL[L] * (a.f[X][L][0] * vl[L][0] + a.f[X][L][1] * vl[L][1]);
      vsh[(size_t)X * ntot + i] = s;
    }
  }
  block_sum<6>(acc, red);
  if (threadIdx.x == 0)
    for (int j = 0; j < 6; ++j) part[(size_t)blockIdx.x * 6 + j] = acc[j];
}

// out[j] = sum_r part[r][j] (also into mirror[j] when given); one workgroup per
// column, fixed summation tree.  Workgroups past ncols take the columns of a
// second array part2 [nrows][gridDim.x - ncols], continuing out and mirror.
__global__ void __launch_bounds__(256) k_reduce_columns(const double* __restrict__ part, int nrows,
                                                        int ncols, double* __restrict__ out,
                                                        double* __restrict__ mirror,
                                                        const double* __restrict__ part2) {
  __shared__ double red[8 * 16];
  const int jo = blockIdx.x;
  const bool second = jo >= ncols;
  const double* src = second ? part2 : part;
  const int nc = second ? (int)gridDim.x - ncols : ncols;
  const int j = second ? jo - ncols : jo;
  double v[1] = {0.0};
  for (int r = threadIdx.x; r < nrows; r += blockDim.x) v[0] += src[(size_t)r * nc + j];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) {
    out[jo] = v[0];
    if (mirror) mirror[jo] = v[0];
  }
}

// ---------------------------------------------------------------------------
// nonlocal energies and D application (per-atom dense blocks)
// ---------------------------------------------------------------------------
// e_n = sum_atoms sum_ij P_in D_ij P_jn (also into mirror[n] when given): one
// wave per band, atoms split over lanes
__global__ void __launch_bounds__(64) k_nl_energy(const double* __restrict__ P, int nb, int natoms,
                                                  const int32_t* __restrict__ off,
                                                  const int32_t* __restrict__ cnt,
                                                  const int32_t* __restrict__ doff,
                                                  const double* __restrict__ D,
                                                  double* __restrict__ out,
                                                  double* __restrict__ mirror) {
  const int n = blockIdx.x;
  double s = 0;
  for (int a = threadIdx.x; a < natoms; a += blockDim.x) {
    const int o = off[a], k = cnt[a];
    const double* Da = D + doff[a];
    for (int i = 0; i < k; ++i) {
      const double pi = P[(size_t)(o + i) * nb + n];
      double t = 0;
      for (int j = 0; j < k; ++j) t += Da[i * k + j] * P[(size_t)(o + j) * nb + n];
      s += pi * t;
    }
  }
  s = wave_sum(s);
  if (threadIdx.x == 0) {
    out[n] = s;
    if (mirror) mirror[n] = s;
  }
}

__global__ void k_apply_D(const double* __restrict__ P, int nb, int nproj,
                          const int32_t* __restrict__ patom, const int32_t* __restrict__ off,
                          const int32_t* __restrict__ cnt, const int32_t* __restrict__ doff,
                          const double* __restrict__ D, const double* __restrict__ w,
                          double* __restrict__ DP) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (t >= (size_t)nproj * nb) return;
  const int i = (int)(t / nb), n = (int)(t - (size_t)i * nb);
  const int a = patom[i];
  const int o = off[a], k = cnt[a];
  const double* Da = D + doff[a] + (i - o) * k;
  double s = 0;
  for (int j = 0; j < k; ++j) s += Da[j] * P[(size_t)(o + j) * nb + n];
  DP[t] = (w ? w[n] : 1.0) * s;
}

// ---------------------------------------------------------------------------
// forces
// ---------------------------------------------------------------------------
// partial sums over G of v_s(G) G_a Im(e^{-iG.R_I} conj(rho(G))), rho(G) already / N^3
// The structure factor e^{-i G.R} = prod_d e^{-i m_d (b_d . R)} comes from
// three per-axis phase tables of the workgroup's atom (index = grid index,
// frequency wrapped), built once per workgroup in LDS.  With an orthogonal
// reciprocal basis (orth) the Gaussian exp(-sigma^2 |G|^2 / 2) factorises
// over the axes too and is folded into the tables.
constexpr int kMaxAxis = 256;

__global__ void __launch_bounds__(256) k_local_force(Lattice L, const AtomP* __restrict__ atoms,
                                                     const double2* __restrict__ rg, size_t ntot,
                                                     double scale, int orth, double* __restrict__ part) {
  __shared__ double red[8 * 16];
  __shared__ double2 ph[3][kMaxAxis];  // (cos, sin) of m_d (b_d . R) [x Gaussian factor]
  const int I = blockIdx.y;
  const AtomP p = atoms[I];
  const double s2 = p.sigma * p.sigma;
  const double pre = -p.A * pow(2.0 * M_PI * s2, 1.5);
  for (int d = 0; d < 3; ++d) {
    const double bR = L.b[d][0] * p.x + L.b[d][1] * p.y + L.b[d][2] * p.z;
    const double bb = L.b[d][0] * L.b[d][0] + L.b[d][1] * L.b[d][1] + L.b[d][2] * L.b[d][2];
    for (int v = threadIdx.x; v < L.N[d]; v += blockDim.x) {
      const int m = 2 * v >= L.N[d] ? v - L.N[d] : v;
      double sn, cs;
      sincos(m * bR, &sn, &cs);
      const double gs = orth ? exp(-0.5 * s2 * (double)m * m * bb) : 1.0;
      ph[d][v] = make_double2(gs * cs, gs * sn);
    }
  }
  __syncthreads();
  double acc[3] = {0, 0, 0};
  const int np2 = L.N[0] * L.N[1];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    int m[3];
    if (grid_freq(L, i, m)) continue;
    double G[3];
    gvec(L, m, G);
    const double vs = orth ? pre : pre * exp(-0.5 * (G[0] * G[0] + G[1] * G[1] + G[2] * G[2]) * s2);
    // grid indices of the frequencies (x, y, z) for the tables
    const int z = (int)(i / np2);
    const int rr = (int)(i - (size_t)z * np2);
    const int x = rr / L.N[1], y = rr - x * L.N[1];
    const double2 a = ph[0][x], b = ph[1][y], e = ph[2][z];
    // e^{i th} = a b e (th = G.R): cos th and sin th
    const double ab_c = a.x * b.x - a.y * b.y, ab_s = a.x * b.y + a.y * b.x;
    const double cs = ab_c * e.x - ab_s * e.y, sn = ab_c * e.y + ab_s * e.x;
    const double2 r = make_double2(rg[i].x * scale, rg[i].y * scale);
    // e^{-i th} conj(r) = (cs - i sn)(r.x - i r.y): imaginary part
    const double im = -cs * r.y - sn * r.x;
    for (int a = 0; a < 3; ++a) acc[a] += vs * G[a] * im;
  }
  block_sum<3>(acc, red);
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) part[((size_t)I * gridDim.x + blockIdx.x) * 3 + a] = acc[a];
}

// Nonlocal force through the force field Phi_i = sum_n w_n (D P)_in psi_n
// (Eq. force_hf, the band sum taken first):
//   dE_nl/dR_I,a = 2 sum_{i of I} sum_n w_n <d_a beta_i|n> (D P)_in
//                = 2 sum_{i of I} <d_a beta_i|Phi_i>,  d_a beta(G) = -i G_a beta(G).
// Over the stored half with the Gamma weights (1 at G = 0, else 2) the inner
// product of coefficient q is wt_q G_a(q) (Im beta Re Phi - Re beta Im Phi).
// One workgroup per projector: the three axes' sums, fixed-order tree.
__global__ void __launch_bounds__(256) k_nl_force_proj(const double2* __restrict__ B,
                                                       const double2* __restrict__ Phi,
                                                       const double* __restrict__ gcart, int npw,
                                                       double* __restrict__ part) {
  __shared__ double red[3 * 16];
  const int i = blockIdx.x;
  const double2* b = B + (size_t)i * npw;
  const double2* f = Phi + (size_t)i * npw;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < npw; q += blockDim.x) {
    const double2 bb = b[q], ff = f[q];
    const double x = (q == 0 ? 1.0 : 2.0) * (bb.y * ff.x - bb.x * ff.y);
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] = fma(gcart[(size_t)a * npw + q], x, acc[a]);
  }
  block_sum<3>(acc, red);
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) part[(size_t)i * 3 + a] = acc[a];
}

// F[I][a] = -(loc[I][a] + 2 sum_{i of atom I} part[i][a]), projectors in order
__global__ void __launch_bounds__(256) k_nl_force_sum(const double* __restrict__ part, int natoms,
                                                      const int32_t* __restrict__ off,
                                                      const int32_t* __restrict__ cnt,
                                                      const double* __restrict__ loc,
                                                      double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * natoms) return;
  const int I = t / 3, a = t - 3 * I;
  double s = 0.0;
  for (int j = 0; j < cnt[I]; ++j) s += part[(size_t)(off[I] + j) * 3 + a];
  out[t] = -(loc[t] + 2.0 * s);
}

// out[o][j] = scale * sum_i part[o][i][j]
// out[o][j] = scale sum_i part[o][i][j]: one wave per output, lanes over i,
// a fixed butterfly across the wave
__global__ void __launch_bounds__(256) k_reduce_strided(const double* __restrict__ part, int nouter,
                                                        int ninner, int ncols, double scale,
                                                        double* __restrict__ out) {
  const int t = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= nouter * ncols) return;
  const int o = t / ncols, j = t - o * ncols;
  double s = 0;
  for (int i = lane; i < ninner; i += 64) s += part[((size_t)o * ninner + i) * ncols + j];
  s = wave_sum(s);
  if (lane == 0) out[t] = scale * s;
}

int grid_blocks(size_t n, int nthr = 256) {
  size_t b = (n + nthr - 1) / nthr;
  return (int)(b > 8192 ? 8192 : (b == 0 ? 1 : b));
}

ShellArgs shell_args(const Ctx& c) {
  ShellArgs a{};
  a.nconf = c.nconf;
  a.nsocc = c.nsocc;
  a.xc = c.xc;
  for (int X = 0; X < 3; ++X)
    for (int L = 0; L < kMaxConf; ++L)
      for (int s = 0; s < 2; ++s) a.f[X][L][s] = X < c.nsocc && L < c.nconf ? c.shell_f[X][L][s] : 0.0;
  for (int L = 0; L < kMaxConf; ++L) a.cL[L] = c.cL[L];
  a.same_rho = 1;
  for (int X = 0; X < c.nsocc; ++X)
    for (int L = 1; L < c.nconf; ++L)
      if (a.f[X][L][0] + a.f[X][L][1] != a.f[X][0][0] + a.f[X][0][1]) a.same_rho = 0;
  return a;
}

// ---------------------------------------------------------------------------
// PBE (spin-polarised GGA; Perdew, Burke and Ernzerhof 1996): the energy
// density e(rho_up, rho_dn, sigma_uu, sigma_ud, sigma_dd) in one template over
// the scalar type, evaluated on forward-mode dual numbers carrying the five
// partial derivatives for the potentials (plain doubles for energies only).
// Exchange by spin scaling, e_x = sum_s n_s eps_x^unif(n_s) F_x(s_s) / 2 with
// n_s = 2 rho_s, F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa),
// s^2 = |grad n_s|^2 / (4 k_F^2 n_s^2); correlation rho (eps_c^PW92 + H),
// H = gamma phi^3 ln(1 + beta/gamma t^2 (1 + A t^2) / (1 + A t^2 + A^2 t^4)),
// A = beta/gamma / (exp(-eps_c / (gamma phi^3)) - 1), t^2 = |grad rho|^2 /
// (4 phi^2 k_s^2 rho^2), k_s^2 = 4 k_F / pi.
// ---------------------------------------------------------------------------
struct D5 {
  double v;
  double d[5];
};
__device__ __forceinline__ D5 d5c(double v) {
  D5 r;
  r.v = v;
#pragma unroll
  for (int k = 0; k < 5; ++k) r.d[k] = 0.0;
  return r;
}
__device__ __forceinline__ D5 d5var(double v, int k) {
  D5 r = d5c(v);
  r.d[k] = 1.0;
  return r;
}
// x -> (f(x), f'(x)) applied to a dual
__device__ __forceinline__ D5 d5chain(const D5& x, double f, double fp) {
  D5 r;
  r.v = f;
#pragma unroll
  for (int k = 0; k < 5; ++k) r.d[k] = fp * x.d[k];
  return r;
}
__device__ __forceinline__ D5 operator+(const D5& a, const D5& b) {
  D5 r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < 5; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
__device__ __forceinline__ D5 operator-(const D5& a, const D5& b) {
  D5 r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < 5; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
__device__ __forceinline__ D5 operator*(const D5& a, const D5& b) {
  D5 r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < 5; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
__device__ __forceinline__ D5 operator/(const D5& a, const D5& b) {
  const double ib = 1.0 / b.v;
  D5 r;
  r.v = a.v * ib;
#pragma unroll
  for (int k = 0; k < 5; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
__device__ __forceinline__ D5 operator*(double a, const D5& b) {
  D5 r;
  r.v = a * b.v;
#pragma unroll
  for (int k = 0; k < 5; ++k) r.d[k] = a * b.d[k];
  return r;
}
__device__ __forceinline__ D5 operator+(const D5& a, double b) { return a + d5c(b); }
__device__ __forceinline__ D5 operator+(double a, const D5& b) { return d5c(a) + b; }
__device__ __forceinline__ D5 operator-(const D5& a, double b) { return a - d5c(b); }
__device__ __forceinline__ D5 operator-(double a, const D5& b) { return d5c(a) - b; }
__device__ __forceinline__ D5 operator*(const D5& a, double b) { return b * a; }
__device__ __forceinline__ D5 operator/(const D5& a, double b) { return (1.0 / b) * a; }
__device__ __forceinline__ D5 operator/(double a, const D5& b) { return d5c(a) / b; }
__device__ __forceinline__ D5 operator-(const D5& a) { return -1.0 * a; }
__device__ __forceinline__ D5 gpow(const D5& x, double p) {
  const double v = pow(x.v, p);
  return d5chain(x, v, p * v / x.v);
}
__device__ __forceinline__ D5 gsqrt(const D5& x) {
  const double v = sqrt(x.v);
  return d5chain(x, v, 0.5 / v);
}
__device__ __forceinline__ D5 glog(const D5& x) { return d5chain(x, log(x.v), 1.0 / x.v); }
__device__ __forceinline__ D5 gexp(const D5& x) {
  const double v = exp(x.v);
  return d5chain(x, v, v);
}
__device__ __forceinline__ double gpow(double x, double p) { return pow(x, p); }
__device__ __forceinline__ double gsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ double glog(double x) { return log(x); }
__device__ __forceinline__ double gexp(double x) { return exp(x); }

constexpr double kPbeKappa = 0.804, kPbeBeta = 0.06672455060314922;
constexpr double kPi = 3.141592653589793;

template <typename T>
__device__ T pw92_g_t(const T& rs, const T& srs, double A, double a1, double b1, double b2, double b3,
                      double b4) {
  const T Q = 2.0 * A * (b1 * srs + b2 * rs + b3 * (rs * srs) + b4 * (rs * rs));
  return -2.0 * A * (1.0 + a1 * rs) * glog(1.0 + 1.0 / Q);
}

template <typename T>
__device__ T pbe_ex_spin(const T& r, const T& sig) {
  const double mu = kPbeBeta * kPi * kPi / 3.0;
  const T n = 2.0 * r;
  const T kf = gpow(3.0 * kPi * kPi * n, 1.0 / 3.0);
  const T s2 = sig / (kf * kf * (n * n));  // 4 sigma / (4 k_F^2 n^2)
  const T Fx = (1.0 + kPbeKappa) - kPbeKappa / (1.0 + (mu / kPbeKappa) * s2);
  const T exu = -0.75 * gpow(3.0 / kPi, 1.0 / 3.0) * gpow(n, 1.0 / 3.0);
  return 0.5 * n * exu * Fx;
}

template <typename T>
__device__ T pbe_energy(const T& ru, const T& rd, const T& suu, const T& sud, const T& sdd, double xs) {
  const double gam = (1.0 - 0.6931471805599453) / (kPi * kPi);
  const T rho = ru + rd;
  const T z = (ru - rd) / rho;
  const T rs = gpow(3.0 / (4.0 * kPi) / rho, 1.0 / 3.0);
  const T srs = gsqrt(rs);
  const T ec0 = pw92_g_t(rs, srs, 0.031091, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294);
  const T ec1 = pw92_g_t(rs, srs, 0.015545, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517);
  const T ac = -pw92_g_t(rs, srs, 0.016887, 0.11125, 10.357, 3.6231, 0.88026, 0.49671);
  const double fz20 = 1.709921, fzden = 0.5198420997897464;
  const T opz = 1.0 + z, omz = 1.0 - z;
  const T f = (gpow(opz, 4.0 / 3.0) + gpow(omz, 4.0 / 3.0) - 2.0) / fzden;
  const T z2 = z * z;
  const T z4 = z2 * z2;
  const T eps = ec0 + ac * f / fz20 * (1.0 - z4) + (ec1 - ec0) * f * z4;
  const T phi = 0.5 * (gpow(opz, 2.0 / 3.0) + gpow(omz, 2.0 / 3.0));
  const T kf = gpow(3.0 * kPi * kPi * rho, 1.0 / 3.0);
  const T ks2 = (4.0 / kPi) * kf;
  const T g2 = suu + 2.0 * sud + sdd;
  const T t2 = g2 / (4.0 * (phi * phi) * ks2 * (rho * rho));
  const T phi3 = phi * phi * phi;
  const T A = (kPbeBeta / gam) / (gexp(-eps / (gam * phi3)) - 1.0);
  const T At2 = A * t2;
  const T H = gam * phi3 * glog(1.0 + (kPbeBeta / gam) * t2 * (1.0 + At2) / (1.0 + At2 + At2 * At2));
  return xs * (pbe_ex_spin(ru, suu) + pbe_ex_spin(rd, sdd)) + rho * (eps + H);
}

// configuration L's spin densities (clamped at 0) packed as rho_up + i rho_dn
__global__ void k_gga_pack(ShellArgs a, const double* __restrict__ rho, int L, size_t ntot,
                           double2* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    double ru = 0, rd = 0;
    for (int X = 0; X < a.nsocc; ++X) {
      const double v = rho[(size_t)X * ntot + i];
      ru += a.f[X][L][0] * v;
      rd += a.f[X][L][1] * v;
    }
    out[i] = make_double2(fmax(ru, 0.0), fmax(rd, 0.0));
  }
}

// out_a = i G_a S scale for a = 0, 1, 2 (zero on Nyquist planes): the spectra
// of the three Cartesian derivatives of the two real fields packed in S
__global__ void k_gga_grad(Lattice Lt, const double2* __restrict__ S, size_t ntot, double scale,
                           double2* __restrict__ o0, double2* __restrict__ o1,
                           double2* __restrict__ o2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    int m[3];
    const bool nyq = grid_freq(Lt, i, m);
    double G[3];
    gvec(Lt, m, G);
    const double2 v = S[i];
    double g = nyq ? 0.0 : G[0] * scale;
    o0[i] = make_double2(-g * v.y, g * v.x);
    g = nyq ? 0.0 : G[1] * scale;
    o1[i] = make_double2(-g * v.y, g * v.x);
    g = nyq ? 0.0 : G[2] * scale;
    o2[i] = make_double2(-g * v.y, g * v.x);
  }
}

// out = sum_a i G_a H_a scale (zero on Nyquist planes): the spectrum of the
// divergence of the two real vector fields packed in H_0..2
__global__ void k_gga_div(Lattice Lt, const double2* __restrict__ H0, const double2* __restrict__ H1,
                          const double2* __restrict__ H2, size_t ntot, double scale,
                          double2* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    int m[3];
    const bool nyq = grid_freq(Lt, i, m);
    double G[3];
    gvec(Lt, m, G);
    double re = 0.0, im = 0.0;
    if (!nyq) {
      const double2 h0 = H0[i], h1 = H1[i], h2 = H2[i];
      re = -(G[0] * h0.y + G[1] * h1.y + G[2] * h2.y);
      im = G[0] * h0.x + G[1] * h1.x + G[2] * h2.x;
    }
    out[i] = make_double2(re * scale, im * scale);
  }
}

// per point of configuration L: the PBE energy density (exchange scaled by
// xs: 1 - a for a hybrid) into e; with WRITE the
// density derivatives into vu / vd and the gradient terms
// h_s = 2 de/dsigma_ss grad rho_s + de/dsigma_ud grad rho_s' over the
// gradients g_a (packed up + i down, overwritten by h_up + i h_dn)
template <bool WRITE>
__global__ void __launch_bounds__(256) k_gga_point(ShellArgs a, const double* __restrict__ rho, int L,
                                                   size_t ntot, double2* __restrict__ g0,
                                                   double2* __restrict__ g1, double2* __restrict__ g2,
                                                   double* __restrict__ e, double* __restrict__ vu,
                                                   double* __restrict__ vd, double xs) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    double ru = 0, rd = 0;
    for (int X = 0; X < a.nsocc; ++X) {
      const double v = rho[(size_t)X * ntot + i];
      ru += a.f[X][L][0] * v;
      rd += a.f[X][L][1] * v;
    }
    ru = fmax(ru, 0.0);
    rd = fmax(rd, 0.0);
    const double2 x0 = g0[i], x1 = g1[i], x2 = g2[i];
    const double suu = x0.x * x0.x + x1.x * x1.x + x2.x * x2.x;
    const double sud = x0.x * x0.y + x1.x * x1.y + x2.x * x2.y;
    const double sdd = x0.y * x0.y + x1.y * x1.y + x2.y * x2.y;
    const bool live = ru + rd >= 1e-12;
    ru = fmax(ru, 1e-30);
    rd = fmax(rd, 1e-30);
    if (!WRITE) {
      e[i] = live ? pbe_energy<double>(ru, rd, suu, sud, sdd, xs) : 0.0;
      continue;
    }
    double ev = 0.0, fu = 0.0, fd = 0.0, fuu = 0.0, fud = 0.0, fdd = 0.0;
    if (live) {
      const D5 r =
          pbe_energy<D5>(d5var(ru, 0), d5var(rd, 1), d5var(suu, 2), d5var(sud, 3), d5var(sdd, 4), xs);
      ev = r.v;
      fu = r.d[0];
      fd = r.d[1];
      fuu = r.d[2];
      fud = r.d[3];
      fdd = r.d[4];
    }
    e[i] = ev;
    vu[i] = fu;
    vd[i] = fd;
    g0[i] = make_double2(2.0 * fuu * x0.x + fud * x0.y, 2.0 * fdd * x0.y + fud * x0.x);
    g1[i] = make_double2(2.0 * fuu * x1.x + fud * x1.y, 2.0 * fdd * x1.y + fud * x1.x);
    g2[i] = make_double2(2.0 * fuu * x2.x + fud * x2.y, 2.0 * fdd * x2.y + fud * x2.x);
  }
}

// vu -= Re div, vd -= Im div
__global__ void k_gga_sub(const double2* __restrict__ div, size_t ntot, double* __restrict__ vu,
                          double* __restrict__ vd) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 d = div[i];
    vu[i] -= d.x;
    vd[i] -= d.y;
  }
}

// the GGA counterpart of k_xc's assembly: v_xc^{sigma L} already in vloc
// (WRITE) becomes V_loc = V_ext + V_H^L + v_xc, then the shell potentials;
// partial sums of e_xc (from e), V_ext rho and V_H rho per configuration
template <bool WRITE>
__global__ void __launch_bounds__(256) k_gga_assemble(ShellArgs a, const double* __restrict__ rho,
                                                      const double* __restrict__ vext,
                                                      const double2* __restrict__ vh,
                                                      const double* __restrict__ e, size_t ntot,
                                                      double* __restrict__ vloc, double* __restrict__ vsh,
                                                      double* __restrict__ part) {
  __shared__ double red[8 * 16];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < ntot;
       i += (size_t)gridDim.x * blockDim.x) {
    double rX[3] = {0, 0, 0};
    for (int X = 0; X < a.nsocc; ++X) rX[X] = rho[(size_t)X * ntot + i];
    const double ve = vext[i];
    const double2 vhp = WRITE ? vh[i] : make_double2(0.0, 0.0);
    double vl[kMaxConf][2];
    for (int L = 0; L < a.nconf; ++L) {
      double ru = 0, rd = 0;
      for (int X = 0; X < a.nsocc; ++X) {
        ru += a.f[X][L][0] * rX[X];
        rd += a.f[X][L][1] * rX[X];
      }
      ru = fmax(ru, 0.0);
      rd = fmax(rd, 0.0);
      acc[3 * L + 0] += e[(size_t)L * ntot + i];
      acc[3 * L + 1] += ve * (ru + rd);
      if (!WRITE) continue;
      const double h = L == 0 ? vhp.x : vhp.y;
      vl[L][0] = ve + h + vloc[(size_t)(2 * L) * ntot + i];
      vl[L][1] = ve + h + vloc[(size_t)(2 * L + 1) * ntot + i];
      vloc[(size_t)(2 * L) * ntot + i] = vl[L][0];
      vloc[(size_t)(2 * L + 1) * ntot + i] = vl[L][1];
      acc[3 * L + 2] += h * (ru + rd);
    }
    if (!WRITE) continue;
    for (int X = 0; X < a.nsocc; ++X) {
      double s = 0;
      for (int L = 0; L < a.nconf; ++L)
        s += a.cL[L] * (a.f[X][L][0] * vl[L][0] + a.f[X][L][1] * vl[L][1]);
      vsh[(size_t)X * ntot + i] = s;
    }
  }
  block_sum<6>(acc, red);
  if (threadIdx.x == 0)
    for (int j = 0; j < 6; ++j) part[(size_t)blockIdx.x * 6 + j] = acc[j];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static AtomP* atoms_dev(Ctx& c) {
  static_assert(sizeof(AtomP) == 5 * sizeof(double), "AtomP layout");
  return reinterpret_cast<AtomP*>(c.d_atoms);
}

size_t atom_info_bytes() { return sizeof(AtomP); }
size_t proj_info_bytes() { return sizeof(ProjP); }

void upload_positions(Ctx& c) {
  std::vector<AtomP> h(c.natoms);
  for (int a = 0; a < c.natoms; ++a) {
    const Ctx::Species& sp = c.species[c.spec_of[a]];
    h[a] = AtomP{c.pos[3 * a], c.pos[3 * a + 1], c.pos[3 * a + 2], sp.A, sp.sigma};
  }
  if (c.natoms > 0)
    ROKS_HIP(hipMemcpyAsync(atoms_dev(c), h.data(), h.size() * sizeof(AtomP), hipMemcpyHostToDevice,
                            c.stream));
  // projector descriptors live right after the atoms
  std::vector<ProjP> pp(c.nproj);
  for (int i = 0; i < c.nproj; ++i) pp[i] = ProjP{c.proj_atom[i], c.proj_l[i], c.proj_m[i], c.proj_rp[i]};
  if (c.nproj > 0)
    ROKS_HIP(hipMemcpyAsync(c.d_projinfo, pp.data(),
                            pp.size() * sizeof(ProjP), hipMemcpyHostToDevice, c.stream));
  ROKS_HIP(hipStreamSynchronize(c.stream));  // the host vectors go out of scope
  launch_vext(c);
  if (c.nproj > 0) launch_projectors(c, c.d_B, -1);
  c.bsplit_valid = false;  // the BF16x3 split of the table is stale
  c.potentials_valid = false;
}

void launch_vext(Ctx& c) {
  const size_t n = c.ntot;
  hipLaunchKernelGGL(k_vext_G, dim3(grid_blocks(n)), dim3(256), 0, c.stream, lattice(c), atoms_dev(c),
                     c.natoms, c.d_fft, n);
  ROKS_HIP(hipGetLastError());
  launch_fft3d(c, c.d_fft, +1);
  hipLaunchKernelGGL(k_take_real, dim3(grid_blocks(n)), dim3(256), 0, c.stream, c.d_fft, c.d_vext, n);
  ROKS_HIP(hipGetLastError());
}

void launch_projectors(Ctx& c, double2* B, int axis) {
  const size_t n = (size_t)c.nproj * c.npw;
  if (n == 0) return;
  const ProjP* pp = reinterpret_cast<const ProjP*>(c.d_projinfo);
  hipLaunchKernelGGL(k_projectors, dim3(grid_blocks(n)), dim3(256), 0, c.stream, lattice(c), c.d_miller,
                     c.npw, pp, c.nproj, atoms_dev(c), axis, B);
  ROKS_HIP(hipGetLastError());
}

void launch_gcart(Ctx& c, double* gcart) {
  const size_t n = c.npw;
  hipLaunchKernelGGL(k_gcart, dim3(grid_blocks(n)), dim3(256), 0, c.stream, lattice(c), c.d_miller,
                     c.npw, gcart);
  ROKS_HIP(hipGetLastError());
}

void launch_density_reduce(Ctx& c, const double* rho_part, int nchunk, double* rho) {
  const size_t n = c.ntot;
  hipLaunchKernelGGL(k_density_reduce, dim3(grid_blocks(n)), dim3(256), 0, c.stream, shell_args(c),
                     rho_part, nchunk, n, 1.0 / c.omega, rho, c.d_fft);
  ROKS_HIP(hipGetLastError());
}

// d_fft holds the packed configuration densities (launch_density_reduce)
void launch_hartree(Ctx& c) {
  // forward transform, 4 pi / (G^2 N^3), inverse transform (the multiply
  // rides on the z pass); the xc pass reads V_H^0 + i V_H^1 from d_fft as the
  // transform leaves it
  launch_hartree_fft(c, c.d_fft);
}

int xc_blocks(const Ctx& c) {
  int b = grid_blocks(c.ntot);
  return b < kRedBlocks ? b : kRedBlocks;
}

void launch_xc_potentials(Ctx& c, double* part, int nblocks) {
  // reads shell densities, V_ext, V_H; writes V_loc and the shell potentials
  KernelTimer kt(c, "xc", (double)(2 * c.nsocc + 1 + 3 * c.nconf) * c.ntot * sizeof(double));
  hipLaunchKernelGGL(k_xc<true>, dim3(nblocks), dim3(256), 0, c.stream, shell_args(c), c.d_rho,
                     c.d_vext, c.d_fft, (size_t)c.ntot, c.d_vloc, c.d_vsh, part);
  ROKS_HIP(hipGetLastError());
}

void launch_xc_energy(Ctx& c, double* part, int nblocks) {
  hipLaunchKernelGGL(k_xc<false>, dim3(nblocks), dim3(256), 0, c.stream, shell_args(c), c.d_rho,
                     c.d_vext, c.d_fft, (size_t)c.ntot, c.d_vloc, c.d_vsh, part);
  ROKS_HIP(hipGetLastError());
}

// d_fft holds the packed configuration densities (launch_density_reduce)
void launch_hartree_energy(Ctx& c, double* part, int nblocks) {
  const size_t n = c.ntot;
  launch_fft3d(c, c.d_fft, -1);
  hipLaunchKernelGGL(k_hartree_energy, dim3(nblocks), dim3(256), 0, c.stream, lattice(c), c.d_fft, n,
                     c.nconf, part);
  ROKS_HIP(hipGetLastError());
}

void launch_reduce_columns(Ctx& c, const double* part, int nrows, int ncols, double* out,
                           double* mirror, const double* part2, int ncols2) {
  hipLaunchKernelGGL(k_reduce_columns, dim3(ncols + (part2 ? ncols2 : 0)), dim3(256), 0, c.stream, part,
                     nrows, ncols, out, mirror, part2);
  ROKS_HIP(hipGetLastError());
}

void launch_to_float(Ctx& c, const double* in, float* out, size_t n) {
  hipLaunchKernelGGL(k_to_float, dim3(grid_blocks(n)), dim3(256), 0, c.stream, in, out, n);
  ROKS_HIP(hipGetLastError());
}

void launch_reduce_strided(Ctx& c, const double* part, int nouter, int ninner, int ncols,
                           double scale, double* out) {
  const int n = nouter * ncols;
  hipLaunchKernelGGL(k_reduce_strided, dim3(cdiv(n, 4)), dim3(256), 0, c.stream, part, nouter, ninner,
                     ncols, scale, out);
  ROKS_HIP(hipGetLastError());
}

void launch_nl_energy(Ctx& c, const double* P, double* out, double* mirror) {
  hipLaunchKernelGGL(k_nl_energy, dim3(c.nb), dim3(64), 0, c.stream, P, c.nb, c.natoms,
                     c.d_atom_proj_off, c.d_atom_proj_cnt, c.d_Dblk_off, c.d_Dblk, out, mirror);
  ROKS_HIP(hipGetLastError());
}

void launch_apply_D(Ctx& c, const double* P, const double* w, double* DP) {
  const size_t n = (size_t)c.nproj * c.nb;
  if (n == 0) return;
  hipLaunchKernelGGL(k_apply_D, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, P, c.nb,
                     c.nproj, c.d_proj_atom, c.d_atom_proj_off, c.d_atom_proj_cnt, c.d_Dblk_off,
                     c.d_Dblk, w, DP);
  ROKS_HIP(hipGetLastError());
}

void launch_apply_Q(Ctx& c, const double* P, double* QP) {
  const size_t n = (size_t)c.nproj * c.nb;
  if (n == 0) return;
  hipLaunchKernelGGL(k_apply_D, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, P, c.nb,
                     c.nproj, c.d_proj_atom, c.d_atom_proj_off, c.d_atom_proj_cnt, c.d_Dblk_off,
                     c.d_Qblk, nullptr, QP);
  ROKS_HIP(hipGetLastError());
}

// the multipliers of Eq. gamma_def restricted to the occupied bands
__global__ void k_overlap_multipliers(const double* __restrict__ theta, int nb,
                                      const int32_t* __restrict__ band_shell, int nsocc,
                                      double* __restrict__ G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * nb) return;
  const int m = t / nb, n = t - m * nb;
  const bool occ = band_shell[m] < nsocc && band_shell[n] < nsocc;
  G[t] = occ ? 0.5 * (theta[t] + theta[n * nb + m]) : 0.0;
}

void launch_overlap_multipliers(Ctx& c, const double* theta, double* G) {
  hipLaunchKernelGGL(k_overlap_multipliers, dim3(cdiv(c.nb * c.nb, 256)), dim3(256), 0, c.stream,
                     theta, c.nb, c.d_band_shell, c.nsocc, G);
  ROKS_HIP(hipGetLastError());
}

void launch_pack_rho_weighted(Ctx& c) {
  const size_t n = c.ntot;
  hipLaunchKernelGGL(k_pack_rho, dim3(grid_blocks(n)), dim3(256), 0, c.stream, shell_args(c), c.d_rho, n,
                     c.d_fft, 1);
  ROKS_HIP(hipGetLastError());
}

void launch_local_force(Ctx& c, const double2* rhoG, double* out_part, int nblk) {
  if (c.natoms == 0) return;
  ROKS_CHECK(c.N[0] <= kMaxAxis && c.N[1] <= kMaxAxis && c.N[2] <= kMaxAxis, ROKS_ERR_SHAPE,
             "grid axis longer than the force kernel's phase tables");
  // is the reciprocal basis orthogonal (the Gaussian then factorises)?
  int orth = 1;
  for (int i = 0; i < 3; ++i)
    for (int j = i + 1; j < 3; ++j) {
      double dij = 0, ni = 0, nj = 0;
      for (int a = 0; a < 3; ++a) {
        dij += c.recip[i][a] * c.recip[j][a];
        ni += c.recip[i][a] * c.recip[i][a];
        nj += c.recip[j][a] * c.recip[j][a];
      }
      if (std::fabs(dij) > 1e-14 * std::sqrt(ni * nj)) orth = 0;
    }
  hipLaunchKernelGGL(k_local_force, dim3(nblk, c.natoms), dim3(256), 0, c.stream, lattice(c),
                     atoms_dev(c), rhoG, (size_t)c.ntot, 1.0 / (double)c.ntot, orth, out_part);
  ROKS_HIP(hipGetLastError());
}

void launch_nl_force(Ctx& c, const double* phi, double* part, const double* loc, double* out) {
  if (c.natoms == 0) return;
  if (c.nproj > 0) {
    hipLaunchKernelGGL(k_nl_force_proj, dim3(c.nproj), dim3(256), 0, c.stream, c.d_B,
                       reinterpret_cast<const double2*>(phi), c.d_gcart, c.npw, part);
    ROKS_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_nl_force_sum, dim3(cdiv(3 * c.natoms, 256)), dim3(256), 0, c.stream, part,
                     c.natoms, c.d_atom_proj_off, c.d_atom_proj_cnt, loc, out);
  ROKS_HIP(hipGetLastError());
}

// PBE potentials (write) or energies: per configuration the spin densities'
// spectral gradients, the pointwise functional, and (write) the divergence
// of its gradient terms; then the assembly of V_loc, the shell potentials and
// the energy sums (the layout of the LDA pass)
void launch_gga(Ctx& c, double* part, int nblocks, bool write) {
  const size_t n = c.ntot;
  if (!c.d_gga) {
    c.d_gga = dalloc<double2>(c, 4 * n);
    c.d_gga_e = dalloc<double>(c, (size_t)c.nconf * n);
  }
  KernelTimer kt(c, "xc", (double)(2 * c.nsocc + 1 + 3 * c.nconf) * n * sizeof(double) +
                              (double)c.nconf * (write ? 16.0 : 8.0) * n * sizeof(double2));
  const ShellArgs a = shell_args(c);
  const Lattice Lt = lattice(c);
  const unsigned gb = (unsigned)grid_blocks(n);
  double2* S = c.d_gga;
  double2* g[3] = {c.d_gga + n, c.d_gga + 2 * n, c.d_gga + 3 * n};
  const double scale = 1.0 / (double)n;
  for (int L = 0; L < c.nconf; ++L) {
    double* vu = c.d_vloc + (size_t)(2 * L) * n;
    double* vd = c.d_vloc + (size_t)(2 * L + 1) * n;
    hipLaunchKernelGGL(k_gga_pack, dim3(gb), dim3(256), 0, c.stream, a, c.d_rho, L, n, S);
    ROKS_HIP(hipGetLastError());
    launch_fft3d(c, S, -1);
    hipLaunchKernelGGL(k_gga_grad, dim3(gb), dim3(256), 0, c.stream, Lt, S, n, scale, g[0], g[1], g[2]);
    ROKS_HIP(hipGetLastError());
    for (int k = 0; k < 3; ++k) launch_fft3d(c, g[k], +1);
    if (write)
      hipLaunchKernelGGL(k_gga_point<true>, dim3(gb), dim3(256), 0, c.stream, a, c.d_rho, L, n, g[0], g[1],
                         g[2], c.d_gga_e + (size_t)L * n, vu, vd, 1.0 - c.exx);
    else
      hipLaunchKernelGGL(k_gga_point<false>, dim3(gb), dim3(256), 0, c.stream, a, c.d_rho, L, n, g[0],
                         g[1], g[2], c.d_gga_e + (size_t)L * n, vu, vd, 1.0 - c.exx);
    ROKS_HIP(hipGetLastError());
    if (!write) continue;
    for (int k = 0; k < 3; ++k) launch_fft3d(c, g[k], -1);
    hipLaunchKernelGGL(k_gga_div, dim3(gb), dim3(256), 0, c.stream, Lt, g[0], g[1], g[2], n, scale, S);
    ROKS_HIP(hipGetLastError());
    launch_fft3d(c, S, +1);
    hipLaunchKernelGGL(k_gga_sub, dim3(gb), dim3(256), 0, c.stream, S, n, vu, vd);
    ROKS_HIP(hipGetLastError());
  }
  if (write)
    hipLaunchKernelGGL(k_gga_assemble<true>, dim3(nblocks), dim3(256), 0, c.stream, a, c.d_rho, c.d_vext,
                       c.d_fft, c.d_gga_e, n, c.d_vloc, c.d_vsh, part);
  else
    hipLaunchKernelGGL(k_gga_assemble<false>, dim3(nblocks), dim3(256), 0, c.stream, a, c.d_rho, c.d_vext,
                       c.d_fft, c.d_gga_e, n, c.d_vloc, c.d_vsh, part);
  ROKS_HIP(hipGetLastError());
}

}  // namespace roks
