// The ROKS hot path on the device, orchestrated from the host:
// densities -> potentials -> energies, shell-operator application, subspace
// matrices, the projected Teter preconditioner, Fletcher-Reeves directions,
// the line search over Cholesky-orthonormalised and rotated trial orbitals,
// and the Hellmann-Feynman forces.  Scalars that steer control flow (energies,
// directional derivatives) are written by the kernels into pinned host memory;
// everything else stays on the GPU.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "roks_internal.h"

namespace roks {

namespace {


// U = exp(X) for X = delta * D (antisymmetric): scaling and squaring around a
// Taylor polynomial evaluated by the Paterson-Stockmeyer scheme, the degree m
// and squarings s with theta^(m+1)/(m+1)! <= 1e-17 (theta = ||X||_1 / 2^s <=
// 1, the single-workgroup kernel's criterion) and the fewest products
void expm(Ctx& c, double delta, const double* D, double* U) {
  if (expm_in_lds(c)) {
    launch_expm_lds(c, D, delta, U, c.stream);
    return;
  }
  const int n = c.nb;
  const size_t nn = (size_t)n * n;
  // scratch of its own (it runs beside the trial's factorisation)
  double* X = c.d_ex;
  double* w[4] = {c.d_ex + nn, c.d_ex + 2 * nn, c.d_ex + 3 * nn, c.d_ex + 4 * nn};
  axpby(c, nn, delta, D, 0.0, nullptr, X);
  // ||delta D||_1 = |delta| ||D||_1: the norm of the search's D was queued by
  // prepare_line_search into the pinned mirror and is read after the
  // synchronisation that follows it (one more only if D changed since)
  if (c.normD_pending) {
    sync(c);
    c.normD_pending = false;
  }
  const double nrm = std::fabs(delta) * c.h_stage[kStageNormD];
  ROKS_CHECK(std::isfinite(nrm), ROKS_ERR_NAN, "non-finite rotation generator");
  int s = 0, m = 30, best = 1 << 30;
  for (int sq = 0; sq <= 60; ++sq) {
    const double th = std::ldexp(nrm, -sq);
    if (th > 1.0) continue;
    double term = th;
    int mm = 0;
    while (term > 1e-17 && mm < 30) {
      ++mm;
      term *= th / (mm + 1);
    }
    if (taylor_products(mm) + sq < best) {
      best = taylor_products(mm) + sq;
      s = sq;
      m = mm;
    }
    if (mm <= 1) break;
  }
  if (s > 0) axpby(c, nn, std::ldexp(1.0, -s), X, 0.0, nullptr, X);
  double* cur = taylor_ps(c, n, m, X, w[0], w[1], w[2], w[3]);
  double* nxt = cur == w[2] ? w[3] : w[2];
  for (int i = 0; i < s; ++i) {
    gemm_small(c, n, n, n, cur, n, false, cur, n, false, nxt, n, 1.0, 0.0);
    std::swap(cur, nxt);
  }
  copy_dev(c, U, cur, nn * sizeof(double));
}

}  // namespace

void compute_potentials_async(Ctx& c, const double2* orb, bool have_P, bool energy_only);
roks_energies assemble_energies(const Ctx& c, bool energy_only);

namespace {

struct Trial {
  double2* psi;
  double* M;
  double* U;
  double E;
  roks_energies e;
  bool ok;
};

// Once per line search (the search direction is fixed): <S|S> and <beta|S>;
// on the step's first search also <beta|psi> of the current orbitals (left
// in d_P by their energy evaluation; trials overwrite d_P afterwards).
void prepare_line_search(Ctx& c, bool first) {
  const int nb = c.nb, K = 2 * c.npw;
  gemm_wdot(c, nb, nb, K, dbl(c.d_S), K, dbl(c.d_S), K, c.d_SS, nb, 1.0, 0.0, true);
  if (!expm_in_lds(c)) {
    // ||D||_1 for the exponentials of the trials, straight into the mirror
    matrix_norm1(c, c.d_D, nb, c.hd_stage + kStageNormD);
    c.normD_pending = true;
  }
  if (c.nproj > 0) {
    // P0 <- the current projections by trading buffers: the trials write d_P,
    // so P (with the densities and potentials, which the trials overwrite too)
    // counts as stale until a step keeps its last trial
    if (first) {
      std::swap(c.d_P0, c.d_P);
      c.potentials_valid = false;
    }
    proj_wdot(c, nb, dbl(c.d_S), K, c.d_PS, nb);
    if (c.has_q) {
      // <S|S|S> = <S|S> + PS^T q PS: the trial Gram matrix in the S metric
      launch_apply_Q(c, c.d_PS, c.d_DP);
      gemm_small(c, nb, nb, c.nproj, c.d_PS, nb, true, c.d_DP, nb, false, c.d_SS, nb, 1.0, 1.0);
    }
  }
}

// Psi(delta) = U^T L^-1 (Psi + delta S), U = exp(delta D); its energy.
// The orbitals are orthonormal and S is orthogonal to them (both in the
// metric of the overlap operator when it is not 1), so the Gram matrix of
// Psi + delta S is I + delta^2 <S|S>, and the trial's projections
// are <beta|Psi + delta S> = P0 + delta PS rotated by M.  One
// synchronisation: the Cholesky status and the energy sums come back together
// (a failed factorisation only makes the rest of the evaluation meaningless).
void evaluate_trial(Ctx& c, double delta, Trial& t, bool energy_only) {
  const int nb = c.nb, K = 2 * c.npw;
  if (expm_in_lds(c)) {
    // factorisation of I + delta^2 <S|S> (formed while loading) and the
    // exponential side by side: one launch, two workgroups
    launch_chol_expm_lds(c, c.d_SS, delta * delta, 1.0, c.d_Linv, c.hd_flag, c.d_D, delta, t.U);
  } else {
    // the rotation on the side stream beside the factorisation (the two are
    // independent short-kernel chains; the exponential has its own scratch)
    if (c.normD_pending) {
      sync(c);
      c.normD_pending = false;
    }
    ensure_side_stream(c);
    ROKS_HIP(hipEventRecord(c.ev_fork, c.stream));
    ROKS_HIP(hipStreamWaitEvent(c.side, c.ev_fork, 0));
    // the split-K partials of the products on the two streams go to the two
    // halves of their buffer (restored on every exit)
    struct Halves {
      Ctx& c;
      double* part;
      size_t cap;
      hipStream_t main;
      ~Halves() {
        c.d_gemm_part = part;
        c.gemm_part_capacity = cap;
        c.stream = main;
      }
    } halves{c, c.d_gemm_part, c.gemm_part_capacity, c.stream};
    const size_t half = c.gemm_part_capacity / 2;
    c.gemm_part_capacity = half;
    c.d_gemm_part = halves.part + half;
    c.stream = c.side;
    expm(c, delta, c.d_D, t.U);
    c.stream = halves.main;
    c.d_gemm_part = halves.part;
    ROKS_HIP(hipEventRecord(c.ev_join, c.side));
    scale_shift(c, c.d_SS, nb, delta * delta, 1.0, c.d_gram);
    cholesky_inverse(c, c.d_gram, nb, c.d_Linv, c.hd_flag);
    ROKS_HIP(hipStreamWaitEvent(c.stream, c.ev_join, 0));
  }
  gemm_small(c, nb, nb, nb, t.U, nb, true, c.d_Linv, nb, false, t.M, nb, 1.0, 0.0);
  // trial orbitals M^T (psi + delta S), the sum formed while loading
  gemm_expand_sum(c, nb, K, nb, t.M, nb, true, dbl(c.d_psi), dbl(c.d_S), delta, K, dbl(t.psi), K,
                  dbl(t.psi), K, 1.0, 0.0);
  if (c.nproj > 0) {
    gemm_small2(c, c.nproj, nb, nb, c.d_P0, c.d_PS, delta, nb, false, t.M, nb, true, c.d_P, nb, 1.0,
                0.0, 0.0);
  }
  compute_potentials_async(c, t.psi, true, energy_only);
  sync(c);
  t.ok = c.h_flag[0] == 0;
  t.E = INFINITY;
  if (!t.ok) return;
  t.e = assemble_energies(c, energy_only);
  t.E = t.e.E;
  if (!std::isfinite(t.E)) {
    t.ok = false;
    t.E = INFINITY;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// densities, potentials and energies of `orb` (Sec. II A, H^{sigma L})
// ---------------------------------------------------------------------------
// every launch of the energy evaluation; the reduced sums also land in the
// pinned mirror h_scal, read by assemble_energies after a synchronisation
// rowW of exx_apply for the shell operators: row n takes -W[X][m], X the
// shell of band n (zero for virtual bands) or, with Xfixed >= 0, that shell
std::vector<double> exx_shell_weights(const Ctx& c, int Xfixed) {
  const int nb = c.nb;
  std::vector<double> W((size_t)nb * nb, 0.0);
  for (int n = 0; n < nb; ++n) {
    const int X = Xfixed >= 0 ? Xfixed : c.band_shell[n];
    if (X >= c.nsocc) continue;
    for (int m = 0; m < nb; ++m) {
      const int Y = c.band_shell[m];
      if (Y >= c.nsocc) continue;
      double w = 0.0;
      for (int L = 0; L < c.nconf; ++L)
        for (int sp = 0; sp < 2; ++sp) w += c.cL[L] * c.shell_f[X][L][sp] * c.shell_f[Y][L][sp];
      W[(size_t)n * nb + m] = -w;
    }
  }
  return W;
}

void compute_potentials_async(Ctx& c, const double2* orb, bool have_P, bool energy_only) {
  const int nb = c.nb, K = 2 * c.npw;
  {
    // the FP32 tier's densities in FP64 where its FP32 planes would be slower
    // (the tier is restored on every exit from this block)
    struct TierScope {
      Ctx& c;
      int prec;
      ~TierScope() { c.prec = prec; }
    } scope{c, c.prec};
    if (scope.prec == ROKS_FP32 && !fp32_density_planes(c)) c.prec = ROKS_FP64;
    launch_zpass_bwd(c, orb, nb, c.d_T, c.npairs);
    c.T_src = orb;
    c.T_prec = c.prec;
    launch_plane_density(c, c.d_T, c.npairs, c.d_rho_part, c.nchunk);
  }
  launch_density_reduce(c, c.d_rho_part, c.nchunk, c.d_rho);
  if (c.exx != 0.0) {
    // exact exchange: the real-space orbitals (kept for the applies of these
    // orbitals) and E_x^HF of every configuration
    exx_orbitals(c, orb);
    exx_energies(c);
  }
  // with the projections at hand, the band kinetic and nonlocal energies run
  // on the side stream beside the Hartree and xc chain (they need neither;
  // graph mode keeps every launch on one stream)
  const bool side = have_P && !c.in_graph;
  if (side) {
    ensure_side_stream(c);
    ROKS_HIP(hipEventRecord(c.ev_fork, c.stream));
    ROKS_HIP(hipStreamWaitEvent(c.side, c.ev_fork, 0));
    const hipStream_t main = c.stream;
    c.stream = c.side;
    band_dots2(c, orb, orb, nb, nullptr, c.d_kin, nullptr, c.hd_scal + 16);
    if (c.nproj > 0) launch_nl_energy(c, c.d_P, c.d_enl, c.hd_scal + 16 + nb);
    c.stream = main;
    ROKS_HIP(hipEventRecord(c.ev_join, c.side));
  }
  const int nblk = xc_blocks(c);
  if (energy_only) {
    // energies only: the Hartree integrals from the forward transform, the
    // xc and external sums without writing any potential
    launch_hartree_energy(c, c.d_part + 6 * (size_t)nblk, nblk);
    if (c.xc == ROKS_XC_PBE)
      launch_gga(c, c.d_part, nblk, false);
    else
      launch_xc_energy(c, c.d_part, nblk);
    launch_reduce_columns(c, c.d_part, nblk, 6, c.d_red, c.hd_scal, c.d_part + 6 * (size_t)nblk, 2);
  } else {
    launch_hartree(c);
    if (c.xc == ROKS_XC_PBE)
      launch_gga(c, c.d_part, nblk, true);
    else
      launch_xc_potentials(c, c.d_part, nblk);
    launch_reduce_columns(c, c.d_part, nblk, 6, c.d_red, c.hd_scal);
  }
  if (c.prec == ROKS_FP32 && !energy_only) {
    // the plane passes of the FP32 tier read FP32 copies of the potentials
    launch_to_float(c, c.d_vsh, c.d_vsh32, (size_t)c.nsocc * c.ntot);
    launch_to_float(c, c.d_vloc, c.d_vloc32, (size_t)2 * c.nconf * c.ntot);
  }
  // (without projectors d_enl and its mirror hold the zeros set at creation)
  if (side) {
    ROKS_HIP(hipStreamWaitEvent(c.stream, c.ev_join, 0));
    return;
  }
  band_dots2(c, orb, orb, nb, nullptr, c.d_kin, nullptr, c.hd_scal + 16);
  if (c.nproj > 0) {
    if (!have_P) proj_wdot(c, nb, dbl(orb), K, c.d_P, nb);
    launch_nl_energy(c, c.d_P, c.d_enl, c.hd_scal + 16 + nb);
  }
}

roks_energies assemble_energies(const Ctx& c, bool energy_only) {
  const int nb = c.nb;
  const double* h = c.h_scal;
  const double* kin = h + 16;
  const double* enl = h + 16 + nb;
  roks_energies out{};
  const double dv = c.omega / (double)c.ntot;
  double E = 0.0;
  for (int L = 0; L < c.nconf; ++L) {
    double k = 0.0, nl = 0.0;
    for (int n = 0; n < nb; ++n) {
      const double f = (double)c.occ[(L * 2 + 0) * nb + n] + (double)c.occ[(L * 2 + 1) * nb + n];
      k += f * kin[n];
      nl += f * enl[n];
    }
    out.kinetic[L] = k;
    out.nonlocal[L] = nl;
    out.xc[L] = dv * h[3 * L + 0] + c.exx * c.exx_E[L];
    out.external[L] = dv * h[3 * L + 1];
    out.hartree[L] = 0.5 * dv * (energy_only ? h[6 + L] : h[3 * L + 2]);
    out.E_L[L] = k + nl + out.external[L] + out.hartree[L] + out.xc[L];
    E += c.cL[L] * out.E_L[L];
  }
  out.E = E;
  return out;
}

void compute_potentials(Ctx& c, const double2* orb, roks_energies* e) {
  compute_potentials_async(c, orb, false, false);
  sync(c);
  const roks_energies out = assemble_energies(c, false);
  if (e) *e = out;
  c.potentials_valid = (orb == c.d_psi);
}

void ensure_potentials(Ctx& c) {
  ROKS_CHECK(c.have_orbitals, ROKS_ERR_STATE, "no orbitals set");
  if (!c.potentials_valid) compute_potentials(c, c.d_psi, &c.last_e);
}

// ---------------------------------------------------------------------------
// operator application: shell mode (F^{X(n)}, Eq. shell_operator) or channels
// ---------------------------------------------------------------------------
void apply_operator(Ctx& c, const double2* vecs, uint32_t mask, double2* out, bool want_Q) {
  const int nb = c.nb, K = 2 * c.npw;
  const size_t band = (size_t)nb * c.npw;
  // <beta|vecs>; for the current orbitals their energy evaluation left it in d_P
  const bool have_P = vecs == c.d_psi && c.potentials_valid;
  const double* P = have_P ? c.d_P : c.d_dP;
  if (c.nproj > 0 && !have_P)
    proj_wdot(c, nb, dbl(vecs), K, c.d_dP, nb);
  if (mask == 0) {
    // the z pass of the orbitals is still in d_T when their energy
    // evaluation was the last writer (an accepted second trial): skipped
    const bool reuse_T = !c.in_graph && vecs == c.d_psi && c.potentials_valid && c.T_src == vecs &&
                         c.T_prec == c.prec;
    if (!reuse_T) launch_zpass_bwd(c, vecs, nb, c.d_T, c.npairs, c.in_graph ? c.zskip : nullptr);
    const void* vsh = c.prec == ROKS_FP32 ? (const void*)c.d_vsh32 : (const void*)c.d_vsh;
    launch_plane_apply(c, c.d_T, c.npairs, vsh, c.nsocc, c.d_potidx, nb, c.d_Qpart,
                       want_Q ? c.nsocc : 0);
    launch_zpass_fwd(c, c.d_T, c.npairs, vecs, nb, c.d_kinw_shell, out);
    if (c.nproj > 0) {
      launch_apply_D(c, P, c.d_kinw_shell, c.d_DP);
      proj_expand(c, nb, c.d_DP, nb, dbl(out), K);
    }
    if (c.exx != 0.0) exx_apply(c, vecs, nb, exx_shell_weights(c, -1).data(), out, want_Q ? c.d_exx_I : nullptr);
    if (want_Q) {
      // Q[n][X] = N^-3 sum_z Qpart[pair][z][b][X], n = 2 pair + b; d_Q holds
      // 2 npairs rows so an odd band count needs no special case
      launch_reduce_strided(c, c.d_Qpart, c.npairs, c.N[2], 2 * c.nsocc, 1.0 / (double)c.ntot,
                            c.d_Q);
      if (c.exx != 0.0) exx_shell_expectations(c);  // + a <n|K^X|n>
    }
    return;
  }
  int idx = 0;
  for (int b = 0; b < 2 * c.nconf; ++b) {
    if (!(mask & (1u << b))) continue;
    double2* o = out + (size_t)idx * band;
    launch_zpass_bwd(c, vecs, nb, c.d_T, c.npairs);
    // one potential grid (channel b); row 1 of d_potidx is all zeros
    const void* vl = c.prec == ROKS_FP32 ? (const void*)(c.d_vloc32 + (size_t)b * c.ntot)
                                         : (const void*)(c.d_vloc + (size_t)b * c.ntot);
    launch_plane_apply(c, c.d_T, c.npairs, vl, 1, c.d_potidx + nb, nb, c.d_Qpart, 0);
    launch_zpass_fwd(c, c.d_T, c.npairs, vecs, nb, c.d_ones, o);
    if (c.nproj > 0) {
      launch_apply_D(c, P, nullptr, c.d_DP);
      proj_expand(c, nb, c.d_DP, nb, dbl(o), K);
    }
    if (c.exx != 0.0) {
      // channel b = 2 L + s: K^{sL}, weights -f_m^{sL}
      std::vector<double> W((size_t)nb * nb, 0.0);
      for (int n = 0; n < nb; ++n)
        for (int m = 0; m < nb; ++m) {
          const int Y = c.band_shell[m];
          W[(size_t)n * nb + m] = Y < c.nsocc ? -c.shell_f[Y][b / 2][b % 2] : 0.0;
        }
      exx_apply(c, vecs, nb, W.data(), o, nullptr);
    }
    ++idx;
  }
}

// ---------------------------------------------------------------------------
// energy, Y = F^n|n>, theta, g_I = (1 - P) Y, and R / kappa / A
// ---------------------------------------------------------------------------
// Eq. r_matrix_singlet puts F^c in the virtual-virtual block of R: F^c is
// applied to the virtual bands (into d_w1) and their band products fill the
// block (needs the potentials and projections of the current orbitals)
static void virtual_block(Ctx& c) {
  const int nb = c.nb, K = 2 * c.npw;
  int v0 = nb, Xc = -1;
  for (int n = 0; n < nb; ++n)
    if (c.shell_virtual[c.band_shell[n]]) {
      v0 = n;
      break;
    }
  for (int X = 0; X < c.nshell; ++X)
    if (c.shell_closed[X] && Xc < 0) Xc = X;
  const int nv = nb - v0;
  if (nv == 0 || Xc < 0) return;  // no closed shell: the block stays zero
  const double2* vv = c.d_psi + (size_t)v0 * c.npw;
  double2* out = c.d_w1;
  const int np = (nv + 1) / 2;
  launch_zpass_bwd(c, vv, nv, c.d_T, np);
  const void* vsh = c.prec == ROKS_FP32 ? (const void*)c.d_vsh32 : (const void*)c.d_vsh;
  launch_plane_apply(c, c.d_T, np, vsh, c.nsocc, c.d_potidx + (size_t)5 * nb, nv, c.d_Qpart, 0);
  launch_zpass_fwd(c, c.d_T, np, vv, nv, c.d_kinw_closed, out);
  if (c.nproj > 0) {
    launch_apply_D(c, c.d_P, c.d_kinw_closed, c.d_DP);
    proj_expand(c, nv, c.d_DP + v0, nb, dbl(out), K);
  }
  if (c.exx != 0.0) {
    // F^c's exchange on the virtual rows
    const std::vector<double> W = exx_shell_weights(c, Xc);
    exx_apply(c, vv, nv, W.data() + (size_t)v0 * nb, out, nullptr);
  }
  gemm_wdot(c, nv, nv, K, dbl(vv), K, dbl(out), K, c.d_R + (size_t)v0 * nb + v0, nb, 1.0, 0.0, true);
  launch_virtual_block(c, v0);
}

// S|psi_n> of the current orbitals into d_Spsi (needs their projections in
// d_P); without overlap coefficients S = 1 and the orbitals serve as they are
static void make_overlap_psi(Ctx& c) {
  if (!c.has_q) return;
  const int K = 2 * c.npw;
  copy_dev(c, c.d_Spsi, c.d_psi, (size_t)c.nb * c.npw * sizeof(double2));
  launch_apply_Q(c, c.d_P, c.d_DP);
  proj_expand(c, c.nb, c.d_DP, c.nb, dbl(c.d_Spsi), K);
}

const double2* overlap_psi(const Ctx& c) { return c.has_q ? c.d_Spsi : c.d_psi; }

// the occupied block of gamma (Eq. gamma_def) of the current orbitals into G
// [nb][nb]: theta from one application of the shell operators
static void overlap_multipliers(Ctx& c, double* G) {
  const int nb = c.nb, K = 2 * c.npw;
  apply_operator(c, c.d_psi, 0, c.d_Y, false);
  gemm_wdot(c, nb, nb, K, dbl(c.d_psi), K, dbl(c.d_Y), K, c.d_theta, nb, 1.0, 0.0, true);
  launch_overlap_multipliers(c, c.d_theta, G);
}

void energy_gradient(Ctx& c, roks_energies* e, double* open_out, bool want_vv) {
  ROKS_CHECK(c.have_orbitals, ROKS_ERR_STATE, "no orbitals set");
  const int nb = c.nb, K = 2 * c.npw;
  const size_t band = (size_t)nb * c.npw;
  if (!c.potentials_valid) compute_potentials(c, c.d_psi, &c.last_e);
  ROKS_CHECK(std::isfinite(c.last_e.E), ROKS_ERR_NAN, "non-finite energy");
  if (e) *e = c.last_e;
  apply_operator(c, c.d_psi, 0, c.d_Y, true);
  make_overlap_psi(c);
  gemm_wdot(c, nb, nb, K, dbl(c.d_psi), K, dbl(c.d_Y), K, c.d_theta, nb, 1.0, 0.0, true);
  // g_I = Y - sum_m S|m> theta_mn (Eq. gradient)
  gemm_expand_to(c, nb, K, nb, c.d_theta, nb, false, dbl(overlap_psi(c)), K, dbl(c.d_Y), K,
                 dbl(c.d_gI), K, -1.0, 1.0);
  launch_subspace(c, open_out);
  if (want_vv || (c.flags & ROKS_FLAG_CANONICALIZE)) virtual_block(c);
}

double smallest_trial_step(const Ctx& c) { return c.dt / std::ldexp(1.0, kHalvings); }

void reset_cg(Ctx& c) {
  c.have_old = false;
  c.pg_old = 0.0;
  c.dt = kDtInit;
  c.since_restart = 0;
  c.psold_iter = -1;
}

// ---------------------------------------------------------------------------
// one CG iteration (Eqs. orbital_update, cg_search, prec_grad_I, prec_k and the
// conjugated rotation; readings R1-R7, R9 of the oracle)
// ---------------------------------------------------------------------------
void pcg_step(Ctx& c, roks_step_info* info) {
  const int nb = c.nb, K = 2 * c.npw;
  const size_t band = (size_t)nb * c.npw, nn = (size_t)nb * nb;
  // periodic restart: every restart_period steps the carried directions and
  // the step length estimate are dropped (a fresh preconditioned gradient)
  reset_diis(c);  // the kept DIIS iterates do not lead to these orbitals
  const bool periodic = c.restart_period > 0 && c.since_restart >= c.restart_period;
  if (periodic) reset_cg(c);
  c.since_restart++;
  // step scalars, written by the kernels straight into the pinned mirror
  // (read after a synchronisation): [0] sum A (theta - theta^T), [1] the same
  // for D, [2] max open-shell coupling, [kStage + n] <p_n|g_n>,
  // [kStage + nb + n] <g_n|g_n>, [kStage + 2 nb + n] <S_n|g_n>; sums over
  // bands in band order
  double* st = c.hd_stage;
  const double* hs = c.h_stage;
  int no = 0;  // open shells
  for (int X = 0; X < c.nshell; ++X)
    if (!c.shell_closed[X] && !c.shell_virtual[X]) ++no;
  roks_energies e0;
  // with the report's open-shell coupling (two open shells)
  energy_gradient(c, &e0, no == 2 ? st + 2 : nullptr);
  const double E0 = e0.E;

  // preconditioned out-of-subspace gradient p = (1 - P) K g_I; with a
  // network attached K carries the learned factor of (band, |G|^2 shell)
  band_dots2(c, c.d_gI, c.d_gI, nb, c.d_bandv + nb, c.d_bandv, st + kStage + nb, nullptr);
  const bool recording = c.rec_max > 0 && c.rec_count < c.rec_max &&
                         (c.iteration % std::max(1, c.rec_stride)) == 0;
  if (c.mlp || recording) {
    band_dots(c, c.d_psi, c.d_psi, nb, 1, c.d_bandv + 4 * nb);
    launch_features(c, c.d_bandv, c.d_bandv + nb, c.d_bandv + 4 * nb);
  }
  if (recording) record_iterate(c, c.d_bandv, c.d_bandv + nb, c.d_bandv + 4 * nb);
  const double* bandw = (c.flags & ROKS_FLAG_WEIGHT_PRECOND) ? c.d_kinw_shell : nullptr;
  auto band_sum = [&](int off) {
    double v = 0.0;
    for (int n = 0; n < nb; ++n) v += hs[kStage + off + n];
    return v;
  };
  // launches of p = (1 - P) K g_I and of the parts of <p|g> = sum <p_I|g_I> +
  // 1/2 sum A (theta - theta^T), kept on the device (d_cg) and mirrored
  // with_sold: the same band product also gives <psi|S_old> (S_old follows w1
  // in memory), in columns nb .. 2 nb - 1 of d_m12
  auto precondition_async = [&](bool learned, bool with_sold) {
    if (learned)
      launch_teter_scaled(c, c.d_bandv, c.d_bandv + nb, c.d_gI, bandw, c.d_w1);
    else
      launch_teter(c, c.d_bandv, c.d_bandv + nb, c.d_gI, bandw, c.d_w1);
    const int nc = with_sold ? 2 * nb : nb;
    // <m|S K g_I> (and <m|S S_old>): the projections of Eq. prec_grad_I
    gemm_wdot(c, nb, nc, K, dbl(overlap_psi(c)), K, dbl(c.d_w1), K, c.d_m12, nc, 1.0, 0.0, true);
    gemm_expand_to(c, nb, K, nb, c.d_m12, nc, false, dbl(c.d_psi), K, dbl(c.d_w1), K, dbl(c.d_p), K,
                   -1.0, 1.0);
    band_dots_asym(c, c.d_p, c.d_gI, nb, c.d_cg + 8, st + kStage, c.d_A, c.d_theta, c.d_cg, st);
  };
  // <p|g> from the mirrored parts, in the order of the device's sum
  auto pg_host = [&]() { return band_sum(0) + 0.5 * hs[0]; };
  const bool learned = c.mlp != nullptr;
  // with carried directions the Fletcher-Reeves ratio is formed on the device
  // and the directions follow without a round trip to the host
  const bool dev_beta = c.have_old && c.pg_old != 0.0;
  // <psi|S_old> is known from the last step's commit when the orbitals and
  // S_old are the ones it left (S = 1): the band product then skips S_old
  const bool psold = c.have_old && !c.has_q && c.psold_iter == c.iteration;
  precondition_async(learned, c.have_old && !psold);
  bool restarted = periodic;

  // Sold projected out of the current span (kept in d_w1)
  if (c.have_old)
    gemm_expand_to(c, nb, K, nb, psold ? c.d_PSold : c.d_m12 + nb, psold ? nb : 2 * nb, false,
                   dbl(c.d_psi), K, dbl(c.d_Sold), K, dbl(c.d_w1), K, -1.0, 1.0);
  // S = p + b S_old', D = A + b D_old (b = 0: plain copies); b_dev: the factor
  // d_cg[1] formed on the device
  auto directions_async = [&](double b, bool b_dev) {
    if (b_dev) {
      cg_directions_dev(c, 2 * band, dbl(c.d_p), dbl(c.d_w1), dbl(c.d_S), nn, c.d_A, c.d_Dold, c.d_D,
                        c.d_cg, c.d_cg + 8, c.pg_old, c.d_cg + 1);
    } else if (b != 0.0) {
      axpby(c, 2 * band, 1.0, dbl(c.d_p), b, dbl(c.d_w1), dbl(c.d_S));
      axpby(c, nn, 1.0, c.d_A, b, c.d_Dold, c.d_D);
    } else {
      copy_dev(c, c.d_S, c.d_p, band * sizeof(double2));
      copy_dev(c, c.d_D, c.d_A, nn * sizeof(double));
    }
    band_dots_asym(c, c.d_S, c.d_gI, nb, nullptr, st + kStage + 2 * nb, c.d_D, c.d_theta, st + 1,
                   nullptr);
  };
  auto dE_host = [&]() { return 2.0 * band_sum(2 * nb) + hs[1]; };
  // the line search's products of S (<S|S>, <beta|S>) are queued with the
  // directions, before the synchronisation that decides on the search;
  // directions formed again drop them
  bool prepared = false, first_search = true;
  auto prepare = [&]() {
    prepare_line_search(c, first_search);
    first_search = false;
    prepared = true;
  };
  auto directions = [&](double b) {
    directions_async(b, false);
    prepared = false;
    sync(c);
    return dE_host();
  };
  double pg, beta, dE0;
  if (dev_beta) {
    directions_async(0.0, true);
    prepare();
    sync(c);
    c.normD_pending = false;
    pg = pg_host();
    beta = pg / c.pg_old;
    dE0 = dE_host();
  } else {
    // no carried directions (or pg_old = 0): beta = 0 without looking at pg
    beta = 0.0;
    directions_async(0.0, false);
    prepare();
    sync(c);
    c.normD_pending = false;
    pg = pg_host();
    dE0 = dE_host();
  }
  const double gnorm = std::sqrt(std::max(0.0, band_sum(nb)));
  const double max_rab = no == 2 ? hs[2] : 0.0;
  if (beta != 0.0 && dE0 >= 0.0) {
    beta = 0.0;
    restarted = true;
    dE0 = directions(0.0);
  }

  Trial tr[2] = {{c.d_trial[0], c.d_M, c.d_U, 0, {}, false},
                 {c.d_trial[1], c.d_Mkeep, c.d_Ukeep, 0, {}, false}};
  double tdelta[2] = {0.0, 0.0};
  // reading R7: trial step, parabola through E(0), E'(0), E(dt), keep the
  // lower of the two if it is below E(0), else halve the trial step
  auto line_search = [&](double dt, int* evals) -> int {
    for (int attempt = 0; attempt <= kHalvings; ++attempt) {
      const double t = dt / std::ldexp(1.0, attempt);
      // the first trial's potentials are never kept (tr[1] is evaluated
      // after it): energies only
      evaluate_trial(c, t, tr[0], true);
      ++*evals;
      double ts;
      if (tr[0].ok) {
        const double curv = (tr[0].E - E0 - dE0 * t) / (t * t);
        ts = curv > 0.0 ? std::min(-dE0 / (2.0 * curv), 4.0 * t) : 2.0 * t;
      } else {
        ts = 0.5 * t;
      }
      evaluate_trial(c, ts, tr[1], false);
      ++*evals;
      tdelta[0] = t;
      tdelta[1] = ts;
      const int best = (tr[1].E <= tr[0].E) ? 1 : 0;
      if (tr[best].E < E0) return best;
    }
    return -1;
  };

  int evals = 0, best = -1;
  bool fallback = false;
  auto search = [&]() {
    if (!prepared) prepare();
    return line_search(c.dt, &evals);
  };
  if (dE0 < 0.0) {
    best = search();
    if (best < 0 && beta != 0.0) {
      beta = 0.0;
      restarted = true;
      dE0 = directions(0.0);
      if (dE0 < 0.0) best = search();
    }
  }
  if (best < 0 && learned) {
    // the learned direction found no decrease: redo the step with the plain
    // Teter preconditioner from the steepest-descent direction
    fallback = true;
    precondition_async(false, false);
    sync(c);
    pg = pg_host();
    beta = 0.0;
    restarted = true;
    dE0 = directions(0.0);
    if (dE0 < 0.0) best = search();
  }
  roks_step_info r{};
  r.E0 = E0;
  r.beta = beta;
  r.dE0 = dE0;
  r.norm_gI = gnorm;
  r.max_Rab = max_rab;
  r.restarted = restarted ? 1 : 0;
  r.evaluations = evals;
  r.learned = learned ? 1 : 0;
  r.fallback = fallback ? 1 : 0;
  if (best < 0) {
    r.E1 = E0;
    r.delta = 0.0;
    r.stalled = 1;
    c.iteration++;
    r.iteration = c.iteration;
    c.potentials_valid = false;
    if (info) *info = r;
    return;
  }
  Trial& t = tr[best];
  const double delta = tdelta[best];
  r.E1 = t.E;
  r.delta = delta;
  // commit: psi <- trial (the buffers trade places), S_old <- M S,
  // D_old <- U^T D U
  std::swap(c.d_psi, c.d_trial[best]);
  gemm_expand(c, nb, K, nb, t.M, nb, true, dbl(c.d_S), K, dbl(c.d_Sold), K, 1.0, 0.0);
  if (!c.has_q) {
    // <psi_new|S_old> = delta M <S|S> M^T: psi_new = M (psi + delta S),
    // S_old = M S and <psi|S> = 0 (S was projected out of the span of psi)
    gemm_small(c, nb, nb, nb, c.d_SS, nb, false, t.M, nb, true, c.d_m3, nb, 1.0, 0.0);
    gemm_small(c, nb, nb, nb, t.M, nb, false, c.d_m3, nb, false, c.d_PSold, nb, delta, 0.0);
  }
  gemm_small(c, nb, nb, nb, c.d_D, nb, false, t.U, nb, false, c.d_m4, nb, 1.0, 0.0);
  gemm_small(c, nb, nb, nb, t.U, nb, true, c.d_m4, nb, false, c.d_Dold, nb, 1.0, 0.0);
  c.have_old = true;
  c.pg_old = pg;
  c.dt = std::min(kDtMax, std::max(kDtMin, delta));
  c.iteration++;
  r.iteration = c.iteration;
  c.psold_iter = c.has_q ? -1 : c.iteration;
  // the last trial evaluated is tr[1]: when it is the one taken, its
  // densities, potentials, projections and energies are those of the new
  // orbitals (the same kernels on the same values), so they are kept
  c.potentials_valid = (best == 1);
  if (best == 1) c.last_e = t.e;
  // no synchronisation: the updates above are stream-ordered before the next
  // call's work, and info holds host values only
  if (info) *info = r;
}

// ---------------------------------------------------------------------------
// Cholesky orthonormalisation in band order
// ---------------------------------------------------------------------------
void orthonormalize(Ctx& c, double2* vecs) {
  const int nb = c.nb, K = 2 * c.npw;
  const size_t band = (size_t)nb * c.npw;
  gemm_wdot(c, nb, nb, K, dbl(vecs), K, dbl(vecs), K, c.d_gram, nb, 1.0, 0.0, true);
  if (c.has_q) {
    // the Gram matrix of the overlap operator: + P^T q P
    proj_wdot(c, nb, dbl(vecs), K, c.d_dP, nb);
    launch_apply_Q(c, c.d_dP, c.d_DP);
    gemm_small(c, nb, nb, c.nproj, c.d_dP, nb, true, c.d_DP, nb, false, c.d_gram, nb, 1.0, 1.0);
  }
  cholesky_inverse(c, c.d_gram, nb, c.d_Linv, c.d_flag);
  int32_t flag = 0;
  to_host(c, &flag, c.d_flag, sizeof(int32_t));
  ROKS_CHECK(flag == 0, ROKS_ERR_NOT_PD, "orbitals are linearly dependent (Gram not positive definite)");
  copy_dev(c, c.d_w1, vecs, band * sizeof(double2));
  gemm_expand(c, nb, K, nb, c.d_Linv, nb, true, dbl(c.d_w1), K, dbl(vecs), K, 1.0, 0.0);
}

// ---------------------------------------------------------------------------
// forces (Eq. force_hf)
// ---------------------------------------------------------------------------
void forces(Ctx& c, double* f_host) {
  ensure_potentials(c);
  const int nb = c.nb, K = 2 * c.npw;
  const int nat = c.natoms;
  if (nat == 0) return;
  if (!c.d_force_loc) c.d_force_loc = dalloc<double>(c, 3 * (size_t)nat);
  // with overlap coefficients: gamma of the occupied bands (Eq. gamma_def)
  if (c.has_q && c.nproj > 0) overlap_multipliers(c, c.d_m1);
  // local part, dE/dR_I from rho_w = sum_L c_L rho_L, on the side stream
  ensure_side_stream(c);
  ROKS_HIP(hipEventRecord(c.ev_fork, c.stream));
  ROKS_HIP(hipStreamWaitEvent(c.side, c.ev_fork, 0));
  {
    const hipStream_t main = c.stream;
    c.stream = c.side;
    launch_pack_rho_weighted(c);
    launch_fft3d(c, c.d_fft, -1);
    const int nblk = 32;
    launch_local_force(c, c.d_fft, c.d_part, nblk);
    launch_reduce_strided(c, c.d_part, nat, nblk, 3, 1.0, c.d_force_loc);
    c.stream = main;
  }
  ROKS_HIP(hipEventRecord(c.ev_join, c.side));
  // nonlocal part on the main stream: 2 sum_n w_n <d beta_i|n> (D P)_in
  // (P = <beta|psi> is current: the energy evaluation of these orbitals left it);
  // the last kernel also adds the local part and negates, F = -dE/dR
  if (c.nproj > 0) {
    if (!c.d_gcart) {
      c.d_gcart = dalloc<double>(c, 3 * (size_t)c.npw);
      launch_gcart(c, c.d_gcart);
    }
    // the field, then 3 nproj partial sums (the side stream's local part
    // uses d_part meanwhile)
    if (!c.d_phi) c.d_phi = dalloc<double>(c, (size_t)c.nproj * (K + 3));
    // w_n (D P)_in, then the force field Phi_i = sum_n w_n (D P)_in psi_n: one
    // product over the bands in place of three derivative projections
    launch_apply_D(c, c.d_P, c.d_kinw_shell, c.d_DP);
    if (c.has_q) {
      // the overlap term -sum_{mn occ} gamma_mn <m|dS/dR|n> enters the same
      // field as -(q P gamma)_in: Tr(gamma S'), which SI S2 evaluates in the
      // eigenbasis of gamma, contracted here by one product instead (gamma
      // in d_m1, formed before the side stream started)
      launch_apply_Q(c, c.d_P, c.d_dP);
      gemm_small(c, c.nproj, nb, nb, c.d_dP, nb, false, c.d_m1, nb, false, c.d_DP, nb, -1.0, 1.0);
    }
    proj_field(c, c.d_DP, nb, dbl(c.d_psi), K, c.d_phi);
    ROKS_HIP(hipStreamWaitEvent(c.stream, c.ev_join, 0));
    // straight into the pinned host mirror
    launch_nl_force(c, c.d_phi, c.d_phi + (size_t)c.nproj * K, c.d_force_loc, c.hd_force);
    sync(c);
    std::memcpy(f_host, c.h_force, 3 * (size_t)nat * sizeof(double));
  } else {
    ROKS_HIP(hipStreamWaitEvent(c.stream, c.ev_join, 0));
    axpby(c, 3 * (size_t)nat, -1.0, c.d_force_loc, 0.0, c.d_force_loc, c.d_force);
    to_host(c, f_host, c.d_force, 3 * (size_t)nat * sizeof(double));
  }
}

}  // namespace roks
