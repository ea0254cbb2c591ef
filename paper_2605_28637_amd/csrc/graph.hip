// Graph mode: CG iterations whose every decision is taken on the device, so
// that k of them form one fixed launch sequence, captured once per context as
// a HIP graph and replayed (for a batch, each context's graph on its worker's
// stream).
//
// The iteration is roks_pcg_step's (Eqs. orbital_update, cg_search,
// prec_grad_I, prec_k and the conjugated rotation; readings R1-R7, R9) with
// the scalars that steer it kept in a device state block instead of host
// variables: the energy of the orbitals (assembled on the device in the
// host's order of sums), the Fletcher-Reeves ratio and the directional
// derivative (the restart to steepest descent when it is not negative), the
// trial step (the previous step length), the parabola's step, the choice of
// the lower trial and its acceptance below E(0), and the new step length.
// Each trial is formed as on the host (Cholesky of I + t^2 <S|S>, exp(t D),
// M^T (psi + t S)) with the scaled inputs prepared by small kernels that read
// t, so the existing launchers run with constant arguments; a trial's
// projections are M^T-rotated from those of psi + t S, as on the host.  Past
// 78 bands the exponential
// takes a fixed Taylor degree and a squaring count chosen on the device
// (squaring launches past it undone), where the host chooses both from the
// norm.  The commit (new orbitals, carried directions S_old = M S, D_old =
// U^T D U, and the potentials of the trial taken) is a set of copies made
// only when the device accepted the step.  The first rejected step halts the
// replay (later iterations commit nothing); what the host path does then
// (halving the trial step, the steepest descent retry) is left to it: the
// caller sees the first rejected iteration and continues with roks_pcg_step.
//
// Scope (checked before capture): FP64 or FP32 tier, LDA or PBE without
// exact exchange, no overlap coefficients, no recording, no
// canonicalisation, no autotuning; periodic restarts and the learned
// rescaling of the preconditioner are taken on the device (the plain
// preconditioner's retry after a failed learned search is the host step's).
#include <cmath>
#include <cstring>
#include <mutex>

#include "roks_internal.h"

namespace roks {

namespace {

// slots of the device state block
enum : int {
  gE0 = 0, gEt, gEts, gT, gTs, gDt, gPg, gPgOld, gBeta, gDE0, gDelta, gE1, gHaveOld, gAccept,
  gBest, gOkT, gOkTs, gHalt, gNormG, gRestart, gNormD, gSq, gSince, gSinceNew, gPeriod, gReuseT, gNSlots
};
constexpr int kRecLen = 8;  // per iteration: E0, E1, delta, beta, dE0, accepted, |g_I|, restarted

__device__ inline double mul(double a, double b) { return __dmul_rn(a, b); }
__device__ inline double add(double a, double b) { return __dadd_rn(a, b); }
__device__ inline double sub(double a, double b) { return __dsub_rn(a, b); }
__device__ inline double dvd(double a, double b) { return __ddiv_rn(a, b); }

// carry: the orbitals are the previous iteration's accepted trial, whose
// energy is E(0) (its potentials and projections were kept)
__global__ void k_g_begin(double* __restrict__ gs, int carry) {
  if (threadIdx.x || blockIdx.x) return;
  if (carry) gs[gE0] = gs[gE1];
  gs[gAccept] = 0.0;
  gs[gBest] = 0.0;
}

// E = sum_L c_L (T_L + NL_L + ext_L + H_L + xc_L) from the reduced partial
// sums, in the host's order (assemble_energies); a failed Cholesky (flag)
// makes the trial's energy +inf
__global__ void k_g_energy(const double* __restrict__ scal, int nb, int nconf,
                           const double* __restrict__ focc, double c0, double c1, double dv,
                           int energy_only, const int32_t* __restrict__ flag, double* __restrict__ gs,
                           int slot, int okslot) {
  if (threadIdx.x || blockIdx.x) return;
  const double* kin = scal + 16;
  const double* enl = scal + 16 + nb;
  double E = 0.0;
  for (int L = 0; L < nconf; ++L) {
    double k = 0.0, nl = 0.0;
    for (int n = 0; n < nb; ++n) {
      const double f = focc[L * nb + n];
      k = add(k, mul(f, kin[n]));
      nl = add(nl, mul(f, enl[n]));
    }
    const double xc = mul(dv, scal[3 * L + 0]);
    const double ext = mul(dv, scal[3 * L + 1]);
    const double har = mul(mul(0.5, dv), energy_only ? scal[6 + L] : scal[3 * L + 2]);
    const double EL = add(add(add(add(k, nl), ext), har), xc);
    E = add(E, mul(L == 0 ? c0 : c1, EL));
  }
  // flag[0]: the factorisation; flag[1]: the exponential past 78 bands
  const bool ok = !flag || (flag[0] | flag[1]) == 0;
  if (!ok || !isfinite(E)) E = INFINITY;
  gs[slot] = E;
  if (okslot >= 0) gs[okslot] = ok ? 1.0 : 0.0;
}

// sum_n x[n] in band order
__device__ inline double band_sum(const double* __restrict__ x, int nb) {
  double s = 0.0;
  for (int n = 0; n < nb; ++n) s = add(s, x[n]);
  return s;
}

// Scalars every block of a fused kernel needs are formed by its thread 0
// from state slots that the kernel does not write, and only block 0 stores
// them; the parallel part follows a barrier.

// <p|g> and the Fletcher-Reeves ratio; the directional derivative of the
// directions S = p + beta w, D = A + beta D_old from the band sums of p and
// w against g_I and the rotation terms; beta = 0 when it is not a descent
// direction; the first trial step is the step length kept from before.
// Then S (n1 values) and D (n2 values).
__global__ void __launch_bounds__(256) k_g_directions(
    const double* __restrict__ pgb, const double* __restrict__ asymA, const double* __restrict__ wgb,
    const double* __restrict__ asymD, const double* __restrict__ gg, int nb, double* __restrict__ gs,
    size_t n1, const double* __restrict__ p, const double* __restrict__ w, double* __restrict__ S,
    size_t n2, const double* __restrict__ A, const double* __restrict__ Dold, double* __restrict__ D) {
  __shared__ double sb;
  if (threadIdx.x == 0) {
    // periodic restart (reading R23): every gPeriod steps the carried
    // directions and the step length are dropped
    const bool periodic = gs[gPeriod] > 0.0 && gs[gSince] >= gs[gPeriod];
    const double spg = band_sum(pgb, nb);
    const double swg = band_sum(wgb, nb);
    const double pg = add(spg, mul(0.5, asymA[0]));
    double beta = 0.0;
    if (!periodic && gs[gHaveOld] != 0.0 && gs[gPgOld] != 0.0) beta = dvd(pg, gs[gPgOld]);
    double dE0 = add(mul(2.0, add(spg, mul(beta, swg))), add(asymA[0], mul(beta, asymD[0])));
    const bool restart = beta != 0.0 && dE0 >= 0.0;
    if (restart) {
      beta = 0.0;
      dE0 = add(mul(2.0, spg), asymA[0]);
    }
    sb = beta;
    if (blockIdx.x == 0) {
      gs[gRestart] = (restart || periodic) ? 1.0 : 0.0;
      gs[gPg] = pg;
      gs[gBeta] = beta;
      gs[gDE0] = dE0;
      gs[gT] = periodic ? (double)kDtInit : gs[gDt];
      gs[gSinceNew] = periodic ? 1.0 : gs[gSince] + 1.0;
      gs[gNormG] = sqrt(fmax(0.0, band_sum(gg, nb)));
    }
  }
  __syncthreads();
  const double b = sb;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n1 + n2;
       i += (size_t)gridDim.x * blockDim.x) {
    const bool first = i < n1;
    const size_t k = first ? i : i - n1;
    double v = 1.0 * (first ? p[k] : A[k]);
    v += b * (first ? w[k] : Dold[k]);
    (first ? S : D)[k] = v;
  }
}

// reading R7 on the device: the parabola through E(0), E'(0), E(t)
__device__ inline double parabola_step(const double* gs) {
  const double t = gs[gT], E0 = gs[gE0], dE0 = gs[gDE0];
  if (gs[gOkT] == 0.0) return mul(0.5, t);
  const double curv = dvd(sub(sub(gs[gEt], E0), mul(dE0, t)), mul(t, t));
  return curv > 0.0 ? fmin(dvd(-dE0, mul(2.0, curv)), mul(4.0, t)) : mul(2.0, t);
}

// the scaled inputs of a trial: gram = t^2 <S|S> + I, Dt = t D (n x n),
// St = t S (m values), PSt = t <beta|S> (mp values), at t = gs[gT] (first
// trial) or at the parabola's step (second trial, stored in gs[gTs])
__global__ void __launch_bounds__(256) k_g_prep(int nb, const double* __restrict__ SS,
                                                double* __restrict__ gram, const double* __restrict__ D,
                                                double* __restrict__ Dt, size_t m,
                                                const double* __restrict__ S, double* __restrict__ St,
                                                size_t mp, const double* __restrict__ PS,
                                                double* __restrict__ PSt, double* __restrict__ gs,
                                                int second) {
  __shared__ double st;
  if (threadIdx.x == 0) {
    st = second ? parabola_step(gs) : gs[gT];
    if (second && blockIdx.x == 0) gs[gTs] = st;
  }
  __syncthreads();
  const double t = st;
  const double t2 = t * t;
  const size_t nn = (size_t)nb * nb;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn + m + mp;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < nn) {
      const int r = (int)(i / nb), q = (int)(i - (size_t)r * nb);
      gram[i] = t2 * SS[i] + (r == q ? 1.0 : 0.0);
      if (Dt) Dt[i] = t * D[i];
    } else if (i < nn + m) {
      St[i - nn] = t * S[i - nn];
    } else {
      PSt[i - nn - m] = t * PS[i - nn - m];
    }
  }
}

// x *= gs[slot]
__global__ void __launch_bounds__(256) k_g_scale(size_t n, double* __restrict__ x,
                                                 const double* __restrict__ gs, int slot) {
  const double f = gs[slot];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] *= f;
}

// Past the single-workgroup exponential: exp(X) by scaling and squaring
// around a Taylor polynomial of fixed degree kTaylor (the launches are fixed;
// the polynomial by the Paterson-Stockmeyer scheme)
// with a squaring count s chosen on the device, the smallest with
// ||X||_1 / 2^s <= 1 (so the truncation error stays below
// 1 / (kTaylor + 1)! < 1e-17); kSqMax squaring launches, those past s undone.
// A count past kSqMax or a non-finite norm marks the trial failed (flag).
constexpr int kTaylor = 18;
constexpr int kSqMax = 12;

// X = t D / 2^s at the trial's t (gs[gTs] for the second trial)
__global__ void __launch_bounds__(256) k_g_expm_prep(int n, const double* __restrict__ D,
                                                     double* __restrict__ X, double* __restrict__ gs,
                                                     int second, int32_t* __restrict__ flag) {
  __shared__ double sc;
  if (threadIdx.x == 0) {
    const double t = second ? gs[gTs] : gs[gT];
    double nrm = fabs(t) * gs[gNormD];
    int sq = 0;
    while (nrm > 1.0 && sq <= kSqMax) {
      nrm *= 0.5;
      ++sq;
    }
    const bool ok = isfinite(nrm) && sq <= kSqMax;
    sc = ok ? ldexp(t, -sq) : 0.0;
    if (blockIdx.x == 0) {
      gs[gSq] = ok ? sq : 0;
      flag[1] = ok ? 0 : 2;
    }
  }
  __syncthreads();
  const double f = sc;
  const size_t nn = (size_t)n * n;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x)
    X[i] = f * D[i];
}

// squaring number `index`: kept only when index < s, else its input stays
__global__ void __launch_bounds__(256) k_g_keep(size_t nn, double* __restrict__ nxt,
                                                const double* __restrict__ cur,
                                                const double* __restrict__ gs, int index) {
  if (index < (int)gs[gSq]) return;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x)
    nxt[i] = cur[i];
}

// conditional copies dst = (best ? t1 : t0), in 4-byte words: always, when
// the step is accepted, or when it is accepted with the first trial
enum : int { kAlways = 0, kAccepted = 1, kFirstTaken = 2 };
constexpr int kMaxSegs = 10;
struct Seg {
  const uint32_t* t0;
  const uint32_t* t1;
  uint32_t* dst;
  size_t n;
  int cond;
};
struct Segs {
  Seg s[kMaxSegs];
  int count;
};

__device__ inline void copy_segs(const Segs& g, bool acc, bool best) {
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int k = 0; k < g.count; ++k) {
    const Seg& q = g.s[k];
    if (q.cond != kAlways && !acc) continue;
    if (q.cond == kFirstTaken && best) continue;
    const uint32_t* src = best ? q.t1 : q.t0;
    for (size_t i = tid; i < q.n; i += stride) q.dst[i] = src[i];
  }
}

// the lower trial, kept if it lies below E(0) and the direction descends;
// then the copies that depend on that choice
__global__ void __launch_bounds__(256) k_g_accept(double* __restrict__ gs, Segs g) {
  __shared__ int sflags;
  if (threadIdx.x == 0) {
    const double Et = gs[gEt], Ets = gs[gEts];
    const int best = Ets <= Et ? 1 : 0;
    const double Eb = best ? Ets : Et;
    const bool acc = gs[gHalt] == 0.0 && gs[gDE0] < 0.0 && Eb < gs[gE0];
    sflags = (acc ? 1 : 0) | (best << 1);
    if (blockIdx.x == 0) {
      gs[gBest] = best;
      gs[gAccept] = acc ? 1.0 : 0.0;
      gs[gDelta] = best ? gs[gTs] : gs[gT];
      gs[gE1] = acc ? Eb : gs[gE0];
    }
  }
  __syncthreads();
  copy_segs(g, (sflags & 1) != 0, (sflags & 2) != 0);
}

// the remaining copies of an accepted step, its carried scalars and the
// iteration's record; the first rejected step halts the rest (they commit
// nothing)
__global__ void __launch_bounds__(256) k_g_finish(double* __restrict__ gs, Segs g,
                                                  double* __restrict__ rec, double* __restrict__ mirror,
                                                  double dt_min, double dt_max) {
  const bool acc = gs[gAccept] != 0.0;
  const bool best = gs[gBest] != 0.0;
  copy_segs(g, acc, best);
  if (threadIdx.x || blockIdx.x) return;
  // the second trial, taken, leaves its z pass in the column buffer
  gs[gReuseT] = (acc && gs[gBest] != 0.0) ? 1.0 : 0.0;
  if (acc) {
    gs[gPgOld] = gs[gPg];
    gs[gHaveOld] = 1.0;
    gs[gDt] = fmin(dt_max, fmax(dt_min, gs[gDelta]));
    gs[gSince] = gs[gSinceNew];
  } else {
    gs[gHalt] = 1.0;
  }
  rec[0] = gs[gE0];
  rec[1] = gs[gE1];
  rec[2] = acc ? gs[gDelta] : 0.0;
  rec[3] = gs[gBeta];
  rec[4] = gs[gDE0];
  rec[5] = acc ? 1.0 : 0.0;
  rec[6] = gs[gNormG];
  rec[7] = gs[gRestart];
  for (int i = 0; i < gNSlots; ++i) mirror[i] = gs[i];
}

size_t grid_for(size_t n) { return std::min<size_t>(4096, (n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------------------
// one iteration, every launch on c.stream, no host reads
// ---------------------------------------------------------------------------
// a list of conditional copies for k_g_accept / k_g_finish
struct SegList {
  Segs g{};
  size_t most = 0;
  void add(const void* t0, const void* t1, void* dst, size_t bytes, int cond) {
    ROKS_CHECK(g.count < kMaxSegs && bytes % 4 == 0, ROKS_ERR_STATE, "copy list overflow");
    g.s[g.count++] = Seg{static_cast<const uint32_t*>(t0), static_cast<const uint32_t*>(t1),
                         static_cast<uint32_t*>(dst), bytes / 4, cond};
    most = std::max(most, bytes / 4);
  }
  unsigned grid() const { return (unsigned)std::max<size_t>(1, grid_for(most)); }
};

// the first trial's potentials, projections and reduced sums (with the
// band kinetic and nonlocal energies, which the subspace matrices read) go
// to the second set of buffers (captured pointers: the members are only
// swapped while the launches are made)
struct AltPotentials {
  Ctx& c;
  AltPotentials(Ctx& cc) : c(cc) { swap(); }
  ~AltPotentials() { swap(); }
  void swap() {
    std::swap(c.d_vsh, c.d_gvsh);
    std::swap(c.d_vloc, c.d_gvloc);
    std::swap(c.d_vsh32, c.d_gvsh32);
    std::swap(c.d_vloc32, c.d_gvloc32);
    std::swap(c.d_P, c.d_gP);
    std::swap(c.d_red, c.d_gscal);
    c.d_kin = c.d_red + 16;
    c.d_enl = c.d_red + 16 + c.nb;
  }
};

static void graph_trial(Ctx& c, double2* out, double* M, double* U, bool alt, int eslot,
                        int okslot) {
  const int nb = c.nb, K = 2 * c.npw;
  const size_t band = (size_t)nb * c.npw, nn = (size_t)nb * nb;
  const bool lds = expm_in_lds(c);
  const size_t mp = (size_t)c.nproj * nb;
  hipLaunchKernelGGL(k_g_prep, dim3((unsigned)grid_for(nn + 2 * band + mp)), dim3(256), 0, c.stream, nb,
                     c.d_SS, c.d_gram, c.d_D, lds ? c.d_m1 : nullptr, 2 * band, dbl(c.d_S), dbl(c.d_Pt),
                     mp, c.d_PS, c.d_gPSt, c.d_gstate, alt ? 0 : 1);
  ROKS_HIP(hipGetLastError());
  if (lds) {
    launch_chol_expm_lds(c, c.d_gram, 1.0, 0.0, c.d_Linv, c.d_flag, c.d_m1, 1.0, U);
  } else {
    // past 128 bands (the panel factorisation) the exponential runs on the
    // side stream, a branch of the graph, beside the factorisation, with
    // scratch of its own and the upper half of the split-K partials buffer
    // (restored on every exit); below, a branch costs more than it hides (the
    // uneven batch replayed 0.84x as fast with branches at 79-120 bands)
    const bool branch = nb > 128;
    if (branch) {
      ensure_side_stream(c);
      ROKS_HIP(hipEventRecord(c.ev_fork, c.stream));
      ROKS_HIP(hipStreamWaitEvent(c.side, c.ev_fork, 0));
    }
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
    if (branch) {
      const size_t half = c.gemm_part_capacity / 2;
      c.gemm_part_capacity = half;
      c.d_gemm_part = halves.part + half;
      c.stream = c.side;
    }
    double* X = c.d_ex;
    double* w[4] = {c.d_ex + nn, c.d_ex + 2 * nn, c.d_ex + 3 * nn, c.d_ex + 4 * nn};
    hipLaunchKernelGGL(k_g_expm_prep, dim3((unsigned)grid_for(nn)), dim3(256), 0, c.stream, nb, c.d_D, X,
                       c.d_gstate, alt ? 0 : 1, c.d_flag);
    ROKS_HIP(hipGetLastError());
    // the series of degree kTaylor (Paterson-Stockmeyer: 8 products), then
    // the squarings
    double* cur = taylor_ps(c, nb, kTaylor, X, w[0], w[1], w[2], w[3]);
    double* nxt = cur == w[2] ? w[3] : w[2];
    for (int i = 0; i < kSqMax; ++i) {
      gemm_small(c, nb, nb, nb, cur, nb, false, cur, nb, false, nxt, nb, 1.0, 0.0);
      hipLaunchKernelGGL(k_g_keep, dim3((unsigned)grid_for(nn)), dim3(256), 0, c.stream, nn, nxt, cur,
                         c.d_gstate, i);
      ROKS_HIP(hipGetLastError());
      std::swap(cur, nxt);
    }
    copy_dev(c, U, cur, nn * sizeof(double));
    if (branch) ROKS_HIP(hipEventRecord(c.ev_join, c.side));
    c.stream = halves.main;
    c.d_gemm_part = halves.part;
    cholesky_inverse(c, c.d_gram, nb, c.d_Linv, c.d_flag);
    if (branch) ROKS_HIP(hipStreamWaitEvent(c.stream, c.ev_join, 0));
  }
  gemm_small(c, nb, nb, nb, U, nb, true, c.d_Linv, nb, false, M, nb, 1.0, 0.0);
  gemm_expand_sum(c, nb, K, nb, M, nb, true, dbl(c.d_psi), dbl(c.d_Pt), 1.0, K, dbl(out), K, dbl(out),
                  K, 1.0, 0.0);
  // the trial's projections M^T-rotated from those of psi + t S (P0 + t PS)
  auto evaluate = [&]() {
    if (c.nproj > 0)
      gemm_small2(c, c.nproj, nb, nb, c.d_P0, c.d_gPSt, 1.0, nb, false, M, nb, true, c.d_P, nb, 1.0, 0.0,
                  0.0);
    compute_potentials_async(c, out, true, false);
  };
  if (alt) {
    AltPotentials swap(c);
    evaluate();
  } else {
    evaluate();
  }
  hipLaunchKernelGGL(k_g_energy, dim3(1), dim3(64), 0, c.stream, alt ? c.d_gscal : c.d_scal, nb, c.nconf,
                     c.d_gfocc, c.cL[0], c.cL[1], c.omega / (double)c.ntot, 0, c.d_flag, c.d_gstate,
                     eslot, okslot);
  ROKS_HIP(hipGetLastError());
}

// carry: the previous iteration (of the same graph) left the potentials and
// projections of the orbitals it accepted, and their energy, in place
static void graph_step(Ctx& c, int step, bool carry) {
  struct InGraph {
    Ctx& c;
    InGraph(Ctx& cc) : c(cc) { c.in_graph = true; }
    ~InGraph() { c.in_graph = false; }
  } in_graph(c);
  const int nb = c.nb, K = 2 * c.npw;
  const size_t band = (size_t)nb * c.npw, nn = (size_t)nb * nb;
  double* gs = c.d_gstate;
  hipLaunchKernelGGL(k_g_begin, dim3(1), dim3(64), 0, c.stream, gs, carry ? 1 : 0);
  ROKS_HIP(hipGetLastError());
  // energy, Y = F^n|n>, theta, g_I = (1 - P) Y, R / kappa / A
  if (!carry) {
    compute_potentials_async(c, c.d_psi, false, false);
    hipLaunchKernelGGL(k_g_energy, dim3(1), dim3(64), 0, c.stream, c.d_scal, nb, c.nconf, c.d_gfocc,
                       c.cL[0], c.cL[1], c.omega / (double)c.ntot, 0,
                       static_cast<const int32_t*>(nullptr), gs, (int)gE0, -1);
    ROKS_HIP(hipGetLastError());
  }
  c.potentials_valid = true;  // the apply reads the projections in d_P
  // after a taken second trial its z pass is still in the column buffer
  // (both in the tier of the apply unless the FP32 tier's densities run in
  // FP64)
  const bool same_tier = !(c.prec == ROKS_FP32 && !fp32_density_planes(c));
  c.zskip = carry && same_tier ? gs + gReuseT : nullptr;
  apply_operator(c, c.d_psi, 0, c.d_Y, true);
  c.zskip = nullptr;
  gemm_wdot(c, nb, nb, K, dbl(c.d_psi), K, dbl(c.d_Y), K, c.d_theta, nb, 1.0, 0.0, true);
  gemm_expand_to(c, nb, K, nb, c.d_theta, nb, false, dbl(c.d_psi), K, dbl(c.d_Y), K, dbl(c.d_gI), K,
                 -1.0, 1.0);
  launch_subspace(c, nullptr);
  // p = (1 - P) K g_I and the projected carried direction (S_old is zero
  // until a step has been accepted)
  band_dots2(c, c.d_gI, c.d_gI, nb, c.d_bandv + nb, c.d_bandv, nullptr, nullptr);
  const double* bandw = (c.flags & ROKS_FLAG_WEIGHT_PRECOND) ? c.d_kinw_shell : nullptr;
  if (c.mlp) {
    // the learned rescaling of K (its features from <g|T|g>, <g|g>, <n|T|n>)
    band_dots(c, c.d_psi, c.d_psi, nb, 1, c.d_bandv + 4 * nb);
    launch_features(c, c.d_bandv, c.d_bandv + nb, c.d_bandv + 4 * nb);
    launch_teter_scaled(c, c.d_bandv, c.d_bandv + nb, c.d_gI, bandw, c.d_w1);
  } else {
    launch_teter(c, c.d_bandv, c.d_bandv + nb, c.d_gI, bandw, c.d_w1);
  }
  // <psi|S_old>: after an accepted iteration of this replay (carry) from its
  // commit (delta M <S|S> M^T), else a band product beside <psi|w>
  const int nc = carry ? nb : 2 * nb;
  gemm_wdot(c, nb, nc, K, dbl(c.d_psi), K, dbl(c.d_w1), K, c.d_m12, nc, 1.0, 0.0, true);
  gemm_expand_to(c, nb, K, nb, c.d_m12, nc, false, dbl(c.d_psi), K, dbl(c.d_w1), K, dbl(c.d_p), K,
                 -1.0, 1.0);
  band_dots_asym(c, c.d_p, c.d_gI, nb, c.d_cg + 8, nullptr, c.d_A, c.d_theta, c.d_cg, nullptr);
  gemm_expand_to(c, nb, K, nb, carry ? c.d_PSold : c.d_m12 + nb, carry ? nb : 2 * nb, false,
                 dbl(c.d_psi), K, dbl(c.d_Sold), K, dbl(c.d_w1), K, -1.0, 1.0);
  double* wgb = gs + gNSlots;          // [nb] <w_n|g_n>
  double* asymD = gs + gNSlots + nb;   // [1] sum D_old (theta - theta^T)
  band_dots_asym(c, c.d_w1, c.d_gI, nb, wgb, nullptr, c.d_Dold, c.d_theta, asymD, nullptr);
  // beta, dE0 and the directions S = p + beta S_old', D = A + beta D_old
  hipLaunchKernelGGL(k_g_directions, dim3((unsigned)grid_for(2 * band + nn)), dim3(256), 0, c.stream,
                     c.d_cg + 8, c.d_cg, wgb, asymD, c.d_bandv + nb, nb, gs, 2 * band, dbl(c.d_p),
                     dbl(c.d_w1), dbl(c.d_S), nn, c.d_A, c.d_Dold, c.d_D);
  ROKS_HIP(hipGetLastError());
  gemm_wdot(c, nb, nb, K, dbl(c.d_S), K, dbl(c.d_S), K, c.d_SS, nb, 1.0, 0.0, true);
  if (!expm_in_lds(c)) matrix_norm1(c, c.d_D, nb, gs + gNormD);
  if (c.nproj > 0) {
    // <beta|S> once per search, and the projections of psi kept as P0 (the
    // trials write d_P)
    proj_wdot(c, nb, dbl(c.d_S), K, c.d_PS, nb);
    copy_dev(c, c.d_P0, c.d_P, (size_t)c.nproj * nb * sizeof(double));
  }
  // the two trials of the line search's first attempt (reading R7)
  graph_trial(c, c.d_trial[0], c.d_M, c.d_U, true, gEt, gOkT);
  graph_trial(c, c.d_trial[1], c.d_Mkeep, c.d_Ukeep, false, gEts, gOkTs);
  // the choice, and the copies that depend on it: psi (and, for the first
  // trial, its potentials, projections and band energies; the second
  // trial's are in place) when accepted, M and U of the trial kept into
  // scratch
  const size_t ng = (size_t)c.ntot;
  SegList a;
  a.add(c.d_trial[0], c.d_trial[1], c.d_psi, band * sizeof(double2), kAccepted);
  a.add(c.d_gvsh, c.d_vsh, c.d_vsh, c.nsocc * ng * sizeof(double), kFirstTaken);
  a.add(c.d_gvloc, c.d_vloc, c.d_vloc, 2 * c.nconf * ng * sizeof(double), kFirstTaken);
  if (c.prec == ROKS_FP32) {
    a.add(c.d_gvsh32, c.d_vsh32, c.d_vsh32, c.nsocc * ng * sizeof(float), kFirstTaken);
    a.add(c.d_gvloc32, c.d_vloc32, c.d_vloc32, 2 * c.nconf * ng * sizeof(float), kFirstTaken);
  }
  if (c.nproj > 0) a.add(c.d_gP, c.d_P, c.d_P, (size_t)c.nproj * nb * sizeof(double), kFirstTaken);
  a.add(c.d_gscal + 16, c.d_scal + 16, c.d_scal + 16, 2 * (size_t)nb * sizeof(double), kFirstTaken);
  a.add(c.d_M, c.d_Mkeep, c.d_m3, nn * sizeof(double), kAlways);
  a.add(c.d_U, c.d_Ukeep, c.d_m4, nn * sizeof(double), kAlways);
  hipLaunchKernelGGL(k_g_accept, dim3(a.grid()), dim3(256), 0, c.stream, gs, a.g);
  ROKS_HIP(hipGetLastError());
  // S_old = M^T S and D_old = U^T D U of the trial kept (formed in scratch,
  // copied in only when accepted)
  gemm_expand(c, nb, K, nb, c.d_m3, nb, true, dbl(c.d_S), K, dbl(c.d_trial[0]), K, 1.0, 0.0);
  gemm_small(c, nb, nb, nb, c.d_D, nb, false, c.d_m4, nb, false, c.d_m2, nb, 1.0, 0.0);
  gemm_small(c, nb, nb, nb, c.d_m4, nb, true, c.d_m2, nb, false, c.d_m1, nb, 1.0, 0.0);
  // <psi_new|S_old> = delta M <S|S> M^T (<psi|S> = 0) for the next iteration
  gemm_small(c, nb, nb, nb, c.d_SS, nb, false, c.d_m3, nb, true, c.d_gram, nb, 1.0, 0.0);
  gemm_small(c, nb, nb, nb, c.d_m3, nb, false, c.d_gram, nb, false, c.d_Linv, nb, 1.0, 0.0);
  hipLaunchKernelGGL(k_g_scale, dim3((unsigned)grid_for(nn)), dim3(256), 0, c.stream, nn, c.d_Linv, gs,
                     (int)gDelta);
  ROKS_HIP(hipGetLastError());
  SegList f;
  f.add(c.d_trial[0], c.d_trial[0], c.d_Sold, band * sizeof(double2), kAccepted);
  f.add(c.d_m1, c.d_m1, c.d_Dold, nn * sizeof(double), kAccepted);
  f.add(c.d_Linv, c.d_Linv, c.d_PSold, nn * sizeof(double), kAccepted);
  hipLaunchKernelGGL(k_g_finish, dim3(f.grid()), dim3(256), 0, c.stream, gs, f.g,
                     c.hd_grec + (size_t)step * kRecLen, c.hd_gmirror, kDtMin, kDtMax);
  ROKS_HIP(hipGetLastError());
  c.potentials_valid = false;
}

// ---------------------------------------------------------------------------
// host side: checks, buffers, capture, replay
// ---------------------------------------------------------------------------
namespace {

void graph_check(const Ctx& c) {
  ROKS_CHECK(c.have_orbitals, ROKS_ERR_STATE, "no orbitals set");
  ROKS_CHECK(!c.bf3 && (c.prec == ROKS_FP64 || c.prec == ROKS_FP32), ROKS_ERR_STATE,
             "graph mode runs in the FP64 or FP32 tier");
  ROKS_CHECK(c.exx == 0.0 && !c.has_q && c.rec_max == 0, ROKS_ERR_STATE,
             "graph mode excludes exact exchange, overlap coefficients and recording");
  ROKS_CHECK(!(c.flags & (ROKS_FLAG_CANONICALIZE | ROKS_FLAG_AUTOTUNE)), ROKS_ERR_STATE,
             "graph mode excludes canonicalisation and autotuning");
}

void graph_buffers(Ctx& c, int k) {
  const int nb = c.nb;
  if (!c.d_gstate) {
    c.d_gstate = dalloc<double>(c, gNSlots + nb + 8);
    std::vector<double> focc((size_t)c.nconf * nb);
    for (int L = 0; L < c.nconf; ++L)
      for (int n = 0; n < nb; ++n)
        focc[(size_t)L * nb + n] =
            (double)c.occ[(L * 2 + 0) * nb + n] + (double)c.occ[(L * 2 + 1) * nb + n];
    c.d_gfocc = dalloc<double>(c, focc.size());
    c.d_gvsh = dalloc<double>(c, (size_t)c.nsocc * c.ntot);
    c.d_gvloc = dalloc<double>(c, (size_t)2 * c.nconf * c.ntot);
    c.d_gP = dalloc<double>(c, (size_t)std::max(1, c.nproj) * nb);
    c.d_gscal = dalloc<double>(c, 16 + 2 * (size_t)nb);
    c.d_gPSt = dalloc<double>(c, (size_t)std::max(1, c.nproj) * nb);
    ROKS_HIP(hipMemcpyAsync(c.d_gfocc, focc.data(), focc.size() * sizeof(double), hipMemcpyHostToDevice,
                            c.stream));
    ROKS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.h_gmirror), gNSlots * sizeof(double),
                           hipHostMallocMapped | hipHostMallocCoherent));
    ROKS_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c.hd_gmirror), c.h_gmirror, 0));
    ROKS_HIP(hipStreamSynchronize(c.stream));
  }
  if (c.d_vsh32 && !c.d_gvsh32) {
    c.d_gvsh32 = dalloc<float>(c, (size_t)c.nsocc * c.ntot);
    c.d_gvloc32 = dalloc<float>(c, (size_t)2 * c.nconf * c.ntot);
    ROKS_HIP(hipStreamSynchronize(c.stream));
  }
  if (k > c.grec_cap) {
    free_graph(c);  // the records move: capture again
    if (c.h_grec) (void)hipHostFree(c.h_grec);
    c.h_grec = c.hd_grec = nullptr;
    c.grec_cap = 0;
    ROKS_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.h_grec), (size_t)k * kRecLen * sizeof(double),
                           hipHostMallocMapped | hipHostMallocCoherent));
    ROKS_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c.hd_grec), c.h_grec, 0));
    c.grec_cap = k;
  }
}

// the host CG state into the device block; halt: nothing may be committed
void graph_load_state(Ctx& c, bool halt) {
  double s[gNSlots] = {0};
  s[gDt] = c.dt;
  s[gPgOld] = c.pg_old;
  s[gHaveOld] = c.have_old ? 1.0 : 0.0;
  s[gHalt] = halt ? 1.0 : 0.0;
  s[gSince] = c.since_restart;
  s[gPeriod] = c.restart_period;
  ROKS_HIP(hipMemcpyAsync(c.d_gstate, s, sizeof s, hipMemcpyHostToDevice, c.stream));
  if (!c.have_old) {
    // no carried direction: S_old and D_old enter with beta = 0, as zeros
    ROKS_HIP(hipMemsetAsync(c.d_Sold, 0, (size_t)c.nb * c.npw * sizeof(double2), c.stream));
    ROKS_HIP(hipMemsetAsync(c.d_Dold, 0, (size_t)c.nb * c.nb * sizeof(double), c.stream));
  }
  ROKS_HIP(hipStreamSynchronize(c.stream));
}

void* const* current_bufs(const Ctx& c, void* out[5]) {
  out[0] = c.d_psi;
  out[1] = c.d_trial[0];
  out[2] = c.d_trial[1];
  out[3] = c.d_P;
  out[4] = c.d_P0;
  return out;
}

// the graph's buffers are the context's, possibly traded by the host CG
// since: {orbitals, trials} and {P, P0} as sets
bool same_sets(void* const* a, void* const* b) {
  auto in = [](void* p, void* const* set, int n) {
    for (int i = 0; i < n; ++i)
      if (set[i] == p) return true;
    return false;
  };
  for (int i = 0; i < 3; ++i)
    if (!in(a[i], b, 3)) return false;
  for (int i = 3; i < 5; ++i)
    if (!in(a[i], b + 3, 2)) return false;
  return true;
}

// put the orbitals in the buffer the graph reads them from and the pointers
// back in the captured arrangement
void restore_bufs(Ctx& c) {
  void** g = c.graph_bufs;
  if (c.d_psi != g[0])
    ROKS_HIP(hipMemcpyAsync(g[0], c.d_psi, (size_t)c.nb * c.npw * sizeof(double2),
                            hipMemcpyDeviceToDevice, c.stream));
  c.d_psi = static_cast<double2*>(g[0]);
  c.d_trial[0] = static_cast<double2*>(g[1]);
  c.d_trial[1] = static_cast<double2*>(g[2]);
  c.d_P = static_cast<double*>(g[3]);
  c.d_P0 = static_cast<double*>(g[4]);
}

// captures of different contexts (the batch's worker threads) one at a
// time: a capture is made once per context and k, the replays stay
// concurrent
std::mutex g_capture_mu;

void capture(Ctx& c, int k) {
  std::lock_guard<std::mutex> lock(g_capture_mu);
  free_graph(c);
  // one iteration outside the capture that commits nothing: first-use work
  // of every launcher (tables, LDS limits) happens here
  graph_load_state(c, true);
  graph_step(c, 0, false);
  ROKS_HIP(hipStreamSynchronize(c.stream));
  hipStream_t st = nullptr;
  ROKS_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  const hipStream_t own = c.stream;
  const bool timing = c.timing;
  c.stream = st;
  c.timing = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    try {
      for (int i = 0; i < k; ++i) graph_step(c, i, i > 0);
    } catch (...) {
      (void)hipStreamEndCapture(st, &g);
      if (g) (void)hipGraphDestroy(g);
      c.stream = own;
      c.timing = timing;
      (void)hipStreamDestroy(st);
      throw;
    }
    e = hipStreamEndCapture(st, &g);
  }
  c.stream = own;
  c.timing = timing;
  (void)hipStreamDestroy(st);
  ROKS_HIP(e);
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  ROKS_HIP(e);
  c.graph_exec = ex;
  c.graph_k = k;
  c.graph_prec = c.prec;
  c.graph_flags = c.flags;
  c.graph_mlp = c.mlp;
  current_bufs(c, c.graph_bufs);
}

}  // namespace

bool graph_eligible(const Ctx& c) {
  try {
    graph_check(c);
  } catch (const Error&) {
    return false;
  }
  return true;
}

void free_graph(Ctx& c) {
  if (c.graph_exec) (void)hipGraphExecDestroy(c.graph_exec);
  c.graph_exec = nullptr;
  c.graph_k = 0;
}

void free_graph_mode(Ctx& c) {
  free_graph(c);
  for (void* h : {(void*)c.h_gmirror, (void*)c.h_grec})
    if (h) (void)hipHostFree(h);
  c.h_gmirror = c.hd_gmirror = c.h_grec = c.hd_grec = nullptr;
  c.grec_cap = 0;
  c.d_gstate = c.d_gfocc = c.d_gvsh = c.d_gvloc = c.d_gP = c.d_gscal = c.d_gPSt = nullptr;  // freed with the others
  c.d_gvsh32 = c.d_gvloc32 = nullptr;
}

int graph_steps(Ctx& c, int k, roks_step_info* info) {
  ROKS_CHECK(k >= 1 && k <= 1024, ROKS_ERR_ARG, "k must be 1 .. 1024");
  graph_check(c);
  reset_diis(c);  // the kept DIIS iterates do not lead to these orbitals
  graph_buffers(c, k);
  void* cur[5];
  current_bufs(c, cur);
  const bool reuse = c.graph_exec && c.graph_k == k && c.graph_prec == c.prec &&
                     c.graph_flags == c.flags && c.graph_mlp == c.mlp &&
                     same_sets(cur, c.graph_bufs);
  if (reuse)
    restore_bufs(c);
  else
    capture(c, k);
  c.potentials_valid = false;
  graph_load_state(c, false);
  ROKS_HIP(hipGraphLaunch(c.graph_exec, c.stream));
  ROKS_HIP(hipStreamSynchronize(c.stream));
  int acc = 0;
  while (acc < k && c.h_grec[(size_t)acc * kRecLen + 5] != 0.0) ++acc;
  if (info) {
    for (int i = 0; i < k; ++i) {
      const double* r = c.h_grec + (size_t)i * kRecLen;
      roks_step_info s{};
      s.E0 = r[0];
      s.E1 = r[1];
      s.delta = r[2];
      s.beta = r[3];
      s.dE0 = r[4];
      s.stalled = r[5] != 0.0 ? 0 : 1;
      s.norm_gI = r[6];
      s.restarted = r[7] != 0.0 ? 1 : 0;
      s.learned = c.mlp ? 1 : 0;
      s.evaluations = i <= acc ? 2 : 0;
      s.iteration = c.iteration + std::min(i + 1, acc);
      info[i] = s;
    }
  }
  if (acc > 0) {
    const double* m = c.h_gmirror;
    c.dt = m[gDt];
    c.pg_old = m[gPgOld];
    c.have_old = true;
    c.since_restart = (int)m[gSince];
    c.iteration += acc;
    c.psold_iter = c.iteration;  // the last accepted iteration left <psi|S_old>
  }
  c.potentials_valid = false;
  c.T_src = nullptr;  // the replay wrote the column buffer
  return acc;
}

}  // namespace roks
