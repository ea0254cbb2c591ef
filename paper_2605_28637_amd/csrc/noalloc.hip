// The operator application without any device allocation: the scratch of
// its kernels (the FFT column buffer, the projections <beta|c> and D<beta|c>,
// the split-K partials of the projection product) lives in one file-scope
// device array instead of the context's buffers.  Each GPU the library runs
// on holds its own copy of the array until the process ends; its address on
// a device is taken once, with that device current, when the first context
// of the device is created, and only that address (never the array's name)
// is handed to kernels.
#include <map>
#include <mutex>

#include "roks_internal.h"

namespace roks {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of its scratch

constexpr size_t kAlign = 256;
size_t up256(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// the context's scratch buffers pointed into the static array for one call,
// restored on every exit
struct ScratchScope {
  Ctx& c;
  double2* T;
  double *DP, *part;
  size_t cap;
  ScratchScope(Ctx& ctx)
      : c(ctx), T(ctx.d_T), DP(ctx.d_DP), part(ctx.d_gemm_part), cap(ctx.gemm_part_capacity) {
    c.no_alloc = true;
  }
  ~ScratchScope() {
    c.d_T = T;
    c.d_DP = DP;
    c.d_gemm_part = part;
    c.gemm_part_capacity = cap;
    c.no_alloc = false;
  }
};

}  // namespace

void init_noalloc_scratch(Ctx& c) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(c.device);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    ROKS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    ROKS_CHECK(p != nullptr, ROKS_ERR_HIP, "no device address for the static scratch");
    it = g_scratch_ptr.emplace(c.device, p).first;
  }
  c.d_noalloc = it->second;
}

void apply_noalloc(Ctx& c, const double2* vecs, uint32_t mask, double2* out) {
  ROKS_CHECK(c.d_noalloc, ROKS_ERR_STATE, "the static scratch of this device is not set up");
  ROKS_CHECK(c.exx == 0.0, ROKS_ERR_STATE,
             "roks_apply_h_noalloc_d does not apply exact exchange (its pair potentials need "
             "band-sized buffers)");
  ROKS_CHECK(!c.bf3, ROKS_ERR_STATE,
             "roks_apply_h_noalloc_d runs in the FP64 and FP32 tiers (the BF16x3 products need "
             "band-sized split buffers)");
  ROKS_CHECK(c.have_orbitals && c.potentials_valid, ROKS_ERR_STATE,
             "the potentials of the current orbitals are not formed (roks_energy_gradient or "
             "roks_apply_h first)");
  const int nb = c.nb, K = 2 * c.npw;
  const size_t band = (size_t)nb * c.npw;
  const bool own = vecs == nullptr;
  if (own) vecs = c.d_psi;
  // carve the array: D<beta|c> | <beta|c> | split-K partials | column buffer
  const size_t proj = (size_t)c.nproj * nb * sizeof(double);
  const size_t col_pair =
      (size_t)c.N[2] * c.ncol * (c.prec == ROKS_FP32 ? sizeof(float2) : sizeof(double2));
  const size_t fixed = up256(proj) + (own ? 0 : up256(proj));
  const size_t part_min = own || c.nproj == 0 ? 0 : up256(proj);  // one split at least
  ROKS_CHECK(fixed + part_min + col_pair <= kNoallocScratchBytes, ROKS_ERR_SHAPE,
             "the system's projections and one band pair's column buffer exceed the static "
             "scratch of roks_apply_h_noalloc_d");
  size_t avail = kNoallocScratchBytes - fixed;
  // the column buffer takes as many band pairs as fit beside the minimal
  // partials; the partials whatever is left of that
  const int chunk = (int)std::min<size_t>(c.npairs, (avail - part_min) / col_pair);
  const size_t col_bytes = up256((size_t)chunk * col_pair);
  const size_t part_bytes = avail - col_bytes;
  unsigned char* base = static_cast<unsigned char*>(c.d_noalloc);
  ScratchScope scope(c);
  c.d_DP = reinterpret_cast<double*>(base);
  double* P = own ? c.d_P : reinterpret_cast<double*>(base + up256(proj));
  c.d_gemm_part = reinterpret_cast<double*>(base + fixed);
  c.gemm_part_capacity = part_bytes / sizeof(double);
  c.d_T = reinterpret_cast<double2*>(base + fixed + part_bytes);
  if (c.nproj > 0 && !own)
    gemm_wdot(c, c.nproj, nb, K, reinterpret_cast<const double*>(c.d_B), K,
              reinterpret_cast<const double*>(vecs), K, P, nb, 1.0, 0.0, true);
  // the band pairs chunk by chunk (chunks start at even bands)
  auto local = [&](const void* pot, int npot, const int32_t* potidx, const double* kinw, double2* o) {
    for (int p0 = 0; p0 < c.npairs; p0 += chunk) {
      const int np = std::min(chunk, c.npairs - p0);
      const int b0 = 2 * p0, nv = std::min(nb - b0, 2 * np);
      const double2* in = vecs + (size_t)b0 * c.npw;
      launch_zpass_bwd(c, in, nv, c.d_T, np);
      launch_plane_apply(c, c.d_T, np, pot, npot, potidx + b0, nv, c.d_Qpart, 0);
      launch_zpass_fwd(c, c.d_T, np, in, nv, kinw + b0, o + (size_t)b0 * c.npw);
    }
  };
  auto nonlocal = [&](const double* w, double2* o) {
    if (c.nproj == 0) return;
    launch_apply_D(c, P, w, c.d_DP);
    gemm_expand(c, nb, K, c.nproj, c.d_DP, nb, false, reinterpret_cast<const double*>(c.d_B), K,
                reinterpret_cast<double*>(o), K, 1.0, 1.0);
  };
  if (mask == 0) {
    const void* vsh = c.prec == ROKS_FP32 ? (const void*)c.d_vsh32 : (const void*)c.d_vsh;
    local(vsh, c.nsocc, c.d_potidx, c.d_kinw_shell, out);
    nonlocal(c.d_kinw_shell, out);
    return;
  }
  int idx = 0;
  for (int b = 0; b < 2 * c.nconf; ++b) {
    if (!(mask & (1u << b))) continue;
    double2* o = out + (size_t)idx * band;
    const void* vl = c.prec == ROKS_FP32 ? (const void*)(c.d_vloc32 + (size_t)b * c.ntot)
                                         : (const void*)(c.d_vloc + (size_t)b * c.ntot);
    local(vl, 1, c.d_potidx + nb, c.d_ones, o);
    nonlocal(nullptr, o);
    ++idx;
  }
}

}  // namespace roks
