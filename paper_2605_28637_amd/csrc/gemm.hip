// The band-space inner products C = alpha * A W B^T + beta * C (FP64) with
// a long K: W is the Gamma half-sphere weight (1 for G = 0, 2 otherwise), so
// C_mn is the real inner product <a_m|b_n> of stored bands.  Small outputs
// (the usual nb x nb or nproj x nb) run on the FP64 matrix cores with the
// operands read straight from HBM; K is split over workgroups and the
// partials are summed in a fixed order (bitwise reproducible); the split
// count comes from a heuristic or, with ROKS_FLAG_AUTOTUNE, from timing
// candidates once per shape.  Products with M, N >= 128 are compute-bound and
// go to the LDS-tiled product of tile_gemm.hip instead.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "roks_internal.h"

namespace roks {

namespace {

// --------------------------------------------------------------------------
// FP64 MFMA 16x16x4, one double per lane per operand: lane l gives the A
// operand's row l%16 and the B operand's column l%16, both at depth slot
// l/16; its 4 accumulator values are rows l/16 + 4r of column l%16.  A and B
// only have to agree on which k each depth slot holds, so each lane reads 4
// consecutive k of its own band: no LDS staging, 16-byte loads.
// --------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kWdotGroup = 16;                  // k columns per wave and MFMA round
constexpr int kWdotStep = 2 * 4 * kWdotGroup;   // per workgroup iteration: 2 rounds x 4 waves

// 4 consecutive k of one band row (zeros beyond the row count or the chunk)
__device__ inline void load4(const double* __restrict__ p, bool row_ok, int k, int ke, bool vec,
                             double* v) {
  if (vec && row_ok && k + 3 < ke) {
    const double2 v0 = *reinterpret_cast<const double2*>(p);
    const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
    v[0] = v0.x;
    v[1] = v0.y;
    v[2] = v1.x;
    v[3] = v1.y;
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = (row_ok && k + t < ke) ? p[t] : 0.0;
  }
}

// C[m][n] (+)= sum_k w_k A[m][k] B[n][k] over one K chunk (blockIdx.z) for
// an output tile of RB x CB blocks of 16 x 16.  The chunk is cut into groups
// of 16 columns dealt to the 4 waves in turn, two groups per wave and
// iteration with every load issued before the MFMAs; the waves' sums are
// added in LDS in wave order, so the result does not depend on timing.
// direct: C = alpha sum + beta C; else the sum goes to out[z][M][N].
template <int RB, int CB>
__global__ void __launch_bounds__(256) k_wdot_mfma(int M, int N, int K, const double* __restrict__ A,
                                                   int lda, const double* __restrict__ B, int ldb,
                                                   double* __restrict__ out, int ldo, int kchunk,
                                                   int hw, int vec, double alpha, double beta,
                                                   int direct) {
  __shared__ double red[RB * CB * 4 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = (int)blockIdx.x * 16 * RB;
  const int n0 = blockIdx.y * 16 * CB;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int r16 = lane & 15, s = lane >> 4;
  d4 acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int g0 = kb; g0 < ke; g0 += kWdotStep) {
    double a[2][RB][4], b[2][CB][4];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = g0 + (4 * q + wave) * kWdotGroup + 4 * s;
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int row = m0 + 16 * i + r16;
        load4(A + (size_t)row * lda + k, row < M, k, ke, vec != 0, a[q][i]);
        if (hw) {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (k + t >= 2) a[q][i][t] *= 2.0;  // stored-half weight; the G = 0 doubles weigh 1
        }
      }
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int row = n0 + 16 * j + r16;
        load4(B + (size_t)row * ldb + k, row < N, k, ke, vec != 0, b[q][j]);
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < CB; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][i][t], b[q][j][t], acc[i][j], 0, 0, 0);
  }
  for (int w = 1; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[((i * CB + j) * 4 + r) * 64 + lane] = acc[i][j][r];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[i][j][r] += red[((i * CB + j) * 4 + r) * 64 + lane];
    }
    __syncthreads();
  }
  if (wave != 0) return;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + 16 * i + s + 4 * r, n = n0 + 16 * j + r16;
        if (m >= M || n >= N) continue;
        if (direct) {
          double v = alpha * acc[i][j][r];
          if (beta != 0.0) v += beta * out[(size_t)m * ldo + n];
          out[(size_t)m * ldo + n] = v;
        } else {
          out[((size_t)blockIdx.z * M + m) * N + n] = acc[i][j][r];
        }
      }
}

// few splits: one thread per output sums them in order
__global__ void k_splitk_reduce(const double* __restrict__ part, int ks, int M, int N,
                                double* __restrict__ C, int ldc, double alpha, double beta) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (t >= (size_t)M * N) return;
  const int m = (int)(t / N), n = (int)(t - (size_t)m * N);
  double s = 0;
  for (int z = 0; z < ks; ++z) s += part[(size_t)z * M * N + t];
  double v = alpha * s;
  if (beta != 0.0) v += beta * C[(size_t)m * ldc + n];
  C[(size_t)m * ldc + n] = v;
}

// many splits: 16 outputs per workgroup (a 128-byte row piece of every
// split), 64 groups of 16 lanes striding over the splits, the groups' sums
// added in group order
__global__ void __launch_bounds__(1024) k_splitk_reduce16(const double* __restrict__ part, int ks,
                                                          int M, int N, double* __restrict__ C,
                                                          int ldc, double alpha, double beta) {
  __shared__ double red[64][17];
  const size_t mn = (size_t)M * N;
  const int c = threadIdx.x & 15, g = threadIdx.x >> 4;
  const size_t o = blockIdx.x * (size_t)16 + c;
  double s = 0.0;
  if (o < mn) {
#pragma unroll 2
    for (int z = g; z < ks; z += 64) s += part[(size_t)z * mn + o];
  }
  red[g][c] = s;
  __syncthreads();
  if (g == 0 && o < mn) {
    double t = 0.0;
#pragma unroll 8
    for (int q = 0; q < 64; ++q) t += red[q][c];
    const int m = (int)(o / N), n = (int)(o - (size_t)m * N);
    double v = alpha * t;
    if (beta != 0.0) v += beta * C[(size_t)m * ldc + n];
    C[(size_t)m * ldc + n] = v;
  }
}

}  // namespace

namespace {

// blocks of 16 per tile side: the count in 1..cap with the least padding,
// the larger on ties
int tile_blocks(int n16, int cap) {
  int best = 1;
  for (int b = 1; b <= cap; ++b)
    if (cdiv(n16, b) * b <= cdiv(n16, best) * best) best = b;
  return best;
}

template <int RB, int CB>
void launch_wdot_mfma(Ctx& c, dim3 grid, int M, int N, int K, const double* A, int lda, const double* B,
                      int ldb, double* out, int ldo, int kchunk, int hw, int vec, double alpha,
                      double beta, int direct) {
  hipLaunchKernelGGL((k_wdot_mfma<RB, CB>), grid, dim3(256), 0, c.stream, M, N, K, A, lda, B, ldb, out,
                     ldo, kchunk, hw, vec, alpha, beta, direct);
}

using WdotLaunch = void (*)(Ctx&, dim3, int, int, int, const double*, int, const double*, int, double*,
                            int, int, int, int, double, double, int);

const WdotLaunch (&wdot_table())[5][3] {
  static const WdotLaunch t[5][3] = {
      {launch_wdot_mfma<1, 1>, launch_wdot_mfma<1, 2>, launch_wdot_mfma<1, 3>},
      {launch_wdot_mfma<2, 1>, launch_wdot_mfma<2, 2>, launch_wdot_mfma<2, 3>},
      {launch_wdot_mfma<3, 1>, launch_wdot_mfma<3, 2>, launch_wdot_mfma<3, 3>},
      {launch_wdot_mfma<4, 1>, launch_wdot_mfma<4, 2>, launch_wdot_mfma<4, 3>},
      {launch_wdot_mfma<5, 1>, launch_wdot_mfma<5, 2>, launch_wdot_mfma<5, 3>}};
  return t;
}

// the ordered sum of ks partials of a rows x N product into C
void splitk_sum(Ctx& c, int ks, int rows, int N, double* C, int ldc, double alpha, double beta) {
  const size_t mn = (size_t)rows * N;
  if (ks > 16)
    hipLaunchKernelGGL(k_splitk_reduce16, dim3((unsigned)((mn + 15) / 16)), dim3(1024), 0, c.stream,
                       c.d_gemm_part, ks, rows, N, C, ldc, alpha, beta);
  else
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, c.stream,
                       c.d_gemm_part, ks, rows, N, C, ldc, alpha, beta);
  ROKS_HIP(hipGetLastError());
}

// the launches of one split count (ks_req < 0: the LDS-tiled product in
// -ks_req chunks of K): partials then the ordered sum, or one pass
void gemm_wdot_launch(Ctx& c, int M, int N, int K, const double* A, int lda, const double* B,
                      int ldb, double* C, int ldc, double alpha, double beta, bool half_weights,
                      int ks_req) {
  if (ks_req < 0) {
    tile_gemm(c, M, N, K, A, lda, 0, B, ldb, 0, nullptr, 0.0, C, ldc, nullptr, 0, alpha, beta,
              half_weights, -ks_req);
    return;
  }
  const int RB = tile_blocks(cdiv(M, 16), 5), CB = tile_blocks(cdiv(N, 16), 3);
  const WdotLaunch launch = wdot_table()[RB - 1][CB - 1];
  // 16-byte loads need 16-byte aligned rows
  const int vec = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) % 16 == 0 &&
                   lda % 2 == 0 && ldb % 2 == 0)
                      ? 1
                      : 0;
  const int hw = half_weights ? 1 : 0;
  const int kchunk = cdiv(cdiv(K, std::max(1, ks_req)), kWdotStep) * kWdotStep;
  const int ks = cdiv(K, kchunk);
  dim3 grid(cdiv(M, 16 * RB), cdiv(N, 16 * CB), ks);
  if (ks == 1) {
    launch(c, grid, M, N, K, A, lda, B, ldb, C, ldc, kchunk, hw, vec, alpha, beta, 1);
    ROKS_HIP(hipGetLastError());
    return;
  }
  launch(c, grid, M, N, K, A, lda, B, ldb, c.d_gemm_part, N, kchunk, hw, vec, 1.0, 0.0, 0);
  ROKS_HIP(hipGetLastError());
  splitk_sum(c, ks, M, N, C, ldc, alpha, beta);
}

// split counts the partial buffer holds, at most one per workgroup step of K
int max_splits(const Ctx& c, int M, int N, int K) {
  int ks = std::max(1, cdiv(K, kWdotStep));
  while ((size_t)ks * M * N > c.gemm_part_capacity && ks > 1) --ks;
  return ks;
}

// A workgroup reads its K chunk once per tile; the smallest chunk (one step,
// 128 columns) is used until the tiles times chunks reach ~256 workgroups.
int heuristic_splits(const Ctx& c, int M, int N, int K) {
  // compute-bound sizes: the LDS-tiled product, K cut so the tiles fill the GPU
  if (M >= 128 && N >= 128) return -tile_gemm_splits(c, M, N, K);
  const int tiles = cdiv(M, 16 * tile_blocks(cdiv(M, 16), 5)) * cdiv(N, 16 * tile_blocks(cdiv(N, 16), 3));
  const int ks = std::max(1, std::min(cdiv(K, kWdotStep), cdiv(256, tiles)));
  return std::min(ks, max_splits(c, M, N, K));
}

// autotuner: the product kernel and split count of each (M, N, K), timed
// once per process, or read from the cache file named by the environment
// variable ROKS_TUNE_CACHE (choices of the same device architecture and
// compute-unit count only; the file is rewritten, through a temporary file
// and a rename, after every new choice).  Format, one entry per line:
//   {"arch": "gfx950", "cus": 256, "wdot": [
//   [M, N, K, choice],
//   ...]}
// choice > 0: the small-output product split over K in that many chunks;
// choice < 0: the LDS-tiled product in -choice chunks of K.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tuned;
bool g_cache_read = false;

std::string device_tag(const Ctx& c, int* cus) {
  hipDeviceProp_t p;
  ROKS_HIP(hipGetDeviceProperties(&p, c.device));
  *cus = p.multiProcessorCount;
  std::string arch(p.gcnArchName);
  const size_t colon = arch.find(':');
  return colon == std::string::npos ? arch : arch.substr(0, colon);
}

void read_tune_cache(const Ctx& c) {
  g_cache_read = true;
  const char* path = std::getenv("ROKS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int cus = 0;
  const std::string arch = device_tag(c, &cus);
  char line[512];
  bool ok = false;
  if (std::fgets(line, sizeof line, f)) {
    char a[128] = {0};
    int fc = 0;
    ok = std::sscanf(line, " {\"arch\": \"%127[^\"]\", \"cus\": %d", a, &fc) == 2 && arch == a &&
         fc == cus;
  }
  while (ok && std::fgets(line, sizeof line, f)) {
    int M, N, K, v;
    if (std::sscanf(line, " [%d, %d, %d, %d]", &M, &N, &K, &v) == 4 && M > 0 && N > 0 && K > 0 && v != 0)
      g_tuned.emplace(std::make_tuple(M, N, K), v);
  }
  std::fclose(f);
}

void write_tune_cache(const Ctx& c) {
  const char* path = std::getenv("ROKS_TUNE_CACHE");
  if (!path || !*path) return;
  int cus = 0;
  const std::string arch = device_tag(c, &cus);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;  // the cache is an optimisation: an unwritable path only costs retuning
  std::fprintf(f, "{\"arch\": \"%s\", \"cus\": %d, \"wdot\": [\n", arch.c_str(), cus);
  size_t i = 0;
  for (const auto& e : g_tuned)
    std::fprintf(f, "[%d, %d, %d, %d]%s\n", std::get<0>(e.first), std::get<1>(e.first),
                 std::get<2>(e.first), e.second, ++i < g_tuned.size() ? "," : "");
  std::fprintf(f, "]}\n");
  const bool good = std::fclose(f) == 0;
  if (good) std::rename(tmp.c_str(), path);
}

int tuned_splits(Ctx& c, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                 bool half_weights) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (!g_cache_read) read_tune_cache(c);
  const auto key = std::make_tuple(M, N, K);
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) {
    // a cached choice the buffers of this context cannot take is timed again
    const int v = it->second;
    const bool fits = v < 0 ? (size_t)(-v) * M * N <= c.gemm_part_capacity
                            : v <= max_splits(c, M, N, K);
    if (fits) return v;
  }
  const int h = heuristic_splits(c, M, N, K), hi = max_splits(c, M, N, K);
  std::vector<int> cand;
  if (M >= 64 && N >= 64)
    for (int v : {-1, -4, -8, -16, -32, -64})  // the LDS-tiled product in |v| chunks of K
      if ((size_t)(-v) * M * N <= c.gemm_part_capacity) cand.push_back(v);
  const int hh = std::max(1, std::abs(h));
  for (int v : {hh / 4, hh / 2, hh, 2 * hh, 4 * hh, 1, 32, 64})
    if (v >= 1 && v <= hi && std::find(cand.begin(), cand.end(), v) == cand.end()) cand.push_back(v);
  double* scratch = dalloc<double>(c, (size_t)M * N);
  hipEvent_t e0, e1;
  ROKS_HIP(hipEventCreate(&e0));
  ROKS_HIP(hipEventCreate(&e1));
  int best = h;
  float best_ms = 1e30f;
  for (int v : cand) {
    float tmin = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      ROKS_HIP(hipEventRecord(e0, c.stream));
      gemm_wdot_launch(c, M, N, K, A, lda, B, ldb, scratch, N, 1.0, 0.0, half_weights, v);
      ROKS_HIP(hipEventRecord(e1, c.stream));
      ROKS_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      ROKS_HIP(hipEventElapsedTime(&ms, e0, e1));
      tmin = std::min(tmin, ms);
    }
    if (tmin < best_ms) {
      best_ms = tmin;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the timing buffer goes (the stream is idle after the last event)
  for (size_t i = 0; i < c.allocations.size(); ++i)
    if (c.allocations[i].p == scratch) {
      ROKS_HIP(hipFree(scratch));
      c.allocations.erase(c.allocations.begin() + (long)i);
      break;
    }
  g_tuned[key] = best;
  write_tune_cache(c);
  return best;
}

}  // namespace

void gemm_wdot(Ctx& c, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
               double* C, int ldc, double alpha, double beta, bool half_weights) {
  if (M == 0 || N == 0) return;
  // (the autotuner allocates a timing buffer: not inside an allocation-free call)
  const int ks = ((c.flags & ROKS_FLAG_AUTOTUNE) && !c.no_alloc)
                     ? tuned_splits(c, M, N, K, A, lda, B, ldb, half_weights)
                     : heuristic_splits(c, M, N, K);
  KernelTimer kt(c, "gemm_wdot", ((double)M + N) * K * sizeof(double) + (double)M * N * sizeof(double),
                 2.0 * M * N * (double)K);
  gemm_wdot_launch(c, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, half_weights, ks);
}

}  // namespace roks
