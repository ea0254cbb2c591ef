// The band-space inner products C = alpha * A W B^T + beta * C (FP64) with
// a long K: W is the Gamma half-sphere weight (1 for G = 0, 2 otherwise), so
// C_mn is the real inner product <a_m|b_n> of stored bands.  K is split over
// workgroups and the partials are summed in a fixed order (bitwise
// reproducible); the split count comes from a heuristic or, with
// ROKS_FLAG_AUTOTUNE, from timing candidates once per shape.  Products with
// M, N >= 128 are compute-bound and go to the rocBLAS DGEMM instead.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include <rocblas/rocblas.h>

#include "roks_internal.h"

namespace roks {

namespace {

// --------------------------------------------------------------------------
// C[m][n] (+)= sum_k w_k A[m][k] B[n][k]: 64 x 64 tile, 16-deep k slices,
// 4 x 4 outputs per thread; blockIdx.z splits K.
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gemm_wdot(int M, int N, int K, const double* __restrict__ A,
                                                   int lda, const double* __restrict__ B, int ldb,
                                                   double* __restrict__ out, int ldo, int kchunk,
                                                   int hw, double alpha, double beta, int direct) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  const int tm = tid >> 4, tn = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  // the next k slice is loaded into registers while the current one is used
  double pa[4], pb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + q * 256;
      const int row = idx >> 4, kk = idx & 15;
      const int k = k0 + kk;
      pa[q] = 0.0;
      pb[q] = 0.0;
      if (k < ke) {
        const double w = (hw && k >= 2) ? 2.0 : 1.0;
        if (m0 + row < M) pa[q] = w * A[(size_t)(m0 + row) * lda + k];
        if (n0 + row < N) pb[q] = B[(size_t)(n0 + row) * ldb + k];
      }
    }
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = tid + q * 256;
      const int row = idx >> 4, kk = idx & 15;
      As[kk][row] = pa[q];
      Bs[kk][row] = pb[q];
    }
    __syncthreads();
    if (k0 + 16 < ke) load(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tm * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + tm * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tn * 4 + j;
      if (n >= N) continue;
      if (direct) {
        double v = alpha * acc[i][j];
        if (beta != 0.0) v += beta * out[(size_t)m * ldo + n];
        out[(size_t)m * ldo + n] = v;
      } else {
        out[((size_t)blockIdx.z * M + m) * N + n] = acc[i][j];
      }
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

// many splits: 64 outputs per workgroup, 16 groups of 64 lanes stride over
// the splits (each split's row read coalesced), groups summed in order in LDS
__global__ void __launch_bounds__(1024) k_splitk_reduce_cols(const double* __restrict__ part, int ks,
                                                             int M, int N, double* __restrict__ C,
                                                             int ldc, double alpha, double beta) {
  __shared__ double red[16][64];
  const size_t mn = (size_t)M * N;
  const size_t o = blockIdx.x * (size_t)64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  double s = 0.0;
  if (o < mn)
    for (int z = g; z < ks; z += 16) s += part[(size_t)z * mn + o];
  red[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && o < mn) {
    double t = 0.0;
    for (int q = 0; q < 16; ++q) t += red[q][threadIdx.x];
    const int m = (int)(o / N), n = (int)(o - (size_t)m * N);
    double v = alpha * t;
    if (beta != 0.0) v += beta * C[(size_t)m * ldc + n];
    C[(size_t)m * ldc + n] = v;
  }
}

// C[m][n] -= a (A[m][0] B[n][0] + A[m][1] B[n][1]): the G = 0 doubles weigh
// 1, not the 2 a library product with doubled alpha gave them
__global__ void k_g0_correction(int M, int N, const double* __restrict__ A, int lda,
                                const double* __restrict__ B, int ldb, double* __restrict__ C,
                                int ldc, double a) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (t >= (size_t)M * N) return;
  const int m = (int)(t / N), n = (int)(t - (size_t)m * N);
  C[(size_t)m * ldc + n] -=
      a * (A[(size_t)m * lda] * B[(size_t)n * ldb] + A[(size_t)m * lda + 1] * B[(size_t)n * ldb + 1]);
}

}  // namespace

namespace {

// C (row-major M x N) = alpha A W B^T + beta C with the rocBLAS DGEMM on the
// column-major views (C^T = B_cm^T A_cm): K is cut into nchunk equal chunks
// (one strided-batched call; the rest of K, if any, in one more call), each
// giving a partial product in d_gemm_part, summed in chunk order with alpha
// doubled (the stored-half weight), then the G = 0 correction.  rocBLAS runs
// without atomics, so the sums are reproducible.
void gemm_wdot_blas(Ctx& c, int M, int N, int K, const double* A, int lda, const double* B,
                    int ldb, double* C, int ldc, double alpha, double beta, bool half_weights,
                    int nchunk) {
  const rocblas_handle h = static_cast<rocblas_handle>(blas_handle(c));
  const double one = 1.0, zero = 0.0;
  const size_t mn = (size_t)M * N;
  nchunk = std::max(1, std::min<int>(nchunk, (int)(c.gemm_part_capacity / mn) - 1));
  const int kc = K / nchunk;
  const int rest = K - kc * nchunk;
  ROKS_CHECK(rocblas_dgemm_strided_batched(h, rocblas_operation_transpose, rocblas_operation_none, N,
                                           M, kc, &one, B, ldb, (rocblas_stride)kc, A, lda,
                                           (rocblas_stride)kc, &zero, c.d_gemm_part, N,
                                           (rocblas_stride)mn, nchunk) == rocblas_status_success,
             ROKS_ERR_HIP, "rocblas_dgemm_strided_batched failed");
  int ks = nchunk;
  if (rest > 0) {
    ROKS_CHECK(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, N, M, rest, &one,
                             B + (size_t)kc * nchunk, ldb, A + (size_t)kc * nchunk, lda, &zero,
                             c.d_gemm_part + (size_t)nchunk * mn, N) == rocblas_status_success,
               ROKS_ERR_HIP, "rocblas_dgemm failed");
    ++ks;
  }
  const double a = half_weights ? 2.0 * alpha : alpha;
  hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, c.stream,
                     c.d_gemm_part, ks, M, N, C, ldc, a, beta);
  ROKS_HIP(hipGetLastError());
  if (half_weights && K >= 2) {
    hipLaunchKernelGGL(k_g0_correction, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, c.stream, M,
                       N, A, lda, B, ldb, C, ldc, alpha);
    ROKS_HIP(hipGetLastError());
  }
}

// the launches of one split count (ks_req < 0: the library DGEMM in -ks_req
// chunks of K): partials then the ordered sum, or one pass
void gemm_wdot_launch(Ctx& c, int M, int N, int K, const double* A, int lda, const double* B,
                      int ldb, double* C, int ldc, double alpha, double beta, bool half_weights,
                      int ks_req) {
  if (ks_req < 0) {
    gemm_wdot_blas(c, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, half_weights, -ks_req);
    return;
  }
  int kchunk = cdiv(cdiv(K, ks_req), 16) * 16;
  const int ks = cdiv(K, kchunk);
  dim3 grid(cdiv(M, 64), cdiv(N, 64), ks);
  if (ks == 1) {
    hipLaunchKernelGGL(k_gemm_wdot, grid, dim3(256), 0, c.stream, M, N, K, A, lda, B, ldb, C, ldc,
                       kchunk, half_weights ? 1 : 0, alpha, beta, 1);
    ROKS_HIP(hipGetLastError());
    return;
  }
  hipLaunchKernelGGL(k_gemm_wdot, grid, dim3(256), 0, c.stream, M, N, K, A, lda, B, ldb, c.d_gemm_part,
                     N, kchunk, half_weights ? 1 : 0, 1.0, 0.0, 0);
  ROKS_HIP(hipGetLastError());
  const size_t mn = (size_t)M * N;
  if (ks > 16)
    hipLaunchKernelGGL(k_splitk_reduce_cols, dim3((unsigned)((mn + 63) / 64)), dim3(1024), 0,
                       c.stream, c.d_gemm_part, ks, M, N, C, ldc, alpha, beta);
  else
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, c.stream,
                       c.d_gemm_part, ks, M, N, C, ldc, alpha, beta);
  ROKS_HIP(hipGetLastError());
}

int max_splits(const Ctx& c, int M, int N, int K) {
  int ks = std::max(1, K / 16);
  while ((size_t)ks * M * N > c.gemm_part_capacity && ks > 1) --ks;
  return ks;
}

// Every k slice costs one global-load latency that one slice of compute
// cannot hide, so small outputs get many workgroups of ~2 slices each
// (several per CU); the split-K partials are summed in a fixed order.
int heuristic_splits(const Ctx& c, int M, int N, int K) {
  const int tiles = cdiv(M, 64) * cdiv(N, 64);
  // compute-bound sizes: the library DGEMM, K cut so ~1 000 tiles fill the GPU
  if (M >= 128 && N >= 128) return -std::max(1, std::min(32, cdiv(1024, tiles)));
  int ks = std::max(1, std::min(2048 / tiles, K / 32));
  return std::min(ks, max_splits(c, M, N, K));
}

// autotuner: the split count of each (M, N, K) timed once per process
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tuned;

int tuned_splits(Ctx& c, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
                 bool half_weights) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const auto key = std::make_tuple(M, N, K);
  auto it = g_tuned.find(key);
  if (it != g_tuned.end()) return it->second;
  const int h = heuristic_splits(c, M, N, K), hi = max_splits(c, M, N, K);
  std::vector<int> cand;
  if (M >= 64 && N >= 64)
    for (int v : {-1, -4, -8, -16, -32})  // the library DGEMM in |v| chunks of K
      if ((size_t)(-v + 1) * M * N <= c.gemm_part_capacity) cand.push_back(v);
  const int hh = std::max(1, std::abs(h));
  for (int v : {hh / 4, hh / 2, hh, 2 * hh, 4 * hh, 1, 64, 128, 256, 512})
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
  g_tuned[key] = best;
  return best;
}

}  // namespace

void gemm_wdot(Ctx& c, int M, int N, int K, const double* A, int lda, const double* B, int ldb,
               double* C, int ldc, double alpha, double beta, bool half_weights) {
  if (M == 0 || N == 0) return;
  const int ks = (c.flags & ROKS_FLAG_AUTOTUNE)
                     ? tuned_splits(c, M, N, K, A, lda, B, ldb, half_weights)
                     : heuristic_splits(c, M, N, K);
  KernelTimer kt(c, "gemm_wdot", ((double)M + N) * K * sizeof(double) + (double)M * N * sizeof(double),
                 2.0 * M * N * (double)K);
  gemm_wdot_launch(c, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, half_weights, ks);
}

}  // namespace roks
