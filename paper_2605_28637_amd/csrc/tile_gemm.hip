// Large band-space contractions on the FP64 matrix cores (gfx950), the
// compute-bound shapes of many bands (the oxide cell, large batch members):
//   C = alpha op(A) op(B) + beta Cin
// with op(A)[m][k] = A[m lda + k] (ALAY 0) or A[k lda + m] (ALAY 1) and
// op(B)[k][n] = B[n ldb + k] (BLAY 0) or B[k ldb + n] (BLAY 1).  The band
// inner products <a_m|b_n> are ALAY 0 / BLAY 0 with the Gamma half-sphere
// weight w_k (1 for the two G = 0 doubles, 2 otherwise) applied to the A
// loads; the expansions Y = alpha M^T X + beta Y are ALAY 1 / BLAY 1.
//
// A workgroup of 512 threads owns a 128 x 128 tile of C and a chunk of K
// (split-K when the tiles alone cannot fill the GPU): per step of 16 k it
// stages the A and B slices in LDS (k-major, so a wave's MFMA operands are
// consecutive doubles), double-buffered with the global loads of the next
// step in registers; the eight waves each hold a 64 x 32 piece as 4 x 2
// blocks of v_mfma_f64_16x16x4 accumulators, two workgroups per CU.  Split-K partials are summed in
// chunk order by a separate pass, so results are reproducible bit for bit.
#include <algorithm>

#include "roks_internal.h"

namespace roks {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 128, kTN = 128, kTK = 16;
constexpr int kTPad = 16;                // LDS row pad (doubles): rows 16 slots apart
constexpr int kTLd = kTM + kTPad;        // LDS row stride
constexpr int kTThreads = 512;
constexpr int kTPer = kTM * kTK / kTThreads;  // doubles of each operand a thread stages

// the 4 doubles of op(X) a thread stages per 16-k step: LAY 0 (k
// contiguous) row r = t / 4, k = 4 (t % 4) .. + 4; LAY 1 (row contiguous)
// k = t / 32, rows 4 (t % 32) .. + 4.
template <int LAY, bool HW, bool SUM>
__device__ __forceinline__ void tile_load(const double* __restrict__ X, const double* __restrict__ X2,
                                          double x2, int ld, int r0, int rows, int k0, int ke,
                                          int vec, double* v) {
  const int t = threadIdx.x;
  if (LAY == 0) {
    const int r = r0 + (t >> 2), kb = k0 + 4 * (t & 3);
    const bool rok = r < rows;
    const double* p = X + (size_t)r * ld + kb;
    if (rok && vec && kb + 3 < ke) {
#pragma unroll
      for (int j = 0; j < 4; j += 2) {
        const double2 a = *reinterpret_cast<const double2*>(p + j);
        v[j] = a.x;
        v[j + 1] = a.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = (rok && kb + j < ke) ? p[j] : 0.0;
    }
    if (HW) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (kb + j >= 2) v[j] *= 2.0;
    }
  } else {
    const int k = k0 + (t >> 5), rb = r0 + 4 * (t & 31);
    const bool kok = k < ke;
    const double* p = X + (size_t)k * ld + rb;
    const double* p2 = SUM ? X2 + (size_t)k * ld + rb : nullptr;
    if (kok && vec && rb + 3 < rows) {
#pragma unroll
      for (int j = 0; j < 4; j += 2) {
        double2 a = *reinterpret_cast<const double2*>(p + j);
        if (SUM) {
          const double2 b = *reinterpret_cast<const double2*>(p2 + j);
          a.x = fma(x2, b.x, a.x);
          a.y = fma(x2, b.y, a.y);
        }
        v[j] = a.x;
        v[j + 1] = a.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool ok = kok && rb + j < rows;
        double a = ok ? p[j] : 0.0;
        if (SUM && ok) a = fma(x2, p2[j], a);
        v[j] = a;
      }
    }
    if (HW && k >= 2) {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] *= 2.0;
    }
  }
}

template <int LAY>
__device__ __forceinline__ void tile_store(double* __restrict__ S, const double* v) {
  const int t = threadIdx.x;
  if (LAY == 0) {
    const int r = t >> 2, kb = 4 * (t & 3);
#pragma unroll
    for (int j = 0; j < 4; ++j) S[(kb + j) * kTLd + r] = v[j];
  } else {
    const int k = t >> 5, rb = 4 * (t & 31);
#pragma unroll
    for (int j = 0; j < 4; ++j) S[k * kTLd + rb + j] = v[j];
  }
}

struct TileOrder {
  int gx;        // m tiles
  int groups;    // K chunks (by_chunk) or column tiles
  int members;   // workgroups per group
  int by_chunk;
};

// the K loop of one workgroup: per step of 16 k the A and B slices staged in
// LDS (double-buffered, the next step's global loads in registers while this
// step's products run); GUARD skips the blocks that vi / vj mark as past the
// matrix
template <int ALAY, int BLAY, bool HW, bool SUM, bool GUARD>
__device__ __forceinline__ void tile_main(const double* __restrict__ A, int lda,
                                          const double* __restrict__ B, const double* __restrict__ B2,
                                          double b2, int ldb, int M, int N, int m0, int n0, int kb,
                                          int ke, int avec, int bvec, int wm, int wn, int r16, int s,
                                          const bool* vi, const bool* vj, double (*As)[kTK * kTLd],
                                          double (*Bs)[kTK * kTLd], d4 (*acc)[2]) {
  double va[kTPer], vb[kTPer];
  int buf = 0;
  if (kb < ke) {
    tile_load<ALAY, HW, false>(A, nullptr, 0.0, lda, m0, M, kb, ke, avec, va);
    tile_load<BLAY, false, SUM>(B, B2, b2, ldb, n0, N, kb, ke, bvec, vb);
    tile_store<ALAY>(As[0], va);
    tile_store<BLAY>(Bs[0], vb);
  }
  __syncthreads();
  for (int k0 = kb; k0 < ke; k0 += kTK) {
    const bool more = k0 + kTK < ke;
    if (more) {
      // the next step's loads in flight while this step's MFMAs run
      tile_load<ALAY, HW, false>(A, nullptr, 0.0, lda, m0, M, k0 + kTK, ke, avec, va);
      tile_load<BLAY, false, SUM>(B, B2, b2, ldb, n0, N, k0 + kTK, ke, bvec, vb);
    }
    const double* as = As[buf];
    const double* bs = Bs[buf];
    // while issuing products a wave runs at raised priority, and the next
    // 4-k slice of its operands is read from LDS before this slice's
    // products (2 % on the band products, 2 % on the expansions)
    __builtin_amdgcn_s_setprio(1);
    double a[4], b[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = as[s * kTLd + wm * 64 + 16 * i + r16];
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = bs[s * kTLd + wn * 32 + 16 * j + r16];
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 4) {
      double an[4], bn[2];
      if (kk + 4 < kTK) {
#pragma unroll
        for (int i = 0; i < 4; ++i) an[i] = as[(kk + 4 + s) * kTLd + wm * 64 + 16 * i + r16];
#pragma unroll
        for (int j = 0; j < 2; ++j) bn[j] = bs[(kk + 4 + s) * kTLd + wn * 32 + 16 * j + r16];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (!GUARD || (vi[i] && vj[j]))
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      if (kk + 4 < kTK) {
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = an[i];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = bn[j];
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if (more) {
      tile_store<ALAY>(As[buf ^ 1], va);
      tile_store<BLAY>(Bs[buf ^ 1], vb);
    }
    __syncthreads();
    buf ^= 1;
  }
}

// DIRECT: C = alpha sum + beta Cin; else the chunk's sum to part[z][M][N]
template <int ALAY, int BLAY, bool HW, bool SUM>
__global__ void __launch_bounds__(kTThreads, 2) k_tile_gemm(
    int M, int N, int K, const double* __restrict__ A, int lda, const double* __restrict__ B,
    const double* __restrict__ B2, double b2, int ldb, double* __restrict__ C, int ldc,
    const double* __restrict__ Cin, int ldcin, double alpha, double beta, int kchunk, int direct,
    int avec, int bvec, double* __restrict__ part, TileOrder ord) {
  __shared__ double As[2][kTK * kTLd];
  __shared__ double Bs[2][kTK * kTLd];
  // XCD-aware order: workgroup L runs on XCD L % 8 (round-robin dispatch);
  // the workgroups sharing operand slices (one K chunk: all tiles; no split:
  // all m tiles of one column tile) form a group, and each group is placed
  // on one XCD so its L2 serves the re-reads
  const int L = blockIdx.x;
  const int s8 = L >> 3;
  const int g = (L & 7) + 8 * (s8 / ord.members), mem = s8 % ord.members;
  if (g >= ord.groups) return;
  int tx, ty, tz;
  if (ord.by_chunk) {
    tz = g;
    tx = mem % ord.gx;
    ty = mem / ord.gx;
  } else {
    tz = 0;
    ty = g;
    tx = mem;
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 2, wn = wave & 3;  // 2 x 4 waves of 64 x 32
  const int m0 = tx * kTM, n0 = ty * kTN;
  const int kb = tz * kchunk, ke = min(K, kb + kchunk);
  const int r16 = lane & 15, s = lane >> 4;
  d4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  // interior tiles run the plain loop; edge tiles skip the 16 x 16 blocks
  // wholly past M or N (the test is uniform over the wave, so the matrix
  // cores go to other waves)
  bool vi[4], vj[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) vi[i] = m0 + wm * 64 + 16 * i < M;
#pragma unroll
  for (int j = 0; j < 2; ++j) vj[j] = n0 + wn * 32 + 16 * j < N;
  if (vi[3] && vj[1])
    tile_main<ALAY, BLAY, HW, SUM, false>(A, lda, B, B2, b2, ldb, M, N, m0, n0, kb, ke, avec, bvec, wm,
                                          wn, r16, s, vi, vj, As, Bs, acc);
  else
    tile_main<ALAY, BLAY, HW, SUM, true>(A, lda, B, B2, b2, ldb, M, N, m0, n0, kb, ke, avec, bvec, wm,
                                         wn, r16, s, vi, vj, As, Bs, acc);
  // accumulator r of lane l in block (i, j): row 16 i + l/16 + 4 r, column 16 j + l%16
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + 16 * i + s + 4 * r;
        const int n = n0 + wn * 32 + 16 * j + r16;
        if (m >= M || n >= N) continue;
        if (direct) {
          double v = alpha * acc[i][j][r];
          if (beta != 0.0) v += beta * Cin[(size_t)m * ldcin + n];
          C[(size_t)m * ldc + n] = v;
        } else {
          part[((size_t)tz * M + m) * N + n] = acc[i][j][r];
        }
      }
}

// C = alpha sum_z part[z] + beta Cin, one thread per output summing the
// chunks in order
__global__ void __launch_bounds__(256) k_tile_reduce(const double* __restrict__ part, int ks, int M,
                                                     int N, double* __restrict__ C, int ldc,
                                                     const double* __restrict__ Cin, int ldcin,
                                                     double alpha, double beta) {
  const size_t mn = (size_t)M * N;
  const size_t o = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (o >= mn) return;
  double sum = 0.0;
  for (int z = 0; z < ks; ++z) sum += part[(size_t)z * mn + o];
  const int m = (int)(o / N), n = (int)(o - (size_t)m * N);
  double v = alpha * sum;
  if (beta != 0.0) v += beta * Cin[(size_t)m * ldcin + n];
  C[(size_t)m * ldc + n] = v;
}

template <int ALAY, int BLAY, bool HW, bool SUM>
void launch_tile(Ctx& c, dim3 grid, int M, int N, int K, const double* A, int lda, const double* B,
                 const double* B2, double b2, int ldb, double* C, int ldc, const double* Cin, int ldcin,
                 double alpha, double beta, int kchunk, int direct, int avec, int bvec, double* part) {
  TileOrder ord;
  ord.gx = (int)grid.x;
  ord.by_chunk = grid.z > 1 ? 1 : 0;
  ord.groups = ord.by_chunk ? (int)grid.z : (int)grid.y;
  ord.members = ord.by_chunk ? (int)(grid.x * grid.y) : (int)grid.x;
  const unsigned nwg = 8u * (unsigned)cdiv(ord.groups, 8) * (unsigned)ord.members;
  hipLaunchKernelGGL((k_tile_gemm<ALAY, BLAY, HW, SUM>), dim3(nwg), dim3(kTThreads), 0, c.stream, M,
                     N, K, A, lda, B, B2, b2, ldb, C, ldc, Cin, ldcin, alpha, beta, kchunk, direct, avec,
                     bvec, part, ord);
}

bool aligned16(const void* p, int ld) {
  return (reinterpret_cast<uintptr_t>(p) % 16 == 0) && (ld % 2 == 0);
}

}  // namespace

// The split count: enough (tile, chunk) workgroups for one round over the
// device's CUs at two per CU, each chunk at least 64 k (four steps), a
// multiple of 8 chunks beyond 8, within the partial buffer.
int tile_gemm_splits(const Ctx& c, int M, int N, int K) {
  const int tiles = cdiv(M, kTM) * cdiv(N, kTN);
  // one resident round (two workgroups per CU): a chunk's workgroups then
  // run together on their XCD and read its operand slices from HBM once (a
  // chunk split over two rounds reads them twice)
  int ks = std::max(1, std::min(cdiv(512, tiles), cdiv(K, 64)));
  // whole rounds of the 8 XCDs (one chunk's workgroups share an XCD)
  if (ks > 8) ks = ks / 8 * 8;
  while (ks > 1 && (size_t)ks * M * N > c.gemm_part_capacity) --ks;
  return ks;
}

void tile_gemm(Ctx& c, int M, int N, int K, const double* A, int lda, int alay, const double* B,
               int ldb, int blay, const double* B2, double b2, double* C, int ldc, const double* Cin,
               int ldcin, double alpha, double beta, bool half_weights, int ks) {
  if (M == 0 || N == 0) return;
  ROKS_CHECK(!(half_weights && B2), ROKS_ERR_ARG, "weighted products take one B operand");
  if (!Cin) {
    Cin = C;
    ldcin = ldc;
  }
  if (ks <= 0) ks = tile_gemm_splits(c, M, N, K);
  const int kchunk = cdiv(cdiv(K, ks), kTK) * kTK;
  ks = std::max(1, cdiv(K, kchunk));
  const int avec = aligned16(A, lda) ? 1 : 0;
  const int bvec = aligned16(B, ldb) && (!B2 || aligned16(B2, ldb)) ? 1 : 0;
  dim3 grid(cdiv(M, kTM), cdiv(N, kTN), ks);
  const int direct = ks == 1 ? 1 : 0;
  double* part = direct ? nullptr : c.d_gemm_part;
  ROKS_CHECK(direct || (size_t)ks * M * N <= c.gemm_part_capacity, ROKS_ERR_SHAPE,
             "split-K partials exceed their buffer");
#define ROKS_TILE(AL, BL, HWV, SUMV)                                                                \
  launch_tile<AL, BL, HWV, SUMV>(c, grid, M, N, K, A, lda, B, B2, b2, ldb, C, ldc, Cin, ldcin, alpha, \
                                 beta, kchunk, direct, avec, bvec, part)
  if (half_weights) {
    ROKS_CHECK(alay == 0 && blay == 0, ROKS_ERR_ARG, "weighted products are inner products");
    ROKS_TILE(0, 0, true, false);
  } else if (B2) {
    ROKS_CHECK(blay == 1, ROKS_ERR_ARG, "the summed operand is an expansion's band array");
    if (alay == 0) ROKS_TILE(0, 1, false, true);
    else ROKS_TILE(1, 1, false, true);
  } else if (alay == 0 && blay == 0) {
    ROKS_TILE(0, 0, false, false);
  } else if (alay == 0) {
    ROKS_TILE(0, 1, false, false);
  } else if (blay == 0) {
    ROKS_TILE(1, 0, false, false);
  } else {
    ROKS_TILE(1, 1, false, false);
  }
#undef ROKS_TILE
  ROKS_HIP(hipGetLastError());
  if (!direct) {
    const size_t mn = (size_t)M * N;
    hipLaunchKernelGGL(k_tile_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, c.stream,
                       c.d_gemm_part, ks, M, N, C, ldc, Cin, ldcin, alpha, beta);
    ROKS_HIP(hipGetLastError());
  }
}

void launch_tile_reduce(Ctx& c, int ks, int M, int N, double* C, int ldc, const double* Cin, int ldcin,
                        double alpha, double beta) {
  const size_t mn = (size_t)M * N;
  if (mn == 0) return;
  hipLaunchKernelGGL(k_tile_reduce, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, c.stream, c.d_gemm_part,
                     ks, M, N, C, ldc, Cin, ldcin, alpha, beta);
  ROKS_HIP(hipGetLastError());
}

}  // namespace roks
