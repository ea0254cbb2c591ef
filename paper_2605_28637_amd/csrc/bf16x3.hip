// The BF16x3 tier of the projector contractions (ROKS_FP32_BF16X3).
//
// The products with the projector table -- <beta_p|X> (the projections of
// the separable nonlocal potential, Sec. II A), the expansion
// sum_p (D P)_pn beta_p, and the force field sum_n w_n (D P)_pn psi_n of
// Eq. force_hf's nonlocal part -- run on the
// BF16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32 accumulation and a
// split-precision correction.  Each FP64 operand x is split once into
// hi = bf16(x) and lo = bf16(x - hi), so |x - hi - lo| <= 2^-16 |x|; a
// product keeps the three terms lo.hi + hi.lo + hi.hi, each exact in FP32,
// and drops lo.lo.  K chunks of at most 4096 terms accumulate in FP32; the
// chunks are added in FP64 in a fixed order.  Error of one inner product:
// at most (3 2^-16 + 4096 2^-24) sum_k |a_k b_k|.
//
// The split is a pass of its own, not part of the product's staging: the
// projector table is split whenever the projectors are formed, in both
// orientations (projector rows for the projections, coefficient rows for the
// expansion, so both products read k-contiguous rows), and the band side
// once per product.  A split operand is two BF16 arrays (hi, lo) of rows
// whose length is a multiple of 64, zero beyond the data.
#include "roks_internal.h"

namespace roks {

namespace {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kQM = 128, kQN = 128;  // output tile
constexpr int kQK = 64;              // k per step (two MFMA depths)
constexpr int kQLd = kQK + 8;        // LDS row (bf16): 144 bytes, conflict-free fragment reads
constexpr int kQThreads = 512;       // 8 waves of 64 x 32 outputs
constexpr int kQChunk = 4096;        // longest FP32 accumulation
// accumulator r of lane l of a 16 x 16 FP32 block holds row 4 (l / 16) + r,
// column l % 16
constexpr bool kRowsConsecutive = true;

int split_ld(int k) { return cdiv(k, 64) * 64; }

__device__ __forceinline__ void split_one(double x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)(float)x;
  lo = (__bf16)(float)(x - (double)(float)hi);
}

// rows of X (nrows x K, leading dimension ldx) split into hi / lo rows of
// length ldo, 8 consecutive k per thread.  mode 0: as they are; 1: with the
// Gamma-point weights (2 beyond the first two reals, the G = 0 coefficient)
__global__ void __launch_bounds__(256) k_split_rows(const double* __restrict__ X, int ldx, int nrows,
                                                    int K, int ldo, int mode, int vec,
                                                    __bf16* __restrict__ hi, __bf16* __restrict__ lo) {
  const int segs = ldo >> 3;
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)nrows * segs) return;
  const int r = (int)(i / segs), k0 = 8 * (int)(i - (size_t)r * segs);
  const double* x = X + (size_t)r * ldx + k0;
  double v[8];
  if (vec && k0 + 8 <= K) {
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
      const double2 a = *reinterpret_cast<const double2*>(x + j);
      v[j] = a.x;
      v[j + 1] = a.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = k0 + j < K ? x[j] : 0.0;
  }
  if (mode == 1) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k0 + j >= 2) v[j] *= 2.0;
  }
  bf8v h, l;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    __bf16 a, b;
    split_one(v[j], a, b);
    h[j] = a;
    l[j] = b;
  }
  *reinterpret_cast<bf8v*>(hi + (size_t)r * ldo + k0) = h;
  *reinterpret_cast<bf8v*>(lo + (size_t)r * ldo + k0) = l;
}

// columns of X (krows x ncols, leading dimension ldx) split into hi / lo rows
// of length ldo (row n holds X[0..krows)[n], then zeros), through a 64 x 64
// LDS tile: coalesced reads along n, 16-byte writes along k
__global__ void __launch_bounds__(256) k_split_cols(const double* __restrict__ X, int ldx, int krows,
                                                    int ncols, int ldo, __bf16* __restrict__ hi,
                                                    __bf16* __restrict__ lo) {
  __shared__ double T[64][65];
  const int k0 = blockIdx.x * 64, n0 = blockIdx.y * 64, t = threadIdx.x;
  for (int e = t; e < 64 * 64; e += 256) {
    const int kk = e >> 6, nn = e & 63, k = k0 + kk, n = n0 + nn;
    T[kk][nn] = (k < krows && n < ncols) ? X[(size_t)k * ldx + n] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < 64 * 8; e += 256) {
    const int nn = e >> 3, s = e & 7, n = n0 + nn;
    if (n >= ncols) continue;
    bf8v h, l;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      __bf16 a, b;
      split_one(T[8 * s + j][nn], a, b);
      h[j] = a;
      l[j] = b;
    }
    *reinterpret_cast<bf8v*>(hi + (size_t)n * ldo + k0 + 8 * s) = h;
    *reinterpret_cast<bf8v*>(lo + (size_t)n * ldo + k0 + 8 * s) = l;
  }
}

struct QOrder {
  int gx;       // m tiles
  int groups;   // K chunks (by_chunk) or column tiles
  int members;  // workgroups per group
  int by_chunk;
};

// C (M x N) = alpha sum_k A[m][k] B[n][k] + beta Cin over one K chunk of the
// split operands (rows of lda / ldb bf16, K padded with zeros to a multiple
// of 64), or the chunk's sum to part[z][M][N].  Rows beyond M / N are read
// clamped and their results dropped.  Staging: every thread moves one
// 16-byte segment of two rows of each of the four arrays per step, through
// registers (the next step's loads are in flight while the current one
// computes); one LDS copy, two workgroups (four waves per SIMD) per CU.
__global__ void __launch_bounds__(kQThreads, 4) k_bf3_nt(
    int M, int N, const __bf16* __restrict__ Ah, const __bf16* __restrict__ Al, int lda,
    const __bf16* __restrict__ Bh, const __bf16* __restrict__ Bl, int ldb, int Kp,
    double* __restrict__ C, int ldc, const double* __restrict__ Cin, int ldcin, double alpha,
    double beta, int kchunk, int direct, double* __restrict__ part, QOrder ord) {
  __shared__ __attribute__((aligned(16))) __bf16 S[4][kQM * kQLd];  // Ah Al Bh Bl
  // XCD-aware order: workgroup L runs on XCD L % 8; the workgroups that share
  // operand rows (one K chunk, or the m tiles of one column tile) are one
  // group, placed on one XCD so its L2 serves the re-reads
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
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;
  const int m0 = tx * kQM, n0 = ty * kQN;
  const int kb = tz * kchunk, ke = min(Kp, kb + kchunk);
  const int r16 = lane & 15, s = lane >> 4;
  // staging rows sr and sr + 64, segment sk
  const int sr = t >> 3, sk = 8 * (t & 7);
  const size_t a0 = (size_t)min(m0 + sr, M - 1) * lda + sk, a1 = (size_t)min(m0 + sr + 64, M - 1) * lda + sk;
  const size_t b0 = (size_t)min(n0 + sr, N - 1) * ldb + sk, b1 = (size_t)min(n0 + sr + 64, N - 1) * ldb + sk;
  const int l0 = sr * kQLd + sk, l1 = (sr + 64) * kQLd + sk;
  const __bf16 *pah0 = Ah + a0, *pah1 = Ah + a1, *pal0 = Al + a0, *pal1 = Al + a1;
  const __bf16 *pbh0 = Bh + b0, *pbh1 = Bh + b1, *pbl0 = Bl + b0, *pbl1 = Bl + b1;
  uint4 s0, s1, s2, s3, s4, s5, s6, s7;
#define ROKS_BF3_LOAD(k)                                  \
  s0 = *reinterpret_cast<const uint4*>(pah0 + (k));       \
  s1 = *reinterpret_cast<const uint4*>(pah1 + (k));       \
  s2 = *reinterpret_cast<const uint4*>(pal0 + (k));       \
  s3 = *reinterpret_cast<const uint4*>(pal1 + (k));       \
  s4 = *reinterpret_cast<const uint4*>(pbh0 + (k));       \
  s5 = *reinterpret_cast<const uint4*>(pbh1 + (k));       \
  s6 = *reinterpret_cast<const uint4*>(pbl0 + (k));       \
  s7 = *reinterpret_cast<const uint4*>(pbl1 + (k))
  f4v acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
  if (kb < ke) {
    ROKS_BF3_LOAD(kb);
  }
  for (int k0 = kb; k0 < ke; k0 += kQK) {
    *reinterpret_cast<uint4*>(&S[0][l0]) = s0;
    *reinterpret_cast<uint4*>(&S[0][l1]) = s1;
    *reinterpret_cast<uint4*>(&S[1][l0]) = s2;
    *reinterpret_cast<uint4*>(&S[1][l1]) = s3;
    *reinterpret_cast<uint4*>(&S[2][l0]) = s4;
    *reinterpret_cast<uint4*>(&S[2][l1]) = s5;
    *reinterpret_cast<uint4*>(&S[3][l0]) = s6;
    *reinterpret_cast<uint4*>(&S[3][l1]) = s7;
    __syncthreads();
    if (k0 + kQK < ke) {
      ROKS_BF3_LOAD(k0 + kQK);
    }
#pragma unroll
    for (int kk = 0; kk < kQK; kk += 32) {
      bf8v ah[4], al[4], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = (wm * 64 + 16 * i + r16) * kQLd + kk + 8 * s;
        ah[i] = *reinterpret_cast<const bf8v*>(&S[0][o]);
        al[i] = *reinterpret_cast<const bf8v*>(&S[1][o]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int o = (wn * 32 + 16 * j + r16) * kQLd + kk + 8 * s;
        bh[j] = *reinterpret_cast<const bf8v*>(&S[2][o]);
        bl[j] = *reinterpret_cast<const bf8v*>(&S[3][o]);
      }
      // the small terms first; eight independent blocks between dependent MFMAs
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = kRowsConsecutive ? 4 * s + r : s + 4 * r;
        const int m = m0 + wm * 64 + 16 * i + row;
        const int n = n0 + wn * 32 + 16 * j + r16;
        if (m >= M || n >= N) continue;
        const double v = (double)acc[i][j][r];
        if (direct) {
          double o = alpha * v;
          if (beta != 0.0) o += beta * Cin[(size_t)m * ldcin + n];
          C[(size_t)m * ldc + n] = o;
        } else {
          part[((size_t)tz * M + m) * N + n] = v;
        }
      }
}

#undef ROKS_BF3_LOAD

__bf16* bf(uint16_t* p) { return reinterpret_cast<__bf16*>(p); }

void split_rows(Ctx& c, const double* X, int ldx, int nrows, int K, int ldo, int mode, uint16_t* hi,
                uint16_t* lo) {
  const size_t n = (size_t)nrows * (ldo / 8);
  if (n == 0) return;
  const int vec = (reinterpret_cast<uintptr_t>(X) % 16 == 0 && ldx % 2 == 0) ? 1 : 0;
  hipLaunchKernelGGL(k_split_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c.stream, X, ldx,
                     nrows, K, ldo, mode, vec, bf(hi), bf(lo));
  ROKS_HIP(hipGetLastError());
}

void split_cols(Ctx& c, const double* X, int ldx, int krows, int ncols, int ldo, uint16_t* hi,
                uint16_t* lo) {
  if (ncols == 0) return;
  hipLaunchKernelGGL(k_split_cols, dim3(ldo / 64, cdiv(ncols, 64)), dim3(256), 0, c.stream, X, ldx, krows,
                     ncols, ldo, bf(hi), bf(lo));
  ROKS_HIP(hipGetLastError());
}

// C = alpha A B^T + beta Cin over split operands (K padded to Kp).  Split K
// only when asked (the long inner dimension of the projections); chunks of at
// most 4096 k either way.  Where the partials buffer cannot hold all chunks,
// K is taken in ranges, each range's sum added to C in FP64 in order.
void product(Ctx& c, int M, int N, int Kp, const uint16_t* Ah, const uint16_t* Al, int lda,
             const uint16_t* Bh, const uint16_t* Bl, int ldb, double* C, int ldc, const double* Cin,
             int ldcin, double alpha, double beta, bool split) {
  if (M == 0 || N == 0 || Kp == 0) return;
  const int tiles = cdiv(M, kQM) * cdiv(N, kQN);
  const int steps = Kp / kQK;
  int ks = 1;
  if (split) {
    // one resident round of the chip (two workgroups per CU), whole rounds
    // of the 8 XCDs: a chunk's workgroups run together on one XCD and read
    // its operand slices from HBM once
    ks = std::max(1, std::min(steps, cdiv(512, tiles)));
    if (ks > 8) ks = ks / 8 * 8;
  }
  ks = std::max(ks, cdiv(Kp, kQChunk));
  const int kchunk = cdiv(steps, ks) * kQK;  // <= kQChunk
  ks = cdiv(Kp, kchunk);
  const int ks_cap = (int)std::min<size_t>(ks, std::max<size_t>(1, c.gemm_part_capacity / ((size_t)M * N)));
  if (!Cin) {
    Cin = C;
    ldcin = ldc;
  }
  for (int k0 = 0, pass = 0; k0 < Kp; k0 += ks_cap * kchunk, ++pass) {
    const int klen = std::min(Kp - k0, ks_cap * kchunk);
    const int kr = cdiv(klen, kchunk);
    const int direct = kr == 1 ? 1 : 0;
    const double* cin = pass == 0 ? Cin : C;
    const int ldi = pass == 0 ? ldcin : ldc;
    const double bet = pass == 0 ? beta : 1.0;
    QOrder ord;
    ord.gx = cdiv(M, kQM);
    ord.by_chunk = kr > 1 ? 1 : 0;
    ord.groups = ord.by_chunk ? kr : cdiv(N, kQN);
    ord.members = ord.by_chunk ? tiles : ord.gx;
    const unsigned nwg = 8u * (unsigned)cdiv(ord.groups, 8) * (unsigned)ord.members;
    hipLaunchKernelGGL(k_bf3_nt, dim3(nwg), dim3(kQThreads), 0, c.stream, M, N,
                       reinterpret_cast<const __bf16*>(Ah + k0), reinterpret_cast<const __bf16*>(Al + k0),
                       lda, reinterpret_cast<const __bf16*>(Bh + k0),
                       reinterpret_cast<const __bf16*>(Bl + k0), ldb, klen, C, ldc, cin, ldi, alpha, bet,
                       kchunk, direct, direct ? nullptr : c.d_gemm_part, ord);
    ROKS_HIP(hipGetLastError());
    if (!direct) launch_tile_reduce(c, kr, M, N, C, ldc, cin, ldi, alpha, bet);
  }
}

// the split projector table (both orientations) and the band-side buffers,
// allocated on first use; the table is split again after the projectors
// are formed anew
void ensure_tables(Ctx& c) {
  const int K = 2 * c.npw, Kp = split_ld(K), npp = split_ld(c.nproj);
  if (!c.d_bsplit) {
    ROKS_CHECK(!c.no_alloc, ROKS_ERR_STATE, "the BF16x3 tables are not formed");
    c.d_bsplit = dalloc<uint16_t>(c, 2 * (size_t)c.nproj * Kp);
    c.d_bsplit_t = dalloc<uint16_t>(c, 2 * (size_t)K * npp);
    c.d_xsplit = dalloc<uint16_t>(c, 2 * (size_t)c.nb * std::max(Kp, npp));
    c.bsplit_valid = false;
  }
  if (c.bsplit_valid) return;
  const double* B = reinterpret_cast<const double*>(c.d_B);
  split_rows(c, B, K, c.nproj, K, Kp, 0, c.d_bsplit, c.d_bsplit + (size_t)c.nproj * Kp);
  split_cols(c, B, K, c.nproj, K, npp, c.d_bsplit_t, c.d_bsplit_t + (size_t)K * npp);
  c.bsplit_valid = true;
}

}  // namespace

void proj_wdot(Ctx& c, int nrows, const double* X, int ldx, double* C, int ldc) {
  const int K = 2 * c.npw;
  if (c.nproj == 0 || nrows == 0) return;
  if (!c.bf3) {
    gemm_wdot(c, c.nproj, nrows, K, reinterpret_cast<const double*>(c.d_B), K, X, ldx, C, ldc, 1.0, 0.0,
              true);
    return;
  }
  ROKS_CHECK(nrows <= c.nb, ROKS_ERR_ARG, "more rows than bands");
  ensure_tables(c);
  const int Kp = split_ld(K);
  // algorithmic work: the split table (4 bytes an entry), X in FP64, C; the
  // three BF16 products
  KernelTimer kt(c, "proj_bf3", (double)c.nproj * Kp * 4.0 + (double)nrows * K * 8.0 + (double)c.nproj * nrows * 8.0,
                 6.0 * c.nproj * (double)nrows * K);
  uint16_t* xh = c.d_xsplit;
  uint16_t* xl = xh + (size_t)c.nb * Kp;
  split_rows(c, X, ldx, nrows, K, Kp, 1, xh, xl);
  product(c, c.nproj, nrows, Kp, c.d_bsplit, c.d_bsplit + (size_t)c.nproj * Kp, Kp, xh, xl, Kp, C, ldc,
          nullptr, 0, 1.0, 0.0, true);
}

void proj_field(Ctx& c, const double* DPw, int lddp, const double* X, int ldx, double* Phi) {
  const int K = 2 * c.npw, nb = c.nb;
  if (c.nproj == 0) return;
  if (!c.bf3) {
    gemm_expand(c, c.nproj, K, nb, DPw, lddp, true, X, ldx, Phi, K, 1.0, 0.0);
    return;
  }
  // Phi[p][k] = sum_n DPw[p][n] X[n][k]: rows of DPw and of X^T, nb padded
  const int nbp = split_ld(nb);
  if (!c.d_fsplit) {
    ROKS_CHECK(!c.no_alloc, ROKS_ERR_STATE, "the BF16x3 force buffers are not formed");
    c.d_fsplit = dalloc<uint16_t>(c, 2 * ((size_t)c.nproj + K) * nbp);
  }
  KernelTimer kt(c, "proj_bf3", (double)c.nproj * nb * 8.0 + (double)nb * K * 8.0 + (double)c.nproj * K * 8.0,
                 6.0 * c.nproj * (double)nb * K);
  uint16_t* ah = c.d_fsplit;
  uint16_t* al = ah + (size_t)c.nproj * nbp;
  uint16_t* bh = al + (size_t)c.nproj * nbp;
  uint16_t* bl = bh + (size_t)K * nbp;
  split_rows(c, DPw, lddp, c.nproj, nb, nbp, 0, ah, al);
  split_cols(c, X, ldx, nb, K, nbp, bh, bl);
  product(c, c.nproj, K, nbp, ah, al, nbp, bh, bl, nbp, Phi, K, nullptr, 0, 1.0, 0.0, false);
}

void proj_expand(Ctx& c, int nrows, const double* DP, int lddp, double* Y, int ldy) {
  const int K = 2 * c.npw;
  if (c.nproj == 0 || nrows == 0) return;
  if (!c.bf3) {
    gemm_expand(c, nrows, K, c.nproj, DP, lddp, false, reinterpret_cast<const double*>(c.d_B), K, Y, ldy,
                1.0, 1.0);
    return;
  }
  ROKS_CHECK(nrows <= c.nb, ROKS_ERR_ARG, "more rows than bands");
  ensure_tables(c);
  const int npp = split_ld(c.nproj);
  // the split table, D P in FP64, Y read and written
  KernelTimer kt(c, "proj_bf3", (double)K * npp * 4.0 + (double)c.nproj * nrows * 8.0 + 16.0 * nrows * (double)K,
                 6.0 * c.nproj * (double)nrows * K);
  uint16_t* dh = c.d_xsplit;
  uint16_t* dl = dh + (size_t)c.nb * npp;
  split_cols(c, DP, lddp, c.nproj, nrows, npp, dh, dl);
  product(c, nrows, K, npp, dh, dl, npp, c.d_bsplit_t, c.d_bsplit_t + (size_t)K * npp, npp, Y, ldy, Y,
          ldy, 1.0, 1.0, false);
}

}  // namespace roks
