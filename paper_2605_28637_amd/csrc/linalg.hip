// Dense linear algebra for the band and projector spaces (FP64):
//   gemm_expand Y = alpha * M^T X + beta * Y (short inner dimension, on the
//               FP64 matrix cores; from 128 rows of M on, the rocBLAS DGEMM).
//   gemm_small  nb x nb products (rotation, exponential, Cholesky factors).
// plus per-band weighted dots, the Cholesky inverse, the subspace matrices
// R / kappa / A and the Teter preconditioner.
#include <algorithm>
#include <cmath>


#include "roks_internal.h"

namespace roks {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// --------------------------------------------------------------------------
// Y[n][k] = alpha sum_m M(m, n) X[m][k] + beta Y[n][k] on the FP64 matrix
// cores (MFMA 16x16x4: lane l gives the A operand's row l%16 and the B
// operand's column l%16 at depth slot l/16; its 4 results are rows
// l/16 + 4r of column l%16).  Each wave owns 16 columns of K and 16 NB rows
// of Y: A = M^T (rows n), B = X (columns k), so every X load is a 128-byte
// row piece.  The workgroup stages M in LDS 64 rows at a time, and each wave
// issues all of a chunk's X loads before its MFMAs.
// --------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kExpandRows = 64;  // rows of X (depth) per chunk

template <int NB, bool TWO>
__global__ void __launch_bounds__(256) k_expand_mfma(int N, int K, int Md, const double* __restrict__ Mt,
                                                     int ldm, int transM, const double* __restrict__ X,
                                                     int ldx, const double* __restrict__ X2, double dX2,
                                                     const double* Yin, int ldyin, double* Y, int ldy,
                                                     double alpha, double beta) {
  constexpr int MC = kExpandRows, W = 16 * NB, NL = MC * W / 256;
  __shared__ double Ms[MC][W + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k0 = (blockIdx.x * 4 + wave) * 16;
  const bool active = k0 < K;
  const int n0 = blockIdx.y * W;
  const int c16 = lane & 15, s = lane >> 4;
  const int k = k0 + c16;
  double yv[NB][4];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = n0 + 16 * i + s + 4 * r;
      yv[i][r] = (beta != 0.0 && active && n < N && k < K) ? Yin[(size_t)n * ldyin + k] : 0.0;
    }
  d4 acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  for (int mc = 0; mc < Md; mc += MC) {
    double xb[MC / 4];
#pragma unroll
    for (int t = 0; t < MC / 4; ++t) {
      const int m = mc + 4 * t + s;
      xb[t] = (active && m < Md && k < K) ? X[(size_t)m * ldx + k] : 0.0;
    }
    if (TWO) {
      // the second input as its own batch of loads, then added
      double x2[MC / 4];
#pragma unroll
      for (int t = 0; t < MC / 4; ++t) {
        const int m = mc + 4 * t + s;
        x2[t] = (active && m < Md && k < K) ? X2[(size_t)m * ldx + k] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < MC / 4; ++t) xb[t] += dX2 * x2[t];
    }
    double tv[NL];
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int idx = tid + 256 * q;
      const int mm = idx / W, nn = idx - mm * W;
      const int m = mc + mm, n = n0 + nn;
      double v = 0.0;
      if (m < Md && n < N) v = transM ? Mt[(size_t)n * ldm + m] : Mt[(size_t)m * ldm + n];
      tv[q] = v;
    }
    __syncthreads();  // the previous chunk's reads of Ms are done
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int idx = tid + 256 * q;
      const int mm = idx / W;
      Ms[mm][idx - mm * W] = tv[q];
    }
    __syncthreads();
    const int depth = min(MC, Md - mc);
#pragma unroll
    for (int t = 0; t < MC / 4; ++t) {
      if (4 * t < depth) {
#pragma unroll
        for (int i = 0; i < NB; ++i)
          acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ms[4 * t + s][16 * i + c16], xb[t], acc[i], 0, 0, 0);
      }
    }
  }
  if (!active) return;
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = n0 + 16 * i + s + 4 * r;
      if (n < N && k < K) Y[(size_t)n * ldy + k] = alpha * acc[i][r] + beta * yv[i][r];
    }
}

// --------------------------------------------------------------------------
// small products: C = alpha op(A) op(B) + beta C, 16 x 16 tiles
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_gemm_small(int M, int N, int K, const double* __restrict__ A,
                                                    const double* __restrict__ A2, double a2, int lda,
                                                    int tA, const double* __restrict__ B, int ldb, int tB,
                                                    double* __restrict__ C, int ldc, double alpha,
                                                    double beta, double diag) {
  __shared__ double As[16][17];
  __shared__ double Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m = blockIdx.y * 16 + ty, n = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int ka = k0 + tx, kb = k0 + ty;
    // A(m, k) for this thread's row, B(k, n) for this thread's column
    double a = 0.0, b = 0.0;
    if (m < M && ka < K) {
      const size_t ia = tA ? (size_t)ka * lda + m : (size_t)m * lda + ka;
      a = A[ia];
      if (A2) a += a2 * A2[ia];  // op(A + a2 A2)
    }
    if (n < N && kb < K) b = tB ? B[(size_t)n * ldb + kb] : B[(size_t)kb * ldb + n];
    As[ty][tx] = a;
    Bs[ty][tx] = b;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc = fma(As[ty][kk], Bs[kk][tx], acc);
    __syncthreads();
  }
  if (m < M && n < N) {
    double v = alpha * acc;
    if (beta != 0.0) v += beta * C[(size_t)m * ldc + n];
    if (m == n) v += diag;
    C[(size_t)m * ldc + n] = v;
  }
}

// --------------------------------------------------------------------------
// per-band weighted dots: mode 0: sum w x.y; mode 1: sum w |G|^2/2 x.y
// --------------------------------------------------------------------------
// Per-band dots <x_n|y_n> over the stored half sphere (weight 1 at G = 0, 2
// elsewhere), out0 plain and out1 with the weight |G|^2/2 (either may be
// null); one workgroup per band.  (Splitting a band over workgroups with a
// last-arrival sum was slower: the device-scope fences it needs are costly on
// a GPU whose L2 is split over XCDs.)
__global__ void __launch_bounds__(1024) k_band_dots(const double2* __restrict__ X,
                                                   const double2* __restrict__ Yv, int npw,
                                                   const double* __restrict__ g2,
                                                   double* __restrict__ out0, double* __restrict__ out1,
                                                   double* __restrict__ mirror0,
                                                   double* __restrict__ mirror1) {
  __shared__ double red[2][16];
  const int n = blockIdx.x;
  const double2* x = X + (size_t)n * npw;
  const double2* y = Yv + (size_t)n * npw;
  double s0 = 0.0, s1 = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    double v = x[g].x * y[g].x + x[g].y * y[g].y;
    if (g != 0) v *= 2.0;
    s0 += v;
    if (out1) s1 += v * g2[g];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    red[0][wid] = s0;
    red[1][wid] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      t0 += red[0][w];
      t1 += red[1][w];
    }
    if (out0) out0[n] = t0;
    if (out1) out1[n] = t1;
    if (mirror0) mirror0[n] = t0;
    if (mirror1) mirror1[n] = t1;
  }
}

// Im c_n(G = 0) = 0 (G = 0 is entry 0 of every band)
__global__ void k_zero_g0_imag(double2* __restrict__ v, int nvec, int npw) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < nvec) v[(size_t)n * npw].y = 0.0;
}

__global__ void k_axpby(size_t n, double a, const double* __restrict__ x, double b,
                        const double* __restrict__ y, double* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double v = a * x[i];
    if (y) v += b * y[i];
    out[i] = v;
  }
}

__global__ void k_set_identity(double* A, int n, double d) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (t >= (size_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t - (size_t)i * n);
  A[t] = (i == j) ? d : 0.0;
}

// out = c0 I + c1 X + c2 X2 (X2 may be null), n x n
__global__ void k_poly_block(int n, double c0, double c1, const double* __restrict__ X, double c2,
                             const double* __restrict__ X2, double* __restrict__ out) {
  const size_t nn = (size_t)n * n;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < nn; t += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(t / n), j = (int)(t - (size_t)i * n);
    double v = c1 * X[t];
    if (X2) v += c2 * X2[t];
    if (i == j) v += c0;
    out[t] = v;
  }
}

__global__ void k_scale_shift(const double* __restrict__ in, int n, double a, double d,
                              double* __restrict__ out) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (t >= (size_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t - (size_t)i * n);
  out[t] = a * in[t] + ((i == j) ? d : 0.0);
}

// ||A||_1 = max_j sum_i |A_ij| by one 1024-thread workgroup: four
// row-interleaved partial column sums (dynamic LDS [4][n]), then their sum
// per column and the maximum
__global__ void __launch_bounds__(1024) k_norm1(const double* A, int n, double* out) {
  extern __shared__ double part[];
  __shared__ double red[16];
  const int g = threadIdx.x >> 8, tl = threadIdx.x & 255;
  for (int j = tl; j < n; j += 256) {
    double s = 0.0;
#pragma unroll 8
    for (int i = g; i < n; i += 4) s += fabs(A[(size_t)i * n + j]);
    part[g * n + j] = s;
  }
  __syncthreads();
  double mx = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x)
    mx = fmax(mx, ((part[j] + part[n + j]) + part[2 * n + j]) + part[3 * n + j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
    *out = m;
  }
}

// --------------------------------------------------------------------------
// Cholesky G = L L^T and L^-1 (lower); flag[0] = 1 if G is not numerically
// positive definite.  One workgroup in LDS up to 128 bands, blocked beyond
// (cholesky_inverse_blocked).
// --------------------------------------------------------------------------

// Cholesky factorisation G = L L^T and (inv_in_lds, n <= 96) the inverse
// L^-1 in one workgroup, right-looking, one barrier per column.  Threads sit
// on a fixed 32 x 32 grid (rows i = j + 1 + ty + 32 a, columns k = ... + tx).
// At column j: A_ik -= A_ij A_kj / A_jj on the trailing block and
// X_ic -= A_ij X_jc / A_jj on the rows below j of X (the forward elimination
// of L X = I), both from the unscaled column j and row j, which nobody writes
// in that step; row j of X becomes row j of L^-1 = X_j / sqrt(A_jj) one step
// later.  Thread 0, which updates the next diagonal element, also takes the
// next pivot's 1/d and 1/sqrt(d) (a pivot not above 1e-12 of its Gram
// diagonal, or not finite, sets the flag and is replaced by 1).
// Without inv_in_lds (97 <= n <= 128) the factor is scaled in place and
// L^-1 is formed column by column from it.
// LDS row stride of the single-workgroup Cholesky: n rounded up to odd
__host__ __device__ inline int chol_ld(int n) { return n | 1; }

// acc_flag: OR the status into flag[0] (blocks of a larger factorisation);
// gref (stride gref_ld, nullable): the diagonal the pivot test refers to,
// when G is a Schur complement of a larger Gram matrix (its diagonal there)
__device__ void cholesky_lds_body(const double* __restrict__ G, double ga, double gd, int n,
                                  double* __restrict__ Linv, int32_t* __restrict__ flag, int inv_in_lds,
                                  double* A, int acc_flag = 0, const double* __restrict__ gref = nullptr,
                                  int gref_ld = 0) {
  __shared__ int bad;
  __shared__ double gdiag[128];   // the Gram diagonal, the reference of the pivot test
  __shared__ double piv[2][2];    // [step parity]: 1/d, 1/sqrt(d)
  __shared__ double rsv[128];     // 1/L_jj
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int ld = chol_ld(n);  // odd row stride: a column read by a warp of rows spreads the banks
  double* X = A + n * ld;
#pragma unroll 4
  for (int t = tid; t < n * n; t += nthr) {
    const int r = t / n, q = t - r * n;
    const double g = ga * G[t] + (r == q ? gd : 0.0);  // the matrix factorised: ga G + gd I
    A[r * ld + q] = g;
    if (r == q) gdiag[r] = gref ? gref[(size_t)r * gref_ld] : g;
    if (inv_in_lds) X[r * ld + q] = r == q ? 1.0 : 0.0;
  }
  auto pivot = [&](int j, double d) {
    if (!(d > 1e-12 * gdiag[j]) || !isfinite(d)) {
      bad = 1;
      d = 1.0;
    }
    const double rs = 1.0 / sqrt(d);
    piv[j & 1][0] = 1.0 / d;
    piv[j & 1][1] = rs;
    rsv[j] = rs;
  };
  // the last group of 32 threads stays off the trailing update: its first
  // thread computes the next pivot as soon as a column starts (the critical
  // path of the column), the others scale the finished row of the inverse
  const int pivt = nthr - 32;
  __syncthreads();  // gdiag, read by the pivot thread, is written by others
  if (tid == pivt) {
    bad = 0;
    pivot(0, ga * G[0] + gd);
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double rd = piv[j & 1][0];
    if (tid >= pivt) {
      if (tid == pivt) {
        if (j + 1 < n) {
          // the update of element (j+1, j+1), as the update threads would do it
          const double a = A[(j + 1) * ld + j];
          const double f = a * rd;
          const double v = A[(j + 1) * ld + j + 1] - f * a;
          A[(j + 1) * ld + j + 1] = v;
          pivot(j + 1, v);
        }
      } else if (inv_in_lds && j > 0) {
        // the previous row of the inverse is final: scale it
        for (int cc = tid - pivt - 1; cc < j; cc += 31) X[(j - 1) * ld + cc] *= rsv[j - 1];
      }
    } else {
      const int tx = tid & 31, ty = tid >> 5, nyu = pivt >> 5;
      for (int i = j + 1 + ty; i < n; i += nyu) {
        const double f = A[i * ld + j] * rd;
        for (int k = j + 1 + tx; k <= i; k += 32) {
          if (i == j + 1 && k == j + 1) continue;  // the pivot thread's
          A[i * ld + k] = A[i * ld + k] - f * A[k * ld + j];
        }
        if (inv_in_lds)
          for (int cc = tx; cc <= j; cc += 32) X[i * ld + cc] -= f * X[j * ld + cc];
      }
    }
    __syncthreads();
  }
  if (inv_in_lds) {
    for (int cc = tid; cc < n; cc += nthr) X[(n - 1) * ld + cc] *= rsv[n - 1];
    __syncthreads();
    for (int t = tid; t < n * n; t += nthr) {
      const int r = t / n, q = t - r * n;
      Linv[t] = q <= r ? X[r * ld + q] : 0.0;
    }
  } else {
    // L = column j of A scaled by 1/sqrt(d_j), diagonal sqrt(d_j)
    for (int t = tid; t < n * n; t += nthr) {
      const int i = t / n, k = t % n;
      if (k < i) A[i * ld + k] *= rsv[k];
      else if (k == i) A[i * ld + k] = 1.0 / rsv[k];
    }
    __syncthreads();
    for (int col = tid; col < n; col += nthr) {
      for (int i = 0; i < col; ++i) Linv[(size_t)i * n + col] = 0.0;
      Linv[(size_t)col * n + col] = 1.0 / A[col * ld + col];
      for (int i = col + 1; i < n; ++i) {
        double s = 0.0;
        for (int k = col; k < i; ++k) s += A[i * ld + k] * Linv[(size_t)k * n + col];
        Linv[(size_t)i * n + col] = -s / A[i * ld + i];
      }
    }
  }
  if (tid == 0) flag[0] = acc_flag ? (flag[0] | bad) : bad;
}

__global__ void __launch_bounds__(1024) k_cholesky_inverse_lds(const double* __restrict__ G, int n,
                                                               double* __restrict__ Linv,
                                                               int32_t* __restrict__ flag,
                                                               int inv_in_lds, int acc_flag,
                                                               const double* __restrict__ gref,
                                                               int gref_ld) {
  extern __shared__ double A[];
  cholesky_lds_body(G, 1.0, 0.0, n, Linv, flag, inv_in_lds, A, acc_flag, gref, gref_ld);
}

// rows j0 .. j0+rows-1 of the n x n identity, [rows][n]
__global__ void k_eye_rows(double* __restrict__ R, int rows, int n, int j0) {
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (t >= (size_t)rows * n) return;
  const int r = (int)(t / n), col = (int)(t - (size_t)r * n);
  R[t] = (j0 + r == col) ? 1.0 : 0.0;
}

// U = exp(delta D) in one workgroup, the three n x n matrices in LDS:
// scaling and squaring around a Taylor polynomial in Horner form.  The
// degree m and the squarings s minimise the products m + s subject to
// theta^(m+1)/(m+1)! <= 1e-17 with theta = ||delta D||_1 / 2^s <= 1 (the
// Taylor tail; exp of an antisymmetric matrix is orthogonal, so the bound is
// relative).  Products run on the FP64 matrix cores.
__device__ void expm_lds_body(const double* __restrict__ D, int n, double delta,
                              double* __restrict__ U, double* S) {
  __shared__ double nrm;
  __shared__ int plan[2];
  const int tid = threadIdx.x, nthr = blockDim.x, nn = n * n;
  double* X = S;
  double* P = S + nn;
  double* Q = P + nn;
#pragma unroll 4
  for (int t = tid; t < nn; t += nthr) X[t] = delta * D[t];
  __syncthreads();
  // column sums of |X|: C row-interleaved partial sums per column (kept in P,
  // which is not yet in use), then one wave adds them and takes the maximum
  const int C = n < 16 ? n : 16;
  for (int t = tid; t < C * n; t += nthr) {
    const int c = t / n, j = t - c * n;
    double s = 0.0;
    for (int i = c; i < n; i += C) s += fabs(X[i * n + j]);
    P[c * n + j] = s;
  }
  __syncthreads();
  if (tid < 64) {
    double mx = 0.0;
    for (int j = tid; j < n; j += 64) {
      double s = 0.0;
      for (int c = 0; c < C; ++c) s += P[c * n + j];
      mx = fmax(mx, s);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    // lane sq (0..60) prices s = sq squarings: the least degree m whose Taylor
    // tail th^(m+1)/(m+1)! is below 1e-17 (th = ||X||_1 / 2^sq <= 1, m <= 30);
    // the cheapest m + s wins, the fewest squarings on ties.  A norm that is
    // not finite gets m = 1, s = 0 (the rotation is then rejected downstream);
    // one above 2^60 gets m = 30, s = 0.
    constexpr int kNone = 1 << 20;  // no admissible degree at this s
    const int sq = tid;
    int cost = kNone, m = 30;
    const double th = ldexp(mx, -sq);
    if (sq <= 60 && isfinite(mx) && th <= 1.0) {
      double term = th;  // th^(m+1)/(m+1)!
      m = 0;
      while (term > 1e-17 && m < 30) {
        ++m;
        term *= th / (m + 1);
      }
      cost = m + sq;
    }
    int key = cost * 64 + sq;  // the least cost, then the least sq
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) key = min(key, __shfl_xor(key, off, 64));
    const int win = key & 63;
    const int mwin = __shfl(m, win, 64);
    if (tid == 0) {
      nrm = mx;
      if (!isfinite(mx)) {
        plan[0] = 0;
        plan[1] = 1;
      } else if ((key >> 6) >= kNone) {
        plan[0] = 0;
        plan[1] = 30;
      } else {
        plan[0] = win;
        plan[1] = mwin;
      }
    }
  }
  __syncthreads();
  const int sq = plan[0], m = plan[1];
  const double scale = ldexp(1.0, -sq);
  for (int t = tid; t < nn; t += nthr) {
    X[t] *= scale;
    const double id = (t / n) == (t % n) ? 1.0 : 0.0;
    P[t] = m >= 1 ? X[t] / (double)m + id : id;
  }
  __syncthreads();
  // O = L R * f (+ I when add_id) on the FP64 matrix cores: wave w computes
  // the 16 x 16 output blocks w, w + 16, ...  (MFMA 16x16x4 operands from
  // LDS: lane l reads row l%16 of L and column l%16 of R at depth slot l/16;
  // its results are rows l/16 + 4r of column l%16)
  const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  const int nbk = (n + 15) / 16, r16 = lane & 15, s4 = lane >> 4;
  auto product = [&](const double* L, const double* R, double* O, double f, bool add_id) {
    for (int blk = wave; blk < nbk * nbk; blk += nw) {
      const int bi = blk / nbk, bj = blk - bi * nbk;
      const int row = 16 * bi + r16, col = 16 * bj + r16;
      d4 acc = d4{0.0, 0.0, 0.0, 0.0};
      for (int k4 = 0; k4 < n; k4 += 4) {
        const int k = k4 + s4;
        const double a = (row < n && k < n) ? L[row * n + k] : 0.0;
        const double b = (k < n && col < n) ? R[k * n + col] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * bi + s4 + 4 * r, j = 16 * bj + r16;
        if (i < n && j < n) O[i * n + j] = acc[r] * f + ((add_id && i == j) ? 1.0 : 0.0);
      }
    }
    __syncthreads();
  };
  // P_m = I + X/m, P_q = I + X P_{q+1} / q, ..., P_1 = the degree-m polynomial
  for (int q = m - 1; q >= 1; --q) {
    product(X, P, Q, 1.0 / (double)q, true);
    double* tmp = P;
    P = Q;
    Q = tmp;
  }
  for (int r = 0; r < sq; ++r) {
    product(P, P, Q, 1.0, false);
    double* tmp = P;
    P = Q;
    Q = tmp;
  }
  for (int t = tid; t < nn; t += nthr) U[t] = P[t];
}

__global__ void __launch_bounds__(1024) k_expm_lds(const double* __restrict__ D, int n, double delta,
                                                  double* __restrict__ U) {
  extern __shared__ double S[];
  expm_lds_body(D, n, delta, U, S);
}

// the two independent single-workgroup steps of a trial in one launch:
// workgroup 0 factorises the Gram matrix, workgroup 1 exponentiates delta D
__global__ void __launch_bounds__(1024) k_chol_expm_lds(const double* __restrict__ G, double ga,
                                                       double gd, int n, double* __restrict__ Linv,
                                                       int32_t* __restrict__ flag, int inv_in_lds,
                                                       const double* __restrict__ D, double delta,
                                                       double* __restrict__ U) {
  extern __shared__ double S[];
  if (blockIdx.x == 0)
    cholesky_lds_body(G, ga, gd, n, Linv, flag, inv_in_lds, S);
  else
    expm_lds_body(D, n, delta, U, S);
}

// --------------------------------------------------------------------------
// subspace matrices from theta_mn = <m|F^{X(n)}|n>, the band scalars
// t_n = <n|T + V_NL|n> and Q[n][X] = <n|V^X|n> (local part of F^X):
//   cross-shell pairs (m in an earlier shell than n):
//     R_mn = theta_nm - theta_mn = <m|F^X(m) - F^X(n)|n>  (F^virtual = 0)
//     kappa_mn = F^Xm_nn - F^Xm_mm + F^Xn_mm - F^Xn_nn
//     A_mn = atan2(2 R_mn, |kappa_mn|) / 2,  A_nm = -A_mn
//   same occupied shell: R_mn = theta_mn; rotated only when canonicalising,
//     with kappa = R_nn - R_mm (Jacobi angle).
// --------------------------------------------------------------------------
struct SubArgs {
  int nb, nsocc, flags, open_a, open_b;
  double w[kMaxShell];
  int virt[kMaxShell];
};

__device__ void open_coupling_body(const double* __restrict__ theta, int nb,
                                   const int32_t* __restrict__ shell, int sa, int sb,
                                   double* __restrict__ out, double* red);

// oc: when not null, the last workgroup (256 threads) writes the open-shell
// coupling max |theta_nm - theta_mn| (m in shell open_a, n in open_b) there
__global__ void k_subspace(SubArgs a, const double* __restrict__ theta,
                           const int32_t* __restrict__ shell, const double* __restrict__ tkin,
                           const double* __restrict__ tnl, const double* __restrict__ Q,
                           double* __restrict__ R, double* __restrict__ kappa,
                           double* __restrict__ A, double* __restrict__ oc) {
  if (oc && blockIdx.x == gridDim.x - 1) {
    __shared__ double red[256];
    open_coupling_body(theta, a.nb, shell, a.open_a, a.open_b, oc, red);
    return;
  }
  const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int nb = a.nb;
  if (t >= (size_t)nb * nb) return;
  const int m = (int)(t / nb), n = (int)(t - (size_t)m * nb);
  const int Xm = shell[m], Xn = shell[n];
  auto FX = [&](int X, int b) -> double {
    if (a.virt[X]) return 0.0;
    return a.w[X] * (tkin[b] + tnl[b]) + Q[(size_t)b * a.nsocc + X];
  };
  double r = 0.0, k = 0.0, ang = 0.0;
  if (m == n) {
    r = a.virt[Xm] ? 0.0 : theta[(size_t)m * nb + m];
  } else {
    const int lo = m < n ? m : n, hi = m < n ? n : m;
    const int Xl = shell[lo], Xh = shell[hi];
    double rl, kl, al = 0.0;
    if (Xl == Xh) {
      rl = a.virt[Xl] ? 0.0 : theta[(size_t)lo * nb + hi];
      kl = 0.0;
      if ((a.flags & ROKS_FLAG_CANONICALIZE) && !a.virt[Xl]) {
        kl = theta[(size_t)hi * nb + hi] - theta[(size_t)lo * nb + lo];
        al = kl != 0.0 ? 0.5 * atan(2.0 * rl / kl) : (rl > 0 ? M_PI / 4 : (rl < 0 ? -M_PI / 4 : 0.0));
      }
    } else {
      rl = theta[(size_t)hi * nb + lo] - theta[(size_t)lo * nb + hi];
      if ((a.flags & ROKS_FLAG_SUPPRESS_OPEN_COUPLING) && a.open_a >= 0 &&
          ((Xl == a.open_a && Xh == a.open_b) || (Xl == a.open_b && Xh == a.open_a)))
        rl = 0.0;
      kl = FX(Xl, hi) - FX(Xl, lo) + FX(Xh, lo) - FX(Xh, hi);
      al = 0.5 * atan2(2.0 * rl, fabs(kl));
    }
    r = rl;
    k = kl;
    ang = m < n ? al : -al;
  }
  R[t] = r;
  kappa[t] = k;
  A[t] = ang;
}

// the virtual block of R: R[n][m] = R[m][n] for v0 <= m < n (products in
// the upper triangle); with canonicalisation kappa = R_nn - R_mm and the
// Jacobi angle A_mn = 1/2 atan(2 R_mn / kappa) (+-pi/4 for kappa = 0)
__global__ void k_virtual_block(double* __restrict__ R, double* __restrict__ kappa,
                                double* __restrict__ A, int nb, int v0, int canon) {
  const int nv = nb - v0;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nv * nv) return;
  const int m = v0 + t / nv, n = v0 + t % nv;
  if (m >= n) return;
  const double r = R[(size_t)m * nb + n];
  R[(size_t)n * nb + m] = r;
  if (canon) {
    const double k = R[(size_t)n * nb + n] - R[(size_t)m * nb + m];
    const double a = k != 0.0 ? 0.5 * atan(2.0 * r / k) : (r > 0 ? M_PI / 4 : (r < 0 ? -M_PI / 4 : 0.0));
    kappa[(size_t)m * nb + n] = kappa[(size_t)n * nb + m] = k;
    A[(size_t)m * nb + n] = a;
    A[(size_t)n * nb + m] = -a;
  }
}

// sum_mn A_mn (theta_mn - theta_nm), one workgroup
// sum_mn A_mn (th_mn - th_nm) by the first nt threads of the workgroup, nt =
// 256, or every thread (up to 1024) beyond 128 bands (fixed order: nt-strided
// partials, wave sums, the waves in order)
__device__ void asym_dot_body(const double* __restrict__ A, const double* __restrict__ th, int nb,
                              double* __restrict__ out, double* __restrict__ mirror, double* red) {
  const int nt = (nb > 128 && blockDim.x >= 1024) ? 1024 : 256;
  double s = 0.0;
  if ((int)threadIdx.x < nt)
    for (size_t t = threadIdx.x; t < (size_t)nb * nb; t += nt) {
      const int m = (int)(t / nb), n = (int)(t - (size_t)m * nb);
      s += A[t] * (th[t] - th[(size_t)n * nb + m]);
    }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0 && (int)threadIdx.x < nt) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int w = 0; w < nt / 64; ++w) v += red[w];
    *out = v;
    if (mirror) *mirror = v;
  }
}

__global__ void k_asym_dot(const double* __restrict__ A, const double* __restrict__ th, int nb,
                           double* __restrict__ out, double* __restrict__ mirror) {
  __shared__ double red[16];
  asym_dot_body(A, th, nb, out, mirror, red);
}

// band dots <x_n|y_n> (workgroups 0 .. nvec-1, as k_band_dots with out0) and
// the antisymmetric contraction of A with th (workgroup nvec) in one launch
__global__ void __launch_bounds__(1024) k_band_dots_asym(const double2* __restrict__ X,
                                                        const double2* __restrict__ Yv, int npw,
                                                        double* __restrict__ out0,
                                                        double* __restrict__ mirror0,
                                                        const double* __restrict__ A,
                                                        const double* __restrict__ th, int nb,
                                                        double* __restrict__ aout,
                                                        double* __restrict__ amirror) {
  __shared__ double red[16];
  const int n = blockIdx.x;
  if (A && n == (int)gridDim.x - 1) {
    asym_dot_body(A, th, nb, aout, amirror, red);
    return;
  }
  const double2* x = X + (size_t)n * npw;
  const double2* y = Yv + (size_t)n * npw;
  double s0 = 0.0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    double v = x[g].x * y[g].x + x[g].y * y[g].y;
    if (g != 0) v *= 2.0;
    s0 += v;
  }
  s0 = wave_sum(s0);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[wid] = s0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t0 += red[w];
    if (out0) out0[n] = t0;
    if (mirror0) mirror0[n] = t0;
  }
}

// CG directions with the Fletcher-Reeves ratio formed in every workgroup
// (beta = (sum_n pgb[n] + asym / 2) / pg_old, band order): S = p + beta w
// over n1 values, then D = A + beta D_old over n2 values; workgroup 0 keeps
// beta in beta_out
__global__ void k_cg_directions(size_t n1, const double* __restrict__ p, const double* __restrict__ w,
                                double* __restrict__ S, size_t n2, const double* __restrict__ A,
                                const double* __restrict__ Dold, double* __restrict__ D,
                                const double* __restrict__ asym, const double* __restrict__ pgb,
                                int nb, double pg_old, double* __restrict__ beta_out) {
  __shared__ double sb;
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int n = 0; n < nb; ++n) v += pgb[n];
    v += 0.5 * asym[0];
    sb = v / pg_old;
    if (blockIdx.x == 0) beta_out[0] = sb;
  }
  __syncthreads();
  const double bb = sb;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n1 + n2;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < n1) {
      double v = 1.0 * p[i];
      v += bb * w[i];
      S[i] = v;
    } else {
      const size_t j = i - n1;
      double v = 1.0 * A[j];
      v += bb * Dold[j];
      D[j] = v;
    }
  }
}

// Teter-Payne-Allan: K(x) = -(2/E_ref) P(x)/(P(x) + 16 x^4), P = 27 + 18x + 12x^2 + 8x^3,
// x = (|G|^2/2) / E_ref with E_ref = 1.5 <g|T|g>/<g|g> per band
__global__ void k_teter(const double2* __restrict__ g, int npw, int nb, const double* __restrict__ gTg,
                        const double* __restrict__ gg, const double* __restrict__ g2,
                        const double* __restrict__ bandw, double2* __restrict__ out) {
  const size_t total = (size_t)nb * npw;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const int n = (int)(t / npw), q = (int)(t - (size_t)n * npw);
    double2 v = make_double2(0.0, 0.0);
    if (gg[n] > 0.0) {
      const double eref = 1.5 * gTg[n] / gg[n];
      if (eref > 0.0) {
        const double x = g2[q] / eref;
        const double x2 = x * x;
        const double p = 27.0 + 18.0 * x + 12.0 * x2 + 8.0 * x2 * x;
        double K = -(2.0 / eref) * p / (p + 16.0 * x2 * x2);
        if (bandw) K /= bandw[n];
        v = make_double2(K * g[t].x, K * g[t].y);
      }
    }
    out[t] = v;
  }
}

// max |theta_nm - theta_mn| over bands m of shell sa and n of shell sb
// max |theta_nm - theta_mn| over m in shell sa, n in shell sb, by a
// 256-thread workgroup (fixed tree)
__device__ void open_coupling_body(const double* __restrict__ theta, int nb,
                                   const int32_t* __restrict__ shell, int sa, int sb,
                                   double* __restrict__ out, double* red) {
  double mx = 0.0;
  for (int t = threadIdx.x; t < nb * nb; t += 256) {
    const int m = t / nb, n = t - m * nb;
    if (shell[m] == sa && shell[n] == sb)
      mx = fmax(mx, fabs(theta[(size_t)n * nb + m] - theta[(size_t)m * nb + n]));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

int blocks_for(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b > 8192 ? 8192 : (b == 0 ? 1 : b));
}

}  // namespace

void gemm_expand(Ctx& c, int N, int K, int Md, const double* M, int ldm, bool transM,
                 const double* X, int ldx, double* Y, int ldy, double alpha, double beta) {
  gemm_expand_to(c, N, K, Md, M, ldm, transM, X, ldx, Y, ldy, Y, ldy, alpha, beta);
}

void gemm_expand_to(Ctx& c, int N, int K, int Md, const double* M, int ldm, bool transM,
                    const double* X, int ldx, const double* Yin, int ldyin, double* Y, int ldy,
                    double alpha, double beta) {
  gemm_expand_sum(c, N, K, Md, M, ldm, transM, X, nullptr, 0.0, ldx, Yin, ldyin, Y, ldy, alpha, beta);
}

void gemm_expand_sum(Ctx& c, int N, int K, int Md, const double* M, int ldm, bool transM,
                     const double* X, const double* X2, double dX2, int ldx, const double* Yin,
                     int ldyin, double* Y, int ldy, double alpha, double beta) {
  if (N == 0 || K == 0) return;
  KernelTimer kt(c, "gemm_expand",
                 ((double)Md * K + (beta != 0.0 ? 2.0 : 1.0) * N * K) * sizeof(double),
                 2.0 * N * (double)K * Md);
  if (Md >= 128 && N >= 64) {
    // a compute-bound size: the LDS-tiled product, Y[n][k] = alpha sum_i
    // M^(T)[n][i] (X + dX2 X2)[i][k] + beta Yin[n][k], the sum formed while
    // staging X
    tile_gemm(c, N, K, Md, M, ldm, transM ? 0 : 1, X, ldx, 1, X2, dX2, Y, ldy, Yin, ldyin, alpha,
              beta, false, 1);
    return;
  }
  // 16-row blocks of Y per wave: 1..3, the least padding, the larger on ties
  const int n16 = cdiv(N, 16);
  int nb = 1;
  for (int b = 2; b <= 3; ++b)
    if (cdiv(n16, b) * b <= cdiv(n16, nb) * nb) nb = b;
  dim3 grid(cdiv(K, 64), cdiv(N, 16 * nb));
  const int tm = transM ? 1 : 0;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, c.stream, N, K, Md, M, ldm, tm, X, ldx, X2, dX2, Yin,
                       ldyin, Y, ldy, alpha, beta);
  };
  if (X2) {
    if (nb == 1) go(k_expand_mfma<1, true>);
    else if (nb == 2) go(k_expand_mfma<2, true>);
    else go(k_expand_mfma<3, true>);
  } else {
    if (nb == 1) go(k_expand_mfma<1, false>);
    else if (nb == 2) go(k_expand_mfma<2, false>);
    else go(k_expand_mfma<3, false>);
  }
  ROKS_HIP(hipGetLastError());
}

void gemm_small(Ctx& c, int M, int N, int K, const double* A, int lda, bool tA, const double* B,
                int ldb, bool tB, double* C, int ldc, double alpha, double beta, double diag) {
  gemm_small2(c, M, N, K, A, nullptr, 0.0, lda, tA, B, ldb, tB, C, ldc, alpha, beta, diag);
}

static void gemm_rm(Ctx& c, bool tA, bool tB, int M, int N, int K, double alpha, const double* A,
                    int lda, const double* B, int ldb, double beta, double* C, int ldc);

// C[i][i] += d for i < n
__global__ void k_add_diag(double* __restrict__ C, int n, int ldc, double d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) C[(size_t)i * ldc + i] += d;
}

void gemm_small2(Ctx& c, int M, int N, int K, const double* A, const double* A2, double a2, int lda,
                 bool tA, const double* B, int ldb, bool tB, double* C, int ldc, double alpha,
                 double beta, double diag) {
  if (!A2 && M >= 128 && N >= 128 && K >= 128) {
    // a compute-bound size (the large-band exponential): the LDS-tiled product
    gemm_rm(c, tA, tB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    if (diag != 0.0) {
      const int nd = std::min(M, N);
      hipLaunchKernelGGL(k_add_diag, dim3(cdiv(nd, 256)), dim3(256), 0, c.stream, C, nd, ldc, diag);
      ROKS_HIP(hipGetLastError());
    }
    return;
  }
  dim3 grid(cdiv(N, 16), cdiv(M, 16));
  hipLaunchKernelGGL(k_gemm_small, grid, dim3(256), 0, c.stream, M, N, K, A, A2, a2, lda, tA ? 1 : 0, B,
                     ldb, tB ? 1 : 0, C, ldc, alpha, beta, diag);
  ROKS_HIP(hipGetLastError());
}

void band_dots2(Ctx& c, const double2* X, const double2* Y, int nvec, double* out0, double* out1,
                double* mirror0, double* mirror1) {
  if (nvec == 0) return;
  hipLaunchKernelGGL(k_band_dots, dim3(nvec), dim3(1024), 0, c.stream, X, Y, c.npw, c.d_g2, out0, out1,
                     mirror0, mirror1);
  ROKS_HIP(hipGetLastError());
}

void band_dots(Ctx& c, const double2* X, const double2* Y, int nvec, int mode, double* out) {
  if (mode == 1)
    band_dots2(c, X, Y, nvec, nullptr, out);
  else
    band_dots2(c, X, Y, nvec, out, nullptr);
}

void launch_virtual_block(Ctx& c, int v0) {
  const int nv = c.nb - v0;
  if (nv <= 1) return;
  hipLaunchKernelGGL(k_virtual_block, dim3(cdiv(nv * nv, 256)), dim3(256), 0, c.stream, c.d_R,
                     c.d_kappa, c.d_A, c.nb, v0, (c.flags & ROKS_FLAG_CANONICALIZE) ? 1 : 0);
  ROKS_HIP(hipGetLastError());
}

void launch_zero_g0_imag(Ctx& c, double2* vecs, int nvec) {
  if (nvec <= 0) return;
  hipLaunchKernelGGL(k_zero_g0_imag, dim3(cdiv(nvec, 256)), dim3(256), 0, c.stream, vecs, nvec, c.npw);
  ROKS_HIP(hipGetLastError());
}

void axpby(Ctx& c, size_t n, double a, const double* x, double b, const double* y, double* out) {
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n)), dim3(256), 0, c.stream, n, a, x, b, y, out);
  ROKS_HIP(hipGetLastError());
}

int taylor_products(int m) { return (m >= 2) + (m >= 3) + m / 3; }

// T_m(X) = sum_{k <= m} X^k / k! by the Paterson-Stockmeyer scheme with
// blocks of three: T = B_0 + Y (B_1 + Y (B_2 + ...)), Y = X^3, B_j = c_3j I +
// c_3j+1 X + c_3j+2 X^2 (c_k = 1/k!, zero past m): taylor_products(m)
// products instead of m in Horner form.  X2, X3, w0, w1 are n x n scratch;
// returns the buffer (w0 or w1) holding the result.
double* taylor_ps(Ctx& c, int n, int m, const double* X, double* X2, double* X3, double* w0, double* w1) {
  const size_t nn = (size_t)n * n;
  std::vector<double> cf(m + 3, 0.0);
  cf[0] = 1.0;
  for (int k = 1; k <= m; ++k) cf[k] = cf[k - 1] / k;
  if (m >= 2) gemm_small(c, n, n, n, X, n, false, X, n, false, X2, n, 1.0, 0.0);
  const int r = m / 3;
  if (r >= 1) gemm_small(c, n, n, n, X2, n, false, X, n, false, X3, n, 1.0, 0.0);
  const unsigned grid = (unsigned)std::min<size_t>(4096, (nn + 255) / 256);
  auto block = [&](int j, double* out) {
    hipLaunchKernelGGL(k_poly_block, dim3(grid), dim3(256), 0, c.stream, n, cf[3 * j], cf[3 * j + 1], X,
                       cf[3 * j + 2], m >= 2 ? X2 : nullptr, out);
    ROKS_HIP(hipGetLastError());
  };
  double* acc = w0;
  double* nxt = w1;
  block(r, acc);
  for (int j = r - 1; j >= 0; --j) {
    block(j, nxt);
    gemm_small(c, n, n, n, X3, n, false, acc, n, false, nxt, n, 1.0, 1.0);
    std::swap(acc, nxt);
  }
  return acc;
}

void set_identity(Ctx& c, double* A, int n, double diag) {
  const size_t nn = (size_t)n * n;
  hipLaunchKernelGGL(k_set_identity, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, c.stream, A, n,
                     diag);
  ROKS_HIP(hipGetLastError());
}

void scale_shift(Ctx& c, const double* in, int n, double a, double d, double* out) {
  const size_t nn = (size_t)n * n;
  hipLaunchKernelGGL(k_scale_shift, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, c.stream, in, n,
                     a, d, out);
  ROKS_HIP(hipGetLastError());
}

void matrix_norm1(Ctx& c, const double* A, int n, double* out) {
  ROKS_CHECK(n <= 2048, ROKS_ERR_SHAPE, "matrix too large for the 1-norm kernel");
  hipLaunchKernelGGL(k_norm1, dim3(1), dim3(1024), (size_t)4 * n * sizeof(double), c.stream, A, n, out);
  ROKS_HIP(hipGetLastError());
}

// row-major C (M x N) = alpha op(A) op(B) + beta C, the LDS-tiled product
static void gemm_rm(Ctx& c, bool tA, bool tB, int M, int N, int K, double alpha, const double* A,
                    int lda, const double* B, int ldb, double beta, double* C, int ldc) {
  if (M == 0 || N == 0 || K == 0) return;
  tile_gemm(c, M, N, K, A, lda, tA ? 1 : 0, B, ldb, tB ? 0 : 1, nullptr, 0.0, C, ldc, nullptr, 0, alpha,
            beta, false, 0);
}

// L^-1 of G = L L^T for n > 128, blocked by 64: the diagonal block of each
// panel factorised and inverted by the single-workgroup kernel (its status
// ORed into flag[0]; the dependency test refers to the diagonal of G), the panel below L21 = A21 L11^-T and the trailing update
// A22 -= L21 L21^T as GEMMs; then L^-1 by block rows, X_i = L_ii^-1 (I_i -
// L_i,<i X_<i).  Scratch: d_m3 (the updated matrix), d_m4 (L below the
// diagonal blocks), d_m1 (the diagonal blocks' inverses), d_m2 (a block, then
// a block row).
static void cholesky_inverse_blocked(Ctx& c, const double* G, int n, double* Linv, int32_t* flag) {
  constexpr int b = 64;
  double* A = c.d_m3;
  double* Lb = c.d_m4;
  double* Dinv = c.d_m1;
  double* T = c.d_m2;
  const size_t lds = (size_t)2 * b * chol_ld(b) * sizeof(double);
  if (lds > 65536)
    ROKS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cholesky_inverse_lds),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  ROKS_HIP(hipMemcpyAsync(A, G, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
  const int P = cdiv(n, b);
  for (int p = 0; p < P; ++p) {
    const int j0 = p * b, bs = std::min(b, n - j0), j1 = j0 + bs, m = n - j1;
    ROKS_HIP(hipMemcpy2DAsync(T, (size_t)bs * sizeof(double), A + (size_t)j0 * n + j0,
                              (size_t)n * sizeof(double), (size_t)bs * sizeof(double), bs,
                              hipMemcpyDeviceToDevice, c.stream));
    double* Di = Dinv + (size_t)p * b * b;
    // pivots are tested against the diagonal of the original Gram matrix: a
    // band dependent on bands of earlier panels leaves a rounding-level pivot
    // in the updated block
    hipLaunchKernelGGL(k_cholesky_inverse_lds, dim3(1), dim3(1024), lds, c.stream, T, bs, Di, flag, 1,
                       p > 0 ? 1 : 0, G + (size_t)j0 * n + j0, n + 1);
    ROKS_HIP(hipGetLastError());
    if (m > 0) {
      double* L21 = Lb + (size_t)j1 * n + j0;
      gemm_rm(c, false, true, m, bs, bs, 1.0, A + (size_t)j1 * n + j0, n, Di, bs, 0.0, L21, n);
      gemm_rm(c, false, true, m, m, bs, -1.0, L21, n, L21, n, 1.0, A + (size_t)j1 * n + j1, n);
    }
  }
  for (int p = 0; p < P; ++p) {
    const int j0 = p * b, bs = std::min(b, n - j0);
    double* R = T;
    const size_t nr = (size_t)bs * n;
    hipLaunchKernelGGL(k_eye_rows, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, c.stream, R, bs, n,
                       j0);
    ROKS_HIP(hipGetLastError());
    gemm_rm(c, false, false, bs, n, j0, -1.0, Lb + (size_t)j0 * n, n, Linv, n, 1.0, R, n);
    gemm_rm(c, false, false, bs, n, bs, 1.0, Dinv + (size_t)p * b * b, bs, R, n, 0.0,
            Linv + (size_t)j0 * n, n);
  }
}

void cholesky_inverse(Ctx& c, const double* G, int n, double* Linv, int32_t* flag) {
  if (n <= 128) {
    const int inv = n <= 96 ? 1 : 0;
    const size_t lds = (size_t)(inv ? 2 : 1) * n * chol_ld(n) * sizeof(double);
    if (lds > 65536)
      ROKS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cholesky_inverse_lds),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_cholesky_inverse_lds, dim3(1), dim3(1024), lds, c.stream, G, n, Linv, flag,
                       inv, 0, static_cast<const double*>(nullptr), 0);
    ROKS_HIP(hipGetLastError());
  } else {
    cholesky_inverse_blocked(c, G, n, Linv, flag);
  }
}

bool expm_in_lds(const Ctx& c) { return c.nb <= 78; }

void launch_chol_expm_lds(Ctx& c, const double* G, double ga, double gd, double* Linv, int32_t* flag,
                          const double* D, double delta, double* U) {
  const int n = c.nb;
  const int inv = n <= 96 ? 1 : 0;
  const size_t lds = std::max((size_t)(inv ? 2 : 1) * n * chol_ld(n), (size_t)3 * n * n) * sizeof(double);
  allow_dynamic_lds(reinterpret_cast<const void*>(k_chol_expm_lds), lds);
  hipLaunchKernelGGL(k_chol_expm_lds, dim3(2), dim3(1024), lds, c.stream, G, ga, gd, n, Linv, flag, inv,
                     D, delta, U);
  ROKS_HIP(hipGetLastError());
}

void launch_expm_lds(Ctx& c, const double* D, double delta, double* U, hipStream_t stream) {
  const int n = c.nb;
  const size_t lds = (size_t)3 * n * n * sizeof(double);
  allow_dynamic_lds(reinterpret_cast<const void*>(k_expm_lds), lds);
  hipLaunchKernelGGL(k_expm_lds, dim3(1), dim3(1024), lds, stream, D, n, delta, U);
  ROKS_HIP(hipGetLastError());
}

void launch_subspace(Ctx& c, double* open_out) {
  SubArgs a{};
  a.nb = c.nb;
  a.nsocc = c.nsocc;
  a.flags = (int)c.flags;
  a.open_a = a.open_b = -1;
  int opens[kMaxShell], no = 0;
  for (int X = 0; X < c.nshell; ++X) {
    a.w[X] = c.shell_w[X];
    a.virt[X] = c.shell_virtual[X];
    if (!c.shell_closed[X] && !c.shell_virtual[X]) opens[no++] = X;
  }
  if (no == 2) {
    a.open_a = opens[0];
    a.open_b = opens[1];
  }
  const size_t nn = (size_t)c.nb * c.nb;
  // the open-shell coupling rides in one more workgroup when asked for
  double* oc = (open_out && a.open_a >= 0) ? open_out : nullptr;
  const unsigned nblk = (unsigned)((nn + 255) / 256) + (oc ? 1u : 0u);
  hipLaunchKernelGGL(k_subspace, dim3(nblk), dim3(256), 0, c.stream, a, c.d_theta, c.d_band_shell,
                     c.d_kin, c.d_enl, c.d_Q, c.d_R, c.d_kappa, c.d_A, oc);
  ROKS_HIP(hipGetLastError());
}

void launch_asym_dot(Ctx& c, const double* A, const double* theta, double* out, double* mirror) {
  hipLaunchKernelGGL(k_asym_dot, dim3(1), dim3(256), 0, c.stream, A, theta, c.nb, out, mirror);
  ROKS_HIP(hipGetLastError());
}

// sum over one 32 x 32 tile of A_mn (th_mn - th_nm), the transposed tile of
// th staged in LDS; one partial per tile, tiles row-major
__global__ void __launch_bounds__(256) k_asym_tiles(const double* __restrict__ A,
                                                    const double* __restrict__ th, int nb,
                                                    double* __restrict__ part) {
  __shared__ double tt[32][33];
  __shared__ double red[16];
  const int bi = blockIdx.y, bj = blockIdx.x;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows of 32 per pass
  // tt[r][c] = th[(bj 32 + r)][(bi 32 + c)]: rows of the mirrored tile
  for (int r = ty; r < 32; r += 8) {
    const int m = bj * 32 + r, n = bi * 32 + tx;
    tt[r][tx] = (m < nb && n < nb) ? th[(size_t)m * nb + n] : 0.0;
  }
  __syncthreads();
  double s = 0.0;
  for (int r = ty; r < 32; r += 8) {
    const int m = bi * 32 + r, n = bj * 32 + tx;
    if (m < nb && n < nb) s += A[(size_t)m * nb + n] * (th[(size_t)m * nb + n] - tt[tx][r]);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int w = 0; w < 4; ++w) v += red[w];
    part[(size_t)bi * gridDim.x + bj] = v;
  }
}

// out = sum of the np tile partials in order (also into mirror)
__global__ void k_sum_ordered(const double* __restrict__ part, int np, double* __restrict__ out,
                              double* __restrict__ mirror) {
  if (threadIdx.x != 0) return;
  double v = 0.0;
  for (int i = 0; i < np; ++i) v += part[i];
  if (out) out[0] = v;
  if (mirror) mirror[0] = v;
}

void band_dots_asym(Ctx& c, const double2* X, const double2* Y, int nvec, double* out0,
                    double* mirror0, const double* A, const double* theta, double* aout,
                    double* amirror) {
  if (c.nb <= 128) {
    hipLaunchKernelGGL(k_band_dots_asym, dim3(nvec + 1), dim3(1024), 0, c.stream, X, Y, c.npw, out0,
                       mirror0, A, theta, c.nb, aout, amirror);
    ROKS_HIP(hipGetLastError());
    return;
  }
  // many bands: the contraction over 32 x 32 tiles (coalesced transposed
  // reads through LDS) and an ordered sum of the tiles' partials
  if (nvec > 0) {
    hipLaunchKernelGGL(k_band_dots_asym, dim3(nvec), dim3(1024), 0, c.stream, X, Y, c.npw, out0,
                       mirror0, nullptr, theta, c.nb, aout, amirror);
    ROKS_HIP(hipGetLastError());
  }
  const int t = cdiv(c.nb, 32);
  hipLaunchKernelGGL(k_asym_tiles, dim3(t, t), dim3(256), 0, c.stream, A, theta, c.nb, c.d_gemm_part);
  ROKS_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(64), 0, c.stream, c.d_gemm_part, t * t, aout, amirror);
  ROKS_HIP(hipGetLastError());
}

void cg_directions_dev(Ctx& c, size_t n1, const double* p, const double* w, double* S, size_t n2,
                       const double* A, const double* Dold, double* D, const double* asym,
                       const double* pgb, double pg_old, double* beta_out) {
  hipLaunchKernelGGL(k_cg_directions, dim3(blocks_for(n1 + n2)), dim3(256), 0, c.stream, n1, p, w, S,
                     n2, A, Dold, D, asym, pgb, c.nb, pg_old, beta_out);
  ROKS_HIP(hipGetLastError());
}

void launch_teter(Ctx& c, const double* gTg, const double* gg, const double2* g, const double* bandw,
                  double2* out) {
  const size_t n = (size_t)c.nb * c.npw;
  hipLaunchKernelGGL(k_teter, dim3(blocks_for(n)), dim3(256), 0, c.stream, g, c.npw, c.nb, gTg, gg,
                     c.d_g2, bandw, out);
  ROKS_HIP(hipGetLastError());
}

}  // namespace roks
