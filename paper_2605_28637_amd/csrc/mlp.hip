// Learned rescaling of the Teter preconditioner K (Eq. prec_k).
//
// A 3-64-64-1 network with GELU (erf form) activations maps the features of
// a (band n, |G|^2 shell) pair to o; the preconditioner becomes s K with
// s = exp(2 tanh(o)) in [e^-2, e^2], so K stays negative definite.  The
// network is evaluated once per (band, distinct |G|^2) and shared by the G
// vectors of that shell.
//
// Weights: FP32 master copy (Adam updates it) and a BF16 copy that every
// evaluation reads; activations and accumulations are FP32, per-band loss
// sums FP64.  Training pairs are built from recorded iterates psi_i and the
// converged orbitals psi_inf, aligned within every occupation shell by the
// orthogonal polar factor of <psi_inf_m|psi_i,n> (Newton-Schulz iteration).
// Every reduction runs in a fixed order, so results are bit-reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "roks_internal.h"

namespace roks {

namespace {

constexpr int W = kMlpWidth;
constexpr int kW1 = 0, kB1 = kW1 + W * kMlpFeat, kW2 = kB1 + W, kB2 = kW2 + W * W, kW3 = kB2 + W,
              kB3 = kW3 + W;
static_assert(kB3 + 1 == kMlpParams, "flat parameter layout");

constexpr int kChunk = 1024;  // samples per gradient partial
constexpr int kTile = 32;     // samples per LDS tile of the gradient kernel

__device__ __forceinline__ float bf16_to_float(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}
// round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t float_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float gelu(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_prime(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * expf(-0.5f * z * z);
}
__device__ __forceinline__ float scale_of(float o) { return expf(2.0f * tanhf(o)); }

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void params_to_lds(const uint16_t* __restrict__ pb, float* sp) {
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) sp[i] = bf16_to_float(pb[i]);
  __syncthreads();
}

// --------------------------------------------------------------------------
// forward: one thread per sample, weights broadcast from LDS
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_forward(const uint16_t* __restrict__ pb,
                                                     const float* __restrict__ X, int S,
                                                     float* __restrict__ o_out,
                                                     float* __restrict__ s_out) {
  __shared__ float sp[kMlpParams];
  params_to_lds(pb, sp);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const float x0 = X[3 * (size_t)s], x1 = X[3 * (size_t)s + 1], x2 = X[3 * (size_t)s + 2];
  float h1[W];
#pragma unroll
  for (int j = 0; j < W; ++j) {
    float z = sp[kB1 + j];
    z = fmaf(sp[kW1 + 3 * j], x0, z);
    z = fmaf(sp[kW1 + 3 * j + 1], x1, z);
    z = fmaf(sp[kW1 + 3 * j + 2], x2, z);
    h1[j] = gelu(z);
  }
  float o = sp[kB3];
  for (int j = 0; j < W; ++j) {
    float z = sp[kB2 + j];
#pragma unroll
    for (int i = 0; i < W; ++i) z = fmaf(sp[kW2 + W * j + i], h1[i], z);
    o = fmaf(sp[kW3 + j], gelu(z), o);
  }
  if (o_out) o_out[s] = o;
  if (s_out) s_out[s] = scale_of(o);
}

// --------------------------------------------------------------------------
// backward of sum_s dout_s o_s, per sample: writes the activations the
// weight gradients contract over, feature-major [64][ld]
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_backward(const uint16_t* __restrict__ pb,
                                                      const float* __restrict__ X, int S, size_t ld,
                                                      const float* __restrict__ dout,
                                                      float* __restrict__ H1, float* __restrict__ DZ1,
                                                      float* __restrict__ DZ2,
                                                      float* __restrict__ HD3) {
  __shared__ float sp[kMlpParams];
  params_to_lds(pb, sp);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const float x0 = X[3 * (size_t)s], x1 = X[3 * (size_t)s + 1], x2 = X[3 * (size_t)s + 2];
  float z1[W], h1[W], dh[W];
#pragma unroll
  for (int j = 0; j < W; ++j) {
    float z = sp[kB1 + j];
    z = fmaf(sp[kW1 + 3 * j], x0, z);
    z = fmaf(sp[kW1 + 3 * j + 1], x1, z);
    z = fmaf(sp[kW1 + 3 * j + 2], x2, z);
    z1[j] = z;
    h1[j] = gelu(z);
    dh[j] = 0.0f;
  }
  const float d = dout[s];
  for (int j = 0; j < W; ++j) {
    float z = sp[kB2 + j];
#pragma unroll
    for (int i = 0; i < W; ++i) z = fmaf(sp[kW2 + W * j + i], h1[i], z);
    const float dz2 = d * sp[kW3 + j] * gelu_prime(z);
    DZ2[j * ld + s] = dz2;
    HD3[j * ld + s] = d * gelu(z);
#pragma unroll
    for (int i = 0; i < W; ++i) dh[i] = fmaf(sp[kW2 + W * j + i], dz2, dh[i]);
  }
#pragma unroll
  for (int i = 0; i < W; ++i) {
    DZ1[i * ld + s] = dh[i] * gelu_prime(z1[i]);
    H1[i * ld + s] = h1[i];
  }
}

// --------------------------------------------------------------------------
// weight-gradient partial of one chunk of kChunk samples, samples in order:
//   gW2 = DZ2^T H1 (4 x 4 outputs per thread), gb2 = sum DZ2, gw3 = sum HD3,
//   gW1 = DZ1^T X, gb1 = sum DZ1, gb3 = sum dout
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mlp_grad_partial(
    const float* __restrict__ X, const float* __restrict__ dout, int S, size_t ld,
    const float* __restrict__ H1, const float* __restrict__ DZ1, const float* __restrict__ DZ2,
    const float* __restrict__ HD3, float* __restrict__ part) {
  __shared__ float Ds[kTile][W + 4];
  __shared__ float Hs[kTile][W + 4];
  __shared__ float Es[kTile][W + 4];  // DZ1
  __shared__ float Gs[kTile][W + 4];  // HD3
  __shared__ float Xs[kTile][4];      // features and dout
  const int t = threadIdx.x;
  const int j0 = (t >> 4) * 4, i0 = (t & 15) * 4;
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = 0.0f;
  float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f, v3 = 0.0f;  // the vector gradients of thread t
  const int s_begin = blockIdx.x * kChunk;
  const int s_end = min(S, s_begin + kChunk);
  for (int s0 = s_begin; s0 < s_end; s0 += kTile) {
#pragma unroll
    for (int q = 0; q < (kTile * W) / 256; ++q) {
      const int idx = t + q * 256, f = idx / kTile, ss = idx % kTile, s = s0 + ss;
      const bool in = s < s_end;
      Ds[ss][f] = in ? DZ2[f * ld + s] : 0.0f;
      Hs[ss][f] = in ? H1[f * ld + s] : 0.0f;
      Es[ss][f] = in ? DZ1[f * ld + s] : 0.0f;
      Gs[ss][f] = in ? HD3[f * ld + s] : 0.0f;
    }
    if (t < kTile) {
      const int s = s0 + t;
      const bool in = s < s_end;
      Xs[t][0] = in ? X[3 * (size_t)s] : 0.0f;
      Xs[t][1] = in ? X[3 * (size_t)s + 1] : 0.0f;
      Xs[t][2] = in ? X[3 * (size_t)s + 2] : 0.0f;
      Xs[t][3] = in ? dout[s] : 0.0f;
    }
    __syncthreads();
    for (int ss = 0; ss < kTile; ++ss) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a[r] = Ds[ss][j0 + r];
        b[r] = Hs[ss][i0 + r];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = fmaf(a[r], b[q], acc[r][q]);
      if (t < W) {
        v0 += Ds[ss][t];
        v1 += Gs[ss][t];
      } else if (t < 2 * W) {
        const float e = Es[ss][t - W];
        v0 = fmaf(e, Xs[ss][0], v0);
        v1 = fmaf(e, Xs[ss][1], v1);
        v2 = fmaf(e, Xs[ss][2], v2);
        v3 += e;
      } else if (t == 2 * W) {
        v0 += Xs[ss][3];
      }
    }
    __syncthreads();
  }
  float* out = part + (size_t)blockIdx.x * kMlpParams;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) out[kW2 + (j0 + r) * W + i0 + q] = acc[r][q];
  if (t < W) {
    out[kB2 + t] = v0;
    out[kW3 + t] = v1;
  } else if (t < 2 * W) {
    const int j = t - W;
    out[kW1 + 3 * j] = v0;
    out[kW1 + 3 * j + 1] = v1;
    out[kW1 + 3 * j + 2] = v2;
    out[kB1 + j] = v3;
  } else if (t == 2 * W) {
    out[kB3] = v0;
  }
}

__global__ void k_mlp_grad_reduce(const float* __restrict__ part, int nchunk, float* __restrict__ g) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += part[(size_t)c * kMlpParams + p];
  g[p] = (float)acc;
}

// Adam (Kingma & Ba) with bias correction; refreshes the BF16 copy
__global__ void k_mlp_adam(float* __restrict__ p, uint16_t* __restrict__ pb, float* __restrict__ m,
                           float* __restrict__ v, const float* __restrict__ g, float lr, float bc1,
                           float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
  p[i] = pi;
  pb[i] = float_to_bf16(pi);
}

__global__ void k_mlp_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ pb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpParams) pb[i] = float_to_bf16(p[i]);
}

// per band segment (one wave): A = sum s alpha, B = sum s^2 beta, C = sum gamma
__global__ void __launch_bounds__(256) k_mlp_segments(const float* __restrict__ o,
                                                      const double* __restrict__ al,
                                                      const double* __restrict__ be,
                                                      const double* __restrict__ ga,
                                                      const int32_t* __restrict__ off, int nseg,
                                                      double* __restrict__ ABC,
                                                      double* __restrict__ Lseg,
                                                      int32_t* __restrict__ ok) {
  const int wave = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (wave >= nseg) return;
  double A = 0.0, B = 0.0, C = 0.0;
  for (int k = off[wave] + lane; k < off[wave + 1]; k += 64) {
    const double s = scale_of(o[k]);
    A += s * al[k];
    B += s * s * be[k];
    C += ga[k];
  }
  A = wave_sum_d(A);
  B = wave_sum_d(B);
  C = wave_sum_d(C);
  if (lane == 0) {
    ABC[3 * wave] = A;
    ABC[3 * wave + 1] = B;
    ABC[3 * wave + 2] = C;
    const bool g = (C > 0.0) && (B > 0.0);
    ok[wave] = g ? 1 : 0;
    Lseg[wave] = g ? 1.0 - A * A / (B * C) : 0.0;
  }
}

// mean loss over the segments with B, C > 0, and their count: out[0], out[1]
__global__ void __launch_bounds__(256) k_mlp_loss_total(const double* __restrict__ Lseg,
                                                        const int32_t* __restrict__ ok, int nseg,
                                                        double* __restrict__ out) {
  __shared__ double sl[256], sc[256];
  double l = 0.0, n = 0.0;
  for (int i = threadIdx.x; i < nseg; i += 256) {
    l += Lseg[i];
    n += ok[i];
  }
  sl[threadIdx.x] = l;
  sc[threadIdx.x] = n;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sl[threadIdx.x] += sl[threadIdx.x + w];
      sc[threadIdx.x] += sc[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sc[0] > 0.0 ? sl[0] / sc[0] : 0.0;
    out[1] = sc[0];
  }
}

// dL/do per sample: dL/ds = r (alpha B - A s beta), r = -2A/(B^2 C)/nvalid,
// ds/do = 2 s (1 - tanh(o)^2)
__global__ void k_mlp_dout(const float* __restrict__ o, const double* __restrict__ al,
                           const double* __restrict__ be, const int32_t* __restrict__ seg_of,
                           const double* __restrict__ ABC, const int32_t* __restrict__ ok,
                           const double* __restrict__ tot, int S, float* __restrict__ dout) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const int seg = seg_of[s];
  float d = 0.0f;
  if (ok[seg]) {
    const double A = ABC[3 * seg], B = ABC[3 * seg + 1], C = ABC[3 * seg + 2];
    const double r = -2.0 * A / (B * B * C) / tot[1];
    const float th = tanhf(o[s]);
    const double sc = scale_of(o[s]);
    const double dlds = r * (al[s] * B - A * sc * be[s]);
    d = (float)(dlds * sc * 2.0 * (1.0 - (double)th * th));
  }
  dout[s] = d;
}

// --------------------------------------------------------------------------
// inference support and training-pair construction (context side)
// --------------------------------------------------------------------------
// features [n][k][3] of band n and G shell k; valid[n] = the band has a
// nonzero gradient with positive E_ref and kinetic energy
__global__ void k_features(const double* __restrict__ gTg, const double* __restrict__ gg,
                           const double* __restrict__ ekin, const double* __restrict__ g2sh, int nb,
                           int nsh, float* __restrict__ feat, int32_t* __restrict__ valid) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * nsh) return;
  const int n = idx / nsh, k = idx - n * nsh;
  const double eref = gg[n] > 0.0 ? 1.5 * gTg[n] / gg[n] : 0.0;
  const bool ok = gg[n] > 0.0 && eref > 0.0 && ekin[n] > 0.0;
  float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
  if (ok) {
    x0 = (float)log1p(g2sh[k] / eref);
    x1 = (float)log(ekin[n]);
    x2 = (float)(0.5 * log(gg[n]));
  }
  feat[3 * (size_t)idx] = x0;
  feat[3 * (size_t)idx + 1] = x1;
  feat[3 * (size_t)idx + 2] = x2;
  if (k == 0) valid[n] = ok ? 1 : 0;
}

// Teter K (Eq. prec_k, reading R1) times the learned factor of (n, shell of G)
__global__ void k_teter_scaled(const double2* __restrict__ g, int npw, int nb,
                               const double* __restrict__ gTg, const double* __restrict__ gg,
                               const double* __restrict__ g2, const int32_t* __restrict__ gshell,
                               int nsh, const float* __restrict__ scale,
                               const int32_t* __restrict__ valid, const double* __restrict__ ratio,
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
        if (valid[n]) K *= (double)scale[(size_t)n * nsh + gshell[q]] * ratio[0];
        v = make_double2(K * g[t].x, K * g[t].y);
      }
    }
    out[t] = v;
  }
}

// per band, <K g|g> and <s K g|g> (without the common -2/E_ref factor's
// sign; both are positive sums)
__global__ void __launch_bounds__(1024) k_teter_norm(const double2* __restrict__ g, int npw,
                                                     const double* __restrict__ gTg,
                                                     const double* __restrict__ gg,
                                                     const double* __restrict__ g2,
                                                     const int32_t* __restrict__ gshell, int nsh,
                                                     const float* __restrict__ scale,
                                                     const int32_t* __restrict__ valid,
                                                     double* __restrict__ ab) {
  __shared__ double ra[16], rb[16];
  const int n = blockIdx.x;
  double a = 0.0, b = 0.0;
  if (valid[n]) {
    const double eref = 1.5 * gTg[n] / gg[n];
    const double2* x = g + (size_t)n * npw;
    const float* sc = scale + (size_t)n * nsh;
    for (int q = threadIdx.x; q < npw; q += blockDim.x) {
      const double t = g2[q] / eref;
      const double t2 = t * t;
      const double p = 27.0 + 18.0 * t + 12.0 * t2 + 8.0 * t2 * t;
      const double k = (q == 0 ? 1.0 : 2.0) * (2.0 / eref) * p / (p + 16.0 * t2 * t2) *
                       (x[q].x * x[q].x + x[q].y * x[q].y);
      a += k;
      b += (double)sc[gshell[q]] * k;
    }
  }
  a = wave_sum_d(a);
  b = wave_sum_d(b);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    ra[wid] = a;
    rb[wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      sa += ra[w];
      sb += rb[w];
    }
    ab[2 * n] = sa;
    ab[2 * n + 1] = sb;
  }
}

// one factor for all bands: sum <K g|g> / sum <s K g|g>, so the learned
// direction keeps the plain preconditioner's first-order energy change and
// its balance with the rotation step; the network sets the shape and the
// relative weights of the bands
__global__ void __launch_bounds__(256) k_norm_reduce(const double* __restrict__ ab, int nb,
                                                     double* __restrict__ ratio) {
  __shared__ double sa[256], sb[256];
  double a = 0.0, b = 0.0;
  for (int n = threadIdx.x; n < nb; n += 256) {
    a += ab[2 * n];
    b += ab[2 * n + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *ratio = (sa[0] > 0.0 && sb[0] > 0.0) ? sa[0] / sb[0] : 1.0;
}

// energy-norm moments of band n restricted to G shell k: every G weighted
// by h = |G|^2/2 + <n|T|n> (a diagonal model of the band's Hessian) and by
// the half-sphere factor (2 for the stored G != 0, 1 for G = 0); the G
// vectors of a shell in ascending order
__global__ void k_moments(const double2* __restrict__ Kg, const double2* __restrict__ dl, int npw,
                          int nb, int nsh, const int32_t* __restrict__ perm,
                          const int32_t* __restrict__ shoff, const double* __restrict__ g2,
                          const double* __restrict__ ekin, double* __restrict__ a,
                          double* __restrict__ b, double* __restrict__ c) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * nsh) return;
  const int n = idx / nsh, k = idx - n * nsh;
  const double2* x = Kg + (size_t)n * npw;
  const double2* y = dl + (size_t)n * npw;
  const double en = ekin[n];
  double sa = 0.0, sb = 0.0, sc = 0.0;
  for (int i = shoff[k]; i < shoff[k + 1]; ++i) {
    const int q = perm[i];
    const double w = (q == 0 ? 1.0 : 2.0) * (g2[q] + en);
    const double2 u = x[q], v = y[q];
    sa += w * (u.x * v.x + u.y * v.y);
    sb += w * (u.x * u.x + u.y * u.y);
    sc += w * (v.x * v.x + v.y * v.y);
  }
  a[idx] = sa;
  b[idx] = sb;
  c[idx] = sc;
}

__global__ void k_shell_mask(double* __restrict__ O, int nb, const int32_t* __restrict__ bshell) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nb * nb) return;
  const int m = idx / nb, n = idx - m * nb;
  if (bshell[m] != bshell[n]) O[idx] = 0.0;
}

// max |T - I| (one workgroup, fixed-order tree)
__global__ void __launch_bounds__(256) k_identity_dev(const double* __restrict__ T, int n,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n * n; i += 256) {
    const int r = i / n, c = i - r * n;
    m = fmax(m, fabs(T[i] - (r == c ? 1.0 : 0.0)));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// append the selected bands' (features, moments) to the training set as one
// segment (the iterate)
__global__ void k_gather_segments(const float* __restrict__ feat, const double* __restrict__ a,
                                  const double* __restrict__ b, const double* __restrict__ c,
                                  const int32_t* __restrict__ sel, int nsel, int nsh,
                                  float* __restrict__ Xd, double* __restrict__ ad,
                                  double* __restrict__ bd, double* __restrict__ cd,
                                  int32_t* __restrict__ seg_of, int seg_base) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nsel * nsh) return;
  const int j = idx / nsh, k = idx - j * nsh;
  const size_t src = (size_t)sel[j] * nsh + k;
  Xd[3 * (size_t)idx] = feat[3 * src];
  Xd[3 * (size_t)idx + 1] = feat[3 * src + 1];
  Xd[3 * (size_t)idx + 2] = feat[3 * src + 2];
  ad[idx] = a[src];
  bd[idx] = b[src];
  cd[idx] = c[src];
  seg_of[idx] = seg_base;
}

int grid_for(size_t n, int block) { return (int)std::max<size_t>(1, (n + block - 1) / block); }

// ---- network-side allocation ----
template <typename T>
T* malloc_mlp(Mlp& m, size_t count) {
  void* p = nullptr;
  size_t bytes = std::max<size_t>(16, count * sizeof(T));
  if (hipMalloc(&p, bytes) != hipSuccess) throw Error{ROKS_ERR_OOM, "hipMalloc failed"};
  ROKS_HIP(hipMemsetAsync(p, 0, bytes, m.stream));
  m.allocations.push_back({p, bytes});
  return static_cast<T*>(p);
}

void free_mlp_ptr(Mlp& m, void* p) {
  if (!p) return;
  for (size_t i = 0; i < m.allocations.size(); ++i)
    if (m.allocations[i].p == p) {
      ROKS_HIP(hipStreamSynchronize(m.stream));
      ROKS_HIP(hipFree(p));
      m.allocations.erase(m.allocations.begin() + (long)i);
      return;
    }
}

// splitmix64 (Steele, Lea & Flood 2014): the library's own seeded initialiser
uint64_t splitmix64(uint64_t& state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// training-set capacity: samples S (X, moments, segment index, scratch) and
// band segments
void reserve_samples(Mlp& m, int S_new, int nseg_new) {
  if (S_new > m.Scap) {
    int cap = std::max(S_new, 2 * m.Scap);
    cap = (cap + 255) / 256 * 256;
    float* X = malloc_mlp<float>(m, 3 * (size_t)cap);
    double* abg = malloc_mlp<double>(m, 3 * (size_t)cap);
    int32_t* seg = malloc_mlp<int32_t>(m, cap);
    if (m.S > 0) {
      ROKS_HIP(hipMemcpyAsync(X, m.d_X, 3 * (size_t)m.S * sizeof(float), hipMemcpyDeviceToDevice,
                              m.stream));
      for (int r = 0; r < 3; ++r)
        ROKS_HIP(hipMemcpyAsync(abg + (size_t)r * cap, m.d_abg + (size_t)r * m.Scap,
                                (size_t)m.S * sizeof(double), hipMemcpyDeviceToDevice, m.stream));
      ROKS_HIP(hipMemcpyAsync(seg, m.d_band_of, (size_t)m.S * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, m.stream));
    }
    free_mlp_ptr(m, m.d_X);
    free_mlp_ptr(m, m.d_abg);
    free_mlp_ptr(m, m.d_band_of);
    for (float** p : {&m.d_o, &m.d_do, &m.d_H1, &m.d_DZ2, &m.d_DZ1, &m.d_HD3}) {
      free_mlp_ptr(m, *p);
      *p = nullptr;
    }
    free_mlp_ptr(m, m.d_part);
    m.d_X = X;
    m.d_abg = abg;
    m.d_band_of = seg;
    m.Scap = cap;
    m.d_o = malloc_mlp<float>(m, cap);
    m.d_do = malloc_mlp<float>(m, cap);
    m.d_H1 = malloc_mlp<float>(m, (size_t)W * cap);
    m.d_DZ1 = malloc_mlp<float>(m, (size_t)W * cap);
    m.d_DZ2 = malloc_mlp<float>(m, (size_t)W * cap);
    m.d_HD3 = malloc_mlp<float>(m, (size_t)W * cap);
    m.part_cap = (size_t)((cap + kChunk - 1) / kChunk);
    m.d_part = malloc_mlp<float>(m, m.part_cap * kMlpParams);
  }
  if (nseg_new + 1 > (int)m.seg_cap) {
    const size_t cap = std::max<size_t>(nseg_new + 1, 2 * m.seg_cap);
    free_mlp_ptr(m, m.d_band_off);
    free_mlp_ptr(m, m.d_ABC);
    free_mlp_ptr(m, m.d_Lseg);
    free_mlp_ptr(m, m.d_ok);
    m.d_band_off = malloc_mlp<int32_t>(m, cap);
    m.d_ABC = malloc_mlp<double>(m, 3 * cap);
    m.d_Lseg = malloc_mlp<double>(m, cap);
    m.d_ok = malloc_mlp<int32_t>(m, cap);
    m.seg_cap = cap;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// network
// ---------------------------------------------------------------------------
void mlp_init(Mlp& m, const float* theta, uint64_t seed) {
  m.d_p = malloc_mlp<float>(m, kMlpParams);
  m.d_pb = malloc_mlp<uint16_t>(m, kMlpParams);
  m.d_m = malloc_mlp<float>(m, kMlpParams);
  m.d_v = malloc_mlp<float>(m, kMlpParams);
  m.d_g = malloc_mlp<float>(m, kMlpParams);
  m.d_loss = malloc_mlp<double>(m, 2);
  std::vector<float> h(kMlpParams);
  if (theta) {
    std::memcpy(h.data(), theta, kMlpParams * sizeof(float));
  } else {
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)); last layer scaled by 1e-2 and
    // b3 = 0, so the untrained network stays close to s = 1
    uint64_t st = seed;
    auto fill = [&](int off, int count, int fan, double extra) {
      const double bound = extra / std::sqrt((double)fan);
      for (int i = 0; i < count; ++i) {
        const double u = (double)(splitmix64(st) >> 11) * 0x1.0p-53;
        h[off + i] = (float)((2.0 * u - 1.0) * bound);
      }
    };
    fill(kW1, W * kMlpFeat, kMlpFeat, 1.0);
    fill(kB1, W, kMlpFeat, 1.0);
    fill(kW2, W * W, W, 1.0);
    fill(kB2, W, W, 1.0);
    fill(kW3, W, W, 1e-2);
    h[kB3] = 0.0f;
  }
  mlp_set_params(m, h.data());
}

void mlp_free(Mlp& m) {
  if (m.stream) (void)hipStreamSynchronize(m.stream);
  for (auto& a : m.allocations) (void)hipFree(a.p);
  m.allocations.clear();
  if (m.stream && m.own_stream) (void)hipStreamDestroy(m.stream);
  m.stream = nullptr;
}

void mlp_set_params(Mlp& m, const float* host) {
  for (int i = 0; i < kMlpParams; ++i)
    ROKS_CHECK(std::isfinite(host[i]), ROKS_ERR_NAN, "non-finite network parameter");
  ROKS_HIP(hipMemcpyAsync(m.d_p, host, kMlpParams * sizeof(float), hipMemcpyHostToDevice, m.stream));
  ROKS_HIP(hipMemsetAsync(m.d_m, 0, kMlpParams * sizeof(float), m.stream));
  ROKS_HIP(hipMemsetAsync(m.d_v, 0, kMlpParams * sizeof(float), m.stream));
  hipLaunchKernelGGL(k_mlp_to_bf16, dim3(grid_for(kMlpParams, 256)), dim3(256), 0, m.stream, m.d_p,
                     m.d_pb);
  ROKS_HIP(hipGetLastError());
  m.adam_t = 0;
  ROKS_HIP(hipStreamSynchronize(m.stream));
}

void mlp_forward(Mlp& m, const float* dX, int S, float* d_o, float* d_s, hipStream_t stream) {
  if (S <= 0) return;
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid_for(S, 256)), dim3(256), 0, stream, m.d_pb, dX, S,
                     d_o, d_s);
  ROKS_HIP(hipGetLastError());
}

void mlp_loss_grad(Mlp& m, double* d_out) {
  ROKS_CHECK(m.S > 0 && m.nseg > 0, ROKS_ERR_STATE, "the network has no training samples");
  const int S = m.S, nseg = m.nseg;
  const size_t ld = (size_t)m.Scap;
  double* al = m.d_abg;
  double* be = m.d_abg + ld;
  double* ga = m.d_abg + 2 * ld;
  mlp_forward(m, m.d_X, S, m.d_o, nullptr, m.stream);
  hipLaunchKernelGGL(k_mlp_segments, dim3(grid_for((size_t)nseg * 64, 256)), dim3(256), 0, m.stream,
                     m.d_o, al, be, ga, m.d_band_off, nseg, m.d_ABC, m.d_Lseg, m.d_ok);
  hipLaunchKernelGGL(k_mlp_loss_total, dim3(1), dim3(256), 0, m.stream, m.d_Lseg, m.d_ok, nseg,
                     d_out);
  hipLaunchKernelGGL(k_mlp_dout, dim3(grid_for(S, 256)), dim3(256), 0, m.stream, m.d_o, al, be,
                     m.d_band_of, m.d_ABC, m.d_ok, d_out, S, m.d_do);
  hipLaunchKernelGGL(k_mlp_backward, dim3(grid_for(S, 256)), dim3(256), 0, m.stream, m.d_pb, m.d_X,
                     S, ld, m.d_do, m.d_H1, m.d_DZ1, m.d_DZ2, m.d_HD3);
  const int nchunk = (S + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_mlp_grad_partial, dim3(nchunk), dim3(256), 0, m.stream, m.d_X, m.d_do, S, ld,
                     m.d_H1, m.d_DZ1, m.d_DZ2, m.d_HD3, m.d_part);
  hipLaunchKernelGGL(k_mlp_grad_reduce, dim3(grid_for(kMlpParams, 256)), dim3(256), 0, m.stream,
                     m.d_part, nchunk, m.d_g);
  ROKS_HIP(hipGetLastError());
}

void mlp_adam(Mlp& m, double lr) {
  m.adam_t++;
  const double bc1 = 1.0 - std::pow(0.9, m.adam_t);
  const double bc2 = 1.0 - std::pow(0.999, m.adam_t);
  hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(kMlpParams, 256)), dim3(256), 0, m.stream, m.d_p,
                     m.d_pb, m.d_m, m.d_v, m.d_g, (float)lr, (float)bc1, (float)bc2);
  ROKS_HIP(hipGetLastError());
}

void mlp_clear_samples(Mlp& m) {
  m.S = 0;
  m.nseg = 0;
  m.band_off.assign(1, 0);
}

// ---------------------------------------------------------------------------
// context side: G shells, features, scaled Teter, recording, collection
// ---------------------------------------------------------------------------
void build_gshells(Ctx& c) {
  if (c.nsh > 0) return;
  std::vector<int64_t> key(c.npw);
  for (int q = 0; q < c.npw; ++q) key[q] = std::llrint(c.g2half[q] * 1e9);
  std::vector<int32_t> order(c.npw);
  for (int q = 0; q < c.npw; ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  c.gshell.assign(c.npw, 0);
  c.sh_perm = order;
  c.sh_off.clear();
  c.g2sh.clear();
  for (int i = 0; i < c.npw; ++i) {
    if (i == 0 || key[order[i]] != key[order[i - 1]]) {
      c.sh_off.push_back(i);
      c.g2sh.push_back(c.g2half[order[i]]);
    }
    c.gshell[order[i]] = (int32_t)c.g2sh.size() - 1;
  }
  c.sh_off.push_back(c.npw);
  c.nsh = (int)c.g2sh.size();
  const int nb = c.nb, nsh = c.nsh;
  c.d_gshell = dalloc<int32_t>(c, c.npw);
  c.d_sh_perm = dalloc<int32_t>(c, c.npw);
  c.d_sh_off = dalloc<int32_t>(c, nsh + 1);
  c.d_g2sh = dalloc<double>(c, nsh);
  c.d_feat = dalloc<float>(c, 3 * (size_t)nb * nsh);
  c.d_scale = dalloc<float>(c, (size_t)nb * nsh);
  c.d_valid = dalloc<int32_t>(c, nb);
  c.d_mom = dalloc<double>(c, 3 * (size_t)nb * nsh);
  ROKS_HIP(hipMemcpyAsync(c.d_gshell, c.gshell.data(), c.npw * sizeof(int32_t),
                          hipMemcpyHostToDevice, c.stream));
  ROKS_HIP(hipMemcpyAsync(c.d_sh_perm, c.sh_perm.data(), c.npw * sizeof(int32_t),
                          hipMemcpyHostToDevice, c.stream));
  ROKS_HIP(hipMemcpyAsync(c.d_sh_off, c.sh_off.data(), (nsh + 1) * sizeof(int32_t),
                          hipMemcpyHostToDevice, c.stream));
  ROKS_HIP(hipMemcpyAsync(c.d_g2sh, c.g2sh.data(), nsh * sizeof(double), hipMemcpyHostToDevice,
                          c.stream));
  ROKS_HIP(hipStreamSynchronize(c.stream));
}

void launch_features(Ctx& c, const double* gTg, const double* gg, const double* ekin) {
  const int n = c.nb * c.nsh;
  hipLaunchKernelGGL(k_features, dim3(grid_for(n, 256)), dim3(256), 0, c.stream, gTg, gg, ekin,
                     c.d_g2sh, c.nb, c.nsh, c.d_feat, c.d_valid);
  ROKS_HIP(hipGetLastError());
}

void launch_teter_scaled(Ctx& c, const double* gTg, const double* gg, const double2* g,
                         const double* bandw, double2* out) {
  {
    KernelTimer kt(c, "mlp_forward", (double)kMlpParams * 2 + 16.0 * c.nb * c.nsh,
                   2.0 * (W * kMlpFeat + W * W + W) * (double)c.nb * c.nsh);
    mlp_forward(*c.mlp, c.d_feat, c.nb * c.nsh, nullptr, c.d_scale, c.stream);
  }
  double* ab = c.d_bandv + 4 * c.nb;  // [nb][2], after the features are taken
  double* ratio = c.d_bandv + 7 * c.nb;
  hipLaunchKernelGGL(k_teter_norm, dim3(c.nb), dim3(1024), 0, c.stream, g, c.npw, gTg, gg, c.d_g2,
                     c.d_gshell, c.nsh, c.d_scale, c.d_valid, ab);
  hipLaunchKernelGGL(k_norm_reduce, dim3(1), dim3(256), 0, c.stream, ab, c.nb, ratio);
  const size_t n = (size_t)c.nb * c.npw;
  const int blocks = (int)std::min<size_t>(8192, std::max<size_t>(1, (n + 255) / 256));
  hipLaunchKernelGGL(k_teter_scaled, dim3(blocks), dim3(256), 0, c.stream, g, c.npw, c.nb, gTg, gg,
                     c.d_g2, c.d_gshell, c.nsh, c.d_scale, c.d_valid, ratio, bandw, out);
  ROKS_HIP(hipGetLastError());
}

void record_iterate(Ctx& c, const double* gTg, const double* gg, const double* ekin) {
  const int r = c.rec_count;
  const size_t band = (size_t)c.nb * c.npw;
  const size_t fs = 3 * (size_t)c.nb * c.nsh;
  ROKS_HIP(hipMemcpyAsync(c.d_rec_psi + r * band, c.d_psi, band * sizeof(double2),
                          hipMemcpyDeviceToDevice, c.stream));
  launch_teter(c, gTg, gg, c.d_gI, nullptr, c.d_rec_kg + r * band);
  ROKS_HIP(hipMemcpyAsync(c.d_rec_feat + r * fs, c.d_feat, fs * sizeof(float),
                          hipMemcpyDeviceToDevice, c.stream));
  ROKS_HIP(hipMemcpyAsync(c.d_rec_valid + (size_t)r * c.nb, c.d_valid, c.nb * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, c.stream));
  ROKS_HIP(hipMemcpyAsync(c.d_rec_ekin + (size_t)r * c.nb, ekin, c.nb * sizeof(double),
                          hipMemcpyDeviceToDevice, c.stream));
  c.rec_count++;
}

void polar_factor(Ctx& c, double* X, int n, double* T, double* Xn, bool* converged) {
  // X_{k+1} = 3/2 X_k - 1/2 X_k X_k^T X_k: every singular value in (0, sqrt 3)
  // goes to 1 (the overlap of two orthonormal sets has them in [0, 1])
  // (quadratic once close); two more iterations after |X^T X - I| reaches
  // the rounding level of an n-term sum
  *converged = false;
  double dev = 1.0;
  int polish = -1;
  for (int it = 0; it < 120; ++it) {
    gemm_small(c, n, n, n, X, n, true, X, n, false, T, n, 1.0, 0.0);
    if (polish < 0 && it % 4 == 0) {
      hipLaunchKernelGGL(k_identity_dev, dim3(1), dim3(256), 0, c.stream, T, n, c.d_bandv + 5 * c.nb);
      ROKS_HIP(hipGetLastError());
      ROKS_HIP(hipMemcpyAsync(&dev, c.d_bandv + 5 * c.nb, sizeof(double), hipMemcpyDeviceToHost,
                              c.stream));
      ROKS_HIP(hipStreamSynchronize(c.stream));
      if (!std::isfinite(dev)) return;
      if (dev < 4e-15 * std::max(1, n)) polish = 2;
    }
    if (polish == 0) {
      *converged = true;
      return;
    }
    if (polish > 0) --polish;
    ROKS_HIP(hipMemcpyAsync(Xn, X, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice,
                            c.stream));
    gemm_small(c, n, n, n, X, n, false, T, n, false, Xn, n, -0.5, 1.5);
    ROKS_HIP(hipMemcpyAsync(X, Xn, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice,
                            c.stream));
  }
}

void collect_records(Ctx& c, Mlp& m, int* used, int* skipped) {
  *used = 0;
  *skipped = 0;
  if (c.rec_count == 0) return;
  ROKS_CHECK(c.have_orbitals, ROKS_ERR_STATE, "no converged orbitals are set");
  const int nb = c.nb, nsh = c.nsh, K = 2 * c.npw;
  const size_t band = (size_t)nb * c.npw, nn = (size_t)nb * nb;
  const size_t fs = 3 * (size_t)nb * nsh;
  std::vector<int32_t> valid(nb);
  int32_t* d_sel = c.d_rec_sel;
  for (int r = 0; r < c.rec_count; ++r) {
    const double2* psi_i = c.d_rec_psi + r * band;
    // O_mn = <psi_inf_m|psi_i,n> within each occupation shell, its polar factor Q
    gemm_wdot(c, nb, nb, K, reinterpret_cast<const double*>(c.d_psi), K,
              reinterpret_cast<const double*>(psi_i), K, c.d_m2, nb, 1.0, 0.0, true);
    hipLaunchKernelGGL(k_shell_mask, dim3(grid_for(nn, 256)), dim3(256), 0, c.stream, c.d_m2, nb,
                       c.d_band_shell);
    ROKS_HIP(hipGetLastError());
    bool conv = false;
    polar_factor(c, c.d_m2, nb, c.d_m3, c.d_m4, &conv);
    if (!conv) {
      (*skipped)++;
      continue;
    }
    // aligned_n = sum_m Q_mn psi_inf_m;  delta = (1 - P_i) aligned
    gemm_expand(c, nb, K, nb, c.d_m2, nb, false, reinterpret_cast<const double*>(c.d_psi), K,
                reinterpret_cast<double*>(c.d_w1), K, 1.0, 0.0);
    gemm_wdot(c, nb, nb, K, reinterpret_cast<const double*>(psi_i), K,
              reinterpret_cast<const double*>(c.d_w1), K, c.d_m1, nb, 1.0, 0.0, true);
    gemm_expand(c, nb, K, nb, c.d_m1, nb, false, reinterpret_cast<const double*>(psi_i), K,
                reinterpret_cast<double*>(c.d_w1), K, -1.0, 1.0);
    double* da = c.d_mom;
    double* db = c.d_mom + (size_t)nb * nsh;
    double* dc = c.d_mom + 2 * (size_t)nb * nsh;
    hipLaunchKernelGGL(k_moments, dim3(grid_for((size_t)nb * nsh, 128)), dim3(128), 0, c.stream,
                       c.d_rec_kg + r * band, c.d_w1, c.npw, nb, nsh, c.d_sh_perm, c.d_sh_off, c.d_g2,
                       c.d_rec_ekin + (size_t)r * nb, da, db, dc);
    ROKS_HIP(hipGetLastError());
    // bands with a usable gradient become segments of the training set
    ROKS_HIP(hipMemcpyAsync(valid.data(), c.d_rec_valid + (size_t)r * nb, nb * sizeof(int32_t),
                            hipMemcpyDeviceToHost, c.stream));
    ROKS_HIP(hipStreamSynchronize(c.stream));
    std::vector<int32_t> sel;
    for (int n = 0; n < nb; ++n)
      if (valid[n] && !c.shell_virtual[c.band_shell[n]]) sel.push_back(n);
    if (sel.empty()) {
      (*used)++;
      continue;
    }
    const int nsel = (int)sel.size();
    ROKS_HIP(hipStreamSynchronize(m.stream));
    reserve_samples(m, m.S + nsel * nsh, m.nseg + 1);
    ROKS_HIP(hipStreamSynchronize(m.stream));
    ROKS_HIP(hipMemcpyAsync(d_sel, sel.data(), nsel * sizeof(int32_t), hipMemcpyHostToDevice,
                            c.stream));
    const size_t ld = (size_t)m.Scap;
    hipLaunchKernelGGL(k_gather_segments, dim3(grid_for((size_t)nsel * nsh, 256)), dim3(256), 0,
                       c.stream, c.d_rec_feat + r * fs, da, db, dc, d_sel, nsel, nsh,
                       m.d_X + 3 * (size_t)m.S, m.d_abg + m.S, m.d_abg + ld + m.S,
                       m.d_abg + 2 * ld + m.S, m.d_band_of + m.S, m.nseg);
    ROKS_HIP(hipGetLastError());
    m.band_off.push_back(m.band_off.back() + nsel * nsh);
    m.S += nsel * nsh;
    m.nseg += 1;
    ROKS_HIP(hipMemcpyAsync(m.d_band_off, m.band_off.data(), (m.nseg + 1) * sizeof(int32_t),
                            hipMemcpyHostToDevice, c.stream));
    ROKS_HIP(hipStreamSynchronize(c.stream));
    (*used)++;
  }
  c.rec_count = 0;
}

}  // namespace roks
