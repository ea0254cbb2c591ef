// Batched 3D FFTs of Gamma-point bands for gfx950, staged in LDS, in FP64 or
// FP32 (the arithmetic tier of the context).
//
// One band pair (u1 + i u2, both real in r-space) is one complex transform.
// The G -> r direction runs in two kernels:
//   zpass_bwd  : gather the stored sphere into the full sphere's z-columns
//                (column and mirror column from the same half column) and
//                transform along z; writes T[pair][z][col].
//   plane pass : per z-plane, scatter the columns into an N1 x N2 plane in
//                LDS, transform along y (only the rows |h| <= hmax that hold
//                data) and along x, then either multiply by the band's local
//                potential and transform back (apply), or accumulate the
//                squared real / imaginary parts into per-shell densities.
// r -> G is zpass_fwd: transform along z, unpack the two bands with
// c(-G) = conj(c(G)), scale by 1/N^3 and add the kinetic term.
//
// All 1D transforms are in-place mixed-radix Stockham passes (radices 8, 4,
// 2, 3, 5): every thread stages the inputs of its butterflies in registers,
// the block synchronises, and the outputs are written back to the same LDS.
// Band coefficients in and out are FP64 in both tiers; the column buffer,
// the plane arithmetic and the potentials are in the tier's precision R.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <utility>

#include "roks_internal.h"

namespace roks {

namespace {

template <typename R>
struct CT;
template <>
struct CT<double> {
  using V = double2;
};
template <>
struct CT<float> {
  using V = float2;
};
template <typename R>
using C2 = typename CT<R>::V;

template <typename R>
__device__ __forceinline__ C2<R> mk(R x, R y) {
  C2<R> v;
  v.x = x;
  v.y = y;
  return v;
}
template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
  return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R>
__device__ __forceinline__ C2<R> cadd(C2<R> a, C2<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R>
__device__ __forceinline__ C2<R> csub(C2<R> a, C2<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
// multiply by s*i (s = +-1)
template <typename R>
__device__ __forceinline__ C2<R> cmuli(C2<R> a, int s) {
  return s > 0 ? mk<R>(-a.y, a.x) : mk<R>(a.y, -a.x);
}
template <typename R>
__device__ __forceinline__ C2<R> cscale(C2<R> a, R f) { return mk<R>(a.x * f, a.y * f); }

// DFT of length N with kernel exp(s 2 pi i r q / N), in place.
template <typename R, int N>
struct Dft;

template <typename R>
struct Dft<R, 2> {
  static __device__ __forceinline__ void run(C2<R>* v, int) {
    C2<R> a = v[0], b = v[1];
    v[0] = cadd<R>(a, b);
    v[1] = csub<R>(a, b);
  }
};

template <typename R>
struct Dft<R, 4> {
  static __device__ __forceinline__ void run(C2<R>* v, int s) {
    C2<R> a = cadd<R>(v[0], v[2]), b = csub<R>(v[0], v[2]);
    C2<R> c = cadd<R>(v[1], v[3]), d = cmuli<R>(csub<R>(v[1], v[3]), s);
    v[0] = cadd<R>(a, c);
    v[2] = csub<R>(a, c);
    v[1] = cadd<R>(b, d);
    v[3] = csub<R>(b, d);
  }
};

template <typename R>
struct Dft<R, 8> {
  static __device__ __forceinline__ void run(C2<R>* v, int s) {
    const R h = (R)0.70710678118654752440;
    C2<R> e[4] = {v[0], v[2], v[4], v[6]};
    C2<R> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<R, 4>::run(e, s);
    Dft<R, 4>::run(o, s);
    // w8^q = exp(s 2 pi i q / 8)
    C2<R> o1 = mk<R>(h * (o[1].x - s * o[1].y), h * (o[1].y + s * o[1].x));
    C2<R> o2 = cmuli<R>(o[2], s);
    C2<R> o3 = mk<R>(h * (-o[3].x - s * o[3].y), h * (-o[3].y + s * o[3].x));
    v[0] = cadd<R>(e[0], o[0]);
    v[4] = csub<R>(e[0], o[0]);
    v[1] = cadd<R>(e[1], o1);
    v[5] = csub<R>(e[1], o1);
    v[2] = cadd<R>(e[2], o2);
    v[6] = csub<R>(e[2], o2);
    v[3] = cadd<R>(e[3], o3);
    v[7] = csub<R>(e[3], o3);
  }
};

template <typename R>
struct Dft<R, 3> {
  static __device__ __forceinline__ void run(C2<R>* v, int s) {
    const R r3 = (R)0.86602540378443864676;  // sqrt(3)/2
    C2<R> t = cadd<R>(v[1], v[2]);
    C2<R> m = mk<R>(v[0].x - (R)0.5 * t.x, v[0].y - (R)0.5 * t.y);
    C2<R> d = cmuli<R>(cscale<R>(csub<R>(v[1], v[2]), r3), s);
    v[0] = cadd<R>(v[0], t);
    v[1] = cadd<R>(m, d);
    v[2] = csub<R>(m, d);
  }
};

template <typename R>
struct Dft<R, 5> {
  static __device__ __forceinline__ void run(C2<R>* v, int s) {
    const R c1 = (R)0.30901699437494742410, c2 = (R)-0.80901699437494742410;
    const R s1 = (R)0.95105651629515357212, s2 = (R)0.58778525229247312917;
    C2<R> t1 = cadd<R>(v[1], v[4]), t2 = cadd<R>(v[2], v[3]);
    C2<R> d1 = csub<R>(v[1], v[4]), d2 = csub<R>(v[2], v[3]);
    C2<R> a1 = mk<R>(v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y);
    C2<R> a2 = mk<R>(v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y);
    C2<R> b1 = cmuli<R>(mk<R>(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y), s);
    C2<R> b2 = cmuli<R>(mk<R>(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y), s);
    v[0] = cadd<R>(v[0], cadd<R>(t1, t2));
    v[1] = cadd<R>(a1, b1);
    v[4] = csub<R>(a1, b1);
    v[2] = cadd<R>(a2, b2);
    v[3] = csub<R>(a2, b2);
  }
};

struct Strided {
  int stride;
  __device__ int operator()(int l) const { return l * stride; }
};

// Row r of the pruned set maps to h = r - hmax (mod N1).
struct Rows {
  int hmax, n1, rowstride;
  __device__ int operator()(int r) const {
    int h = r - hmax;
    if (h < 0) h += n1;
    return h * rowstride;
  }
};

// One Stockham pass of radix RX over `nlines` lines of length N.
template <typename R, int RX, int MAXBF, typename LineMap>
__device__ __forceinline__ void fft_stage(C2<R>* buf, int N, int Ns, int nlines, LineMap lm,
                                          int estride, const C2<R>* tw, int sign) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int NR = N / RX;
  const int nbf = nlines * NR;
  const int twstep = N / (Ns * RX);
  C2<R> v[MAXBF][RX];
#pragma unroll
  for (int i = 0; i < MAXBF; ++i) {
    const int b = tid + i * nthr;
    if (b < nbf) {
      // lines fastest across lanes: neighbouring lanes hit neighbouring lines
      // (distinct banks for both unit-stride and padded-stride lines)
      const int t = b / nlines, line = b - t * nlines;
      const C2<R>* src = buf + lm(line);
#pragma unroll
      for (int r = 0; r < RX; ++r) v[i][r] = src[(t + r * NR) * estride];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXBF; ++i) {
    const int b = tid + i * nthr;
    if (b < nbf) {
      const int t = b / nlines, line = b - t * nlines;
      const int k = t % Ns;
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < RX; ++r) {
          C2<R> w = tw[k * r * twstep];  // exp(-2 pi i k r / (Ns RX))
          if (sign > 0) w.y = -w.y;
          v[i][r] = cmul<R>(v[i][r], w);
        }
      }
      Dft<R, RX>::run(v[i], sign);
      const int j = (t / Ns) * Ns * RX + k;
      C2<R>* dst = buf + lm(line);
#pragma unroll
      for (int r = 0; r < RX; ++r) dst[(j + r * Ns) * estride] = v[i][r];
    }
  }
  __syncthreads();
}

// The same pass with the length, the radix and the span Ns known at compile
// time: every index comes from shifts and masks, and the first pass (Ns = 1)
// has no twiddles.  Same arithmetic in the same order as fft_stage.
template <typename R, int RX, int MAXBF, int N, int NS, typename LineMap>
__device__ __forceinline__ void fft_stage_c(C2<R>* buf, int nlines, LineMap lm, int estride,
                                            const C2<R>* tw, int sign) {
  constexpr int NR = N / RX;
  constexpr int TWSTEP = N / (NS * RX);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nbf = nlines * NR;
  C2<R> v[MAXBF][RX];
#pragma unroll
  for (int i = 0; i < MAXBF; ++i) {
    const int b = tid + i * nthr;
    if (b < nbf) {
      const int t = b / nlines, line = b - t * nlines;
      const C2<R>* src = buf + lm(line);
#pragma unroll
      for (int r = 0; r < RX; ++r) v[i][r] = src[(t + r * NR) * estride];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MAXBF; ++i) {
    const int b = tid + i * nthr;
    if (b < nbf) {
      const int t = b / nlines, line = b - t * nlines;
      const int k = t % NS;
      if (NS > 1 && k != 0) {
#pragma unroll
        for (int r = 1; r < RX; ++r) {
          C2<R> w = tw[k * r * TWSTEP];  // exp(-2 pi i k r / (Ns RX))
          if (sign > 0) w.y = -w.y;
          v[i][r] = cmul<R>(v[i][r], w);
        }
      }
      Dft<R, RX>::run(v[i], sign);
      const int j = (t / NS) * NS * RX + k;
      C2<R>* dst = buf + lm(line);
#pragma unroll
      for (int r = 0; r < RX; ++r) dst[(j + r * NS) * estride] = v[i][r];
    }
  }
  __syncthreads();
}

// Plan classes a kernel is built for: length 64 (two radix-8 passes with
// compile-time indexing), or any length of radices 8, 4, 2, 3, 5.  The stages
// a kernel can meet are all inlined into its transform loop, and the general
// class needs about twice the registers.
constexpr int kLen64 = 1, kRadixAny = 0;

// Transform `nlines` lines in place; MAXP bounds ceil(nlines N / blockDim).
template <typename R, int MAXP, int RS, typename LineMap>
__device__ void fft_lines(C2<R>* buf, const FftPlan1D& plan, int nlines, LineMap lm, int estride,
                          const C2<R>* tw, int sign) {
  int Ns = 1;
  for (int s = 0; s < plan.nstages; ++s) {
    const int RX = plan.radix[s];
    if constexpr (RS == kLen64) {
      if (s == 0)
        fft_stage_c<R, 8, (MAXP + 7) / 8, 64, 1>(buf, nlines, lm, estride, tw, sign);
      else
        fft_stage_c<R, 8, (MAXP + 7) / 8, 64, 8>(buf, nlines, lm, estride, tw, sign);
    } else {
      switch (RX) {
        case 8: fft_stage<R, 8, (MAXP + 7) / 8>(buf, plan.n, Ns, nlines, lm, estride, tw, sign); break;
        case 4: fft_stage<R, 4, (MAXP + 3) / 4>(buf, plan.n, Ns, nlines, lm, estride, tw, sign); break;
        case 2: fft_stage<R, 2, (MAXP + 1) / 2>(buf, plan.n, Ns, nlines, lm, estride, tw, sign); break;
        case 3: fft_stage<R, 3, (MAXP + 2) / 3>(buf, plan.n, Ns, nlines, lm, estride, tw, sign); break;
        default: fft_stage<R, 5, (MAXP + 4) / 5>(buf, plan.n, Ns, nlines, lm, estride, tw, sign); break;
      }
    }
    Ns *= RX;
  }
}

__device__ __forceinline__ int wrap(int l, int n) {
  int r = l % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// z pass, G -> r
// ---------------------------------------------------------------------------
template <typename R, int MAXP, int RS>
__global__ void __launch_bounds__(512) k_zpass_bwd(const double2* __restrict__ vecs, int nvec,
                                                    int npw, const ColDesc* __restrict__ cols,
                                                    int ndesc, int nH, FftPlan1D plan,
                                                    const C2<R>* __restrict__ twg,
                                                    C2<R>* __restrict__ T, int ncol, int CH,
                                                    const double* __restrict__ skip) {
  // a set skip flag: the column buffer already holds this transform
  if (skip && skip[0] != 0.0) return;
  extern __shared__ char smem_raw[];
  C2<R>* smem = reinterpret_cast<C2<R>*>(smem_raw);
  const int N3 = plan.n, LS = N3 + 1;  // LDS line stride: N3 + 1 spreads the banks
  C2<R>* tw = smem;
  C2<R>* buf = smem + N3;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int pair = blockIdx.y;
  const int j0 = blockIdx.x * CH;
  const int n1 = 2 * pair, n2 = 2 * pair + 1;
  const double2* c1 = vecs + (size_t)n1 * npw;
  const double2* c2 = vecs + (size_t)n2 * npw;
  const bool has2 = n2 < nvec;
  for (int i = tid; i < N3; i += nthr) tw[i] = twg[i];
  for (int i = tid; i < 2 * CH * LS; i += nthr) buf[i] = mk<R>(0, 0);
  __syncthreads();
  for (int idx = tid; idx < CH * N3; idx += nthr) {
    const int c = idx / N3, e = idx - c * N3;
    const int j = j0 + c;
    if (j >= ndesc) continue;
    const ColDesc d = cols[j];
    if (e > d.lmax - d.lmin) continue;
    const int l = d.lmin + e;
    const int g = d.base + e;
    double2 a = c1[g];
    double2 b = has2 ? c2[g] : make_double2(0.0, 0.0);
    if (g == 0) a.y = b.y = 0.0;  // c(0) of a real orbital is real: Im c(0) is not read
    const C2<R> v = mk<R>((R)(a.x - b.y), (R)(a.y + b.x));    // c1 + i c2
    const C2<R> vm = mk<R>((R)(a.x + b.y), (R)(b.x - a.y));   // conj(c1) + i conj(c2)
    buf[(2 * c) * LS + wrap(l, N3)] = v;
    if (j > 0)
      buf[(2 * c + 1) * LS + wrap(-l, N3)] = vm;
    else if (l > 0)
      buf[(2 * c) * LS + wrap(-l, N3)] = vm;
  }
  __syncthreads();
  fft_lines<R, MAXP, RS>(buf, plan, 2 * CH, Strided{LS}, 1, tw, +1);
  for (int idx = tid; idx < CH * N3; idx += nthr) {
    const int z = idx / CH, c = idx - z * CH;
    const int j = j0 + c;
    if (j >= ndesc) continue;
    const size_t row = ((size_t)pair * N3 + z) * ncol;
    T[row + j] = buf[(2 * c) * LS + z];
    if (j > 0) T[row + nH + j] = buf[(2 * c + 1) * LS + z];
  }
}

// ---------------------------------------------------------------------------
// z pass, r -> G, with unpacking, scaling and the (FP64) kinetic term
// ---------------------------------------------------------------------------
template <typename R, int MAXP, int RS>
__global__ void __launch_bounds__(512) k_zpass_fwd(
    const C2<R>* __restrict__ T, int ncol, const ColDesc* __restrict__ cols, int ndesc, int nH,
    FftPlan1D plan, const C2<R>* __restrict__ twg, const double2* __restrict__ vecs, int nvec,
    int npw, const double* __restrict__ kinw, const double* __restrict__ g2, double scale,
    double2* __restrict__ Y, int CH) {
  extern __shared__ char smem_raw[];
  C2<R>* smem = reinterpret_cast<C2<R>*>(smem_raw);
  const int N3 = plan.n, LS = N3 + 1;  // LDS line stride: N3 + 1 spreads the banks
  C2<R>* tw = smem;
  C2<R>* buf = smem + N3;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int pair = blockIdx.y;
  const int j0 = blockIdx.x * CH;
  const int n1 = 2 * pair, n2 = 2 * pair + 1;
  const bool has2 = n2 < nvec;
  for (int i = tid; i < N3; i += nthr) tw[i] = twg[i];
  for (int idx = tid; idx < CH * N3; idx += nthr) {
    const int z = idx / CH, c = idx - z * CH;
    const int j = j0 + c;
    const size_t row = ((size_t)pair * N3 + z) * ncol;
    C2<R> s = mk<R>(0, 0), m = mk<R>(0, 0);
    if (j < ndesc) {
      s = T[row + j];
      if (j > 0) m = T[row + nH + j];
    }
    buf[(2 * c) * LS + z] = s;
    buf[(2 * c + 1) * LS + z] = m;
  }
  __syncthreads();
  fft_lines<R, MAXP, RS>(buf, plan, 2 * CH, Strided{LS}, 1, tw, -1);
  const double w1 = kinw[n1];
  const double w2 = has2 ? kinw[n2] : 0.0;
  for (int idx = tid; idx < CH * N3; idx += nthr) {
    const int c = idx / N3, e = idx - c * N3;
    const int j = j0 + c;
    if (j >= ndesc) continue;
    const ColDesc d = cols[j];
    if (e > d.lmax - d.lmin) continue;
    const int l = d.lmin + e;
    const int g = d.base + e;
    const C2<R> F = buf[(2 * c) * LS + wrap(l, N3)];
    const C2<R> Fm = (j == 0) ? buf[(2 * c) * LS + wrap(-l, N3)] : buf[(2 * c + 1) * LS + wrap(-l, N3)];
    const double y1x = 0.5 * ((double)F.x + (double)Fm.x), y1y = 0.5 * ((double)F.y - (double)Fm.y);
    const double ddx = 0.5 * ((double)F.x - (double)Fm.x), ddy = 0.5 * ((double)F.y + (double)Fm.y);
    const double k = g2[g];
    const double2 a = vecs[(size_t)n1 * npw + g];
    Y[(size_t)n1 * npw + g] = make_double2(scale * y1x + w1 * k * a.x, scale * y1y + w1 * k * a.y);
    if (has2) {
      const double2 b = vecs[(size_t)n2 * npw + g];
      // (F - conj Fm) / (2i)
      Y[(size_t)n2 * npw + g] = make_double2(scale * ddy + w2 * k * b.x, -scale * ddx + w2 * k * b.y);
    }
  }
}

// ---------------------------------------------------------------------------
// plane pass: scatter, y/x backward, potential multiply, x/y forward, gather
// ---------------------------------------------------------------------------
struct PlaneGeom {
  int N1, N2, N3, PS, hmax, ncol;
  FftPlan1D p1, p2;
};

template <typename R, int MAXP, int RS>
__global__ void __launch_bounds__(512) k_plane_apply(
    C2<R>* __restrict__ T, const int32_t* __restrict__ colpos, PlaneGeom g,
    const C2<R>* __restrict__ tw1g, const C2<R>* __restrict__ tw2g,
    const R* __restrict__ pot, int npot, size_t ntot, const int32_t* __restrict__ potidx,
    int nvec, int nQ, double* __restrict__ Qpart, int npairs, int per_chunk) {
  // The workgroup owns one z-plane and a chunk of band pairs.  The npot (<= 3)
  // potentials of its plane points stay in registers across the pairs; nQ > 0
  // also accumulates <n|V^X|n> for X < nQ from the same registers.
  extern __shared__ char smem_raw[];
  C2<R>* smem = reinterpret_cast<C2<R>*>(smem_raw);
  C2<R>* tw1 = smem;
  C2<R>* tw2 = smem + g.N1;
  C2<R>* plane = smem + g.N1 + g.N2;
  double* red = reinterpret_cast<double*>(plane + g.N1 * g.PS + 1);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int z = blockIdx.x, chunk = blockIdx.y;
  const int np2 = g.N1 * g.N2;
  const int nh = 2 * g.hmax + 1;
  const size_t zoff = (size_t)z * np2;
  for (int i = tid; i < g.N1; i += nthr) tw1[i] = tw1g[i];
  for (int i = tid; i < g.N2; i += nthr) tw2[i] = tw2g[i];
  R vr[3][MAXP];
#pragma unroll
  for (int X = 0; X < 3; ++X)
#pragma unroll
    for (int i = 0; i < MAXP; ++i) {
      const int pt = tid + i * nthr;
      vr[X][i] = (X < npot && pt < np2) ? pot[(size_t)X * ntot + zoff + pt] : (R)0;
    }
  const int p0 = chunk * per_chunk;
  const int p1 = min(npairs, p0 + per_chunk);
  for (int pair = p0; pair < p1; ++pair) {
    const int n1 = 2 * pair, n2 = 2 * pair + 1;
    for (int i = tid; i < g.N1 * g.PS; i += nthr) plane[i] = mk<R>(0, 0);
    __syncthreads();
    C2<R>* Tz = T + ((size_t)pair * g.N3 + z) * g.ncol;
    for (int col = tid; col < g.ncol; col += nthr)
      plane[colpos[2 * col] * g.PS + colpos[2 * col + 1]] = Tz[col];
    __syncthreads();
    fft_lines<R, MAXP, RS>(plane, g.p2, nh, Rows{g.hmax, g.N1, g.PS}, 1, tw2, +1);
    fft_lines<R, MAXP, RS>(plane, g.p1, g.N2, Strided{1}, g.PS, tw1, +1);
    const int s1 = potidx[n1];
    const int s2 = n2 < nvec ? potidx[n2] : -1;
    R q1[3] = {0, 0, 0}, q2[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < MAXP; ++i) {
      const int pt = tid + i * nthr;
      if (pt < np2) {
        const int x = pt / g.N2, y = pt - x * g.N2;
        C2<R>& w = plane[x * g.PS + y];
        const R u1 = w.x, u2 = w.y;
        R a = 0, b = 0;
#pragma unroll
        for (int X = 0; X < 3; ++X) {
          if (X < nQ) {
            q1[X] += vr[X][i] * u1 * u1;
            q2[X] += vr[X][i] * u2 * u2;
          }
          if (s1 == X) a = vr[X][i];
          if (s2 == X) b = vr[X][i];
        }
        w = mk<R>(a * u1, b * u2);
      }
    }
    __syncthreads();
    fft_lines<R, MAXP, RS>(plane, g.p1, g.N2, Strided{1}, g.PS, tw1, -1);
    fft_lines<R, MAXP, RS>(plane, g.p2, nh, Rows{g.hmax, g.N1, g.PS}, 1, tw2, -1);
    for (int col = tid; col < g.ncol; col += nthr)
      Tz[col] = plane[colpos[2 * col] * g.PS + colpos[2 * col + 1]];
    if (nQ > 0) {
      const int wid = tid >> 6, lane = tid & 63, nw = nthr >> 6;
#pragma unroll
      for (int X = 0; X < 3; ++X) {
        if (X < nQ) {
          const double t1 = wave_sum((double)q1[X]);
          const double t2 = wave_sum((double)q2[X]);
          if (lane == 0) {
            red[(2 * X) * nw + wid] = t1;
            red[(2 * X + 1) * nw + wid] = t2;
          }
        }
      }
      __syncthreads();
      if (tid < 2 * nQ) {
        double s = 0;
        for (int w = 0; w < nw; ++w) s += red[tid * nw + w];
        const int X = tid >> 1, b = tid & 1;
        // Qpart[pair][z][band b][X]
        Qpart[(((size_t)pair * g.N3 + z) * 2 + b) * nQ + X] = s;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// plane pass for densities: G -> r only, accumulate per-shell |u|^2
// ---------------------------------------------------------------------------
template <typename R, int MAXP, int RS>
__global__ void __launch_bounds__(512) k_plane_density(
    const C2<R>* __restrict__ T, const int32_t* __restrict__ colpos, PlaneGeom g,
    const C2<R>* __restrict__ tw1g, const C2<R>* __restrict__ tw2g,
    const int32_t* __restrict__ band_shell, int nvec, int nsocc, int npairs, int per_chunk,
    double* __restrict__ rho_part, size_t ntot) {
  extern __shared__ char smem_raw[];
  C2<R>* smem = reinterpret_cast<C2<R>*>(smem_raw);
  C2<R>* tw1 = smem;
  C2<R>* tw2 = smem + g.N1;
  C2<R>* plane = smem + g.N1 + g.N2;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int z = blockIdx.x, chunk = blockIdx.y;
  const int np2 = g.N1 * g.N2;
  const int nh = 2 * g.hmax + 1;
  for (int i = tid; i < g.N1; i += nthr) tw1[i] = tw1g[i];
  for (int i = tid; i < g.N2; i += nthr) tw2[i] = tw2g[i];
  // shell 0 (the closed shell, nearly every band) accumulates in registers;
  // the open shells (a band or two each) add into this chunk's slice of
  // rho_part in pair order
  const size_t zoff = (size_t)z * np2;
  R acc[MAXP];
#pragma unroll
  for (int i = 0; i < MAXP; ++i) acc[i] = 0;
  for (int X = 1; X < nsocc; ++X) {
    double* out = rho_part + ((size_t)chunk * nsocc + X) * ntot + zoff;
    for (int pt = tid; pt < np2; pt += nthr) out[pt] = 0.0;
  }
  const int p0 = chunk * per_chunk;
  const int p1 = min(npairs, p0 + per_chunk);
  for (int pair = p0; pair < p1; ++pair) {
    for (int i = tid; i < g.N1 * g.PS; i += nthr) plane[i] = mk<R>(0, 0);
    __syncthreads();
    const C2<R>* Tz = T + ((size_t)pair * g.N3 + z) * g.ncol;
    for (int col = tid; col < g.ncol; col += nthr)
      plane[colpos[2 * col] * g.PS + colpos[2 * col + 1]] = Tz[col];
    __syncthreads();
    fft_lines<R, MAXP, RS>(plane, g.p2, nh, Rows{g.hmax, g.N1, g.PS}, 1, tw2, +1);
    fft_lines<R, MAXP, RS>(plane, g.p1, g.N2, Strided{1}, g.PS, tw1, +1);
    const int s1 = band_shell[2 * pair];
    const int s2 = (2 * pair + 1 < nvec) ? band_shell[2 * pair + 1] : 99;
    const bool open1 = s1 >= 1 && s1 < nsocc, open2 = s2 >= 1 && s2 < nsocc;
#pragma unroll
    for (int i = 0; i < MAXP; ++i) {
      const int pt = tid + i * nthr;
      if (pt < np2) {
        const int x = pt / g.N2, y = pt - x * g.N2;
        const C2<R> w = plane[x * g.PS + y];
        acc[i] += (s1 == 0 ? w.x * w.x : (R)0) + (s2 == 0 ? w.y * w.y : (R)0);
        if (open1) rho_part[((size_t)chunk * nsocc + s1) * ntot + zoff + pt] += (double)(w.x * w.x);
        if (open2) rho_part[((size_t)chunk * nsocc + s2) * ntot + zoff + pt] += (double)(w.y * w.y);
      }
    }
    __syncthreads();
  }
  if (nsocc > 0) {
    double* out = rho_part + ((size_t)chunk * nsocc) * ntot + zoff;
#pragma unroll
    for (int i = 0; i < MAXP; ++i) {
      const int pt = tid + i * nthr;
      if (pt < np2) out[pt] = (double)acc[i];
    }
  }
}

// ---------------------------------------------------------------------------
// full-grid complex 3D FFT on [z][x][y] data (Hartree, V_ext, forces), FP64:
// one pass per axis.  Line c (of ncols) of batch b = blockIdx.y has element
// j at data[b bstride + j estr + c cstr]; a workgroup moves CH consecutive
// lines into LDS (line stride n + 1, so strided loads do not pile onto one
// bank), transforms them and writes them back.  Loads run along the
// contiguous direction: j when estr == 1, else c.
// ---------------------------------------------------------------------------
// Hartree step inside the z pass: after the forward transform of a z line,
// multiply by 4 pi / (|G|^2 N^3) (0 at G = 0) and transform back
struct HartreeMul {
  double b[3][3];  // reciprocal vectors (rows)
  int N[3];
  double inv;      // 1 / N^3
  int on;
};

template <int MAXP, int RS>
__global__ void __launch_bounds__(256) k_fft_axis(double2* __restrict__ data, FftPlan1D plan,
                                                  const double2* __restrict__ twg, int ncols, int CH,
                                                  long estr, long cstr, long bstride, int sign,
                                                  HartreeMul hm) {
  extern __shared__ char smem_raw[];
  double2* smem = reinterpret_cast<double2*>(smem_raw);
  const int L = plan.n, LS = L + 1;
  double2* tw = smem;
  double2* buf = smem + L;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int c0 = blockIdx.x * CH;
  double2* base = data + (size_t)blockIdx.y * bstride;
  const bool contig = estr == 1;
  for (int i = tid; i < L; i += nthr) tw[i] = twg[i];
  for (int idx = tid; idx < CH * L; idx += nthr) {
    int c, j;
    if (contig) {
      c = idx / L;
      j = idx - c * L;
    } else {
      j = idx / CH;
      c = idx - j * CH;
    }
    buf[c * LS + j] = (c0 + c < ncols) ? base[j * estr + (long)(c0 + c) * cstr] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  fft_lines<double, MAXP, RS>(buf, plan, CH, Strided{LS}, 1, tw, sign);
  if (hm.on) {
    // z lines: column c0 + c is (x, y) = divmod(c0 + c, N2), position j is z
    for (int idx = tid; idx < CH * L; idx += nthr) {
      const int j = idx / CH, c = idx - j * CH;
      const int p = c0 + c;
      const int x = p / hm.N[1], y = p - x * hm.N[1];
      const int f[3] = {2 * x >= hm.N[0] ? x - hm.N[0] : x, 2 * y >= hm.N[1] ? y - hm.N[1] : y,
                        2 * j >= hm.N[2] ? j - hm.N[2] : j};
      double G[3];
      for (int a = 0; a < 3; ++a) G[a] = f[0] * hm.b[0][a] + f[1] * hm.b[1][a] + f[2] * hm.b[2][a];
      const double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
      const double sc = g2 > 0.0 ? 4.0 * M_PI * hm.inv / g2 : 0.0;
      double2& v = buf[c * LS + j];
      v = make_double2(v.x * sc, v.y * sc);
    }
    __syncthreads();
    fft_lines<double, MAXP, RS>(buf, plan, CH, Strided{LS}, 1, tw, -sign);
  }
  for (int idx = tid; idx < CH * L; idx += nthr) {
    int c, j;
    if (contig) {
      c = idx / L;
      j = idx - c * L;
    } else {
      j = idx / CH;
      c = idx - j * CH;
    }
    if (c0 + c < ncols) base[j * estr + (long)(c0 + c) * cstr] = buf[c * LS + j];
  }
}

// x and y transforms of whole z-planes of [z][x][y] data in one pass: a
// workgroup loads plane blockIdx.x (contiguous) into LDS with row stride PS,
// transforms its y lines and x lines (y first when yfirst, else x first) and
// writes it back.  Per line the same butterflies as the axis passes.
template <int MAXP, int RS>
__global__ void __launch_bounds__(512) k_fft_plane(double2* __restrict__ data, FftPlan1D px,
                                                   FftPlan1D py, const double2* __restrict__ twx,
                                                   const double2* __restrict__ twy, int PS, int sign,
                                                   int yfirst) {
  extern __shared__ char smem_raw[];
  double2* smem = reinterpret_cast<double2*>(smem_raw);
  const int N0 = px.n, N1 = py.n, np2 = N0 * N1;
  double2* tx = smem;
  double2* ty = smem + N0;
  double2* plane = smem + N0 + N1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  double2* base = data + (size_t)blockIdx.x * np2;
  for (int i = tid; i < N0; i += nthr) tx[i] = twx[i];
  for (int i = tid; i < N1; i += nthr) ty[i] = twy[i];
  for (int p = tid; p < np2; p += nthr) {
    const int x = p / N1, y = p - x * N1;
    plane[x * PS + y] = base[p];
  }
  __syncthreads();
  if (yfirst) {
    fft_lines<double, MAXP, RS>(plane, py, N0, Strided{PS}, 1, ty, sign);
    fft_lines<double, MAXP, RS>(plane, px, N1, Strided{1}, PS, tx, sign);
  } else {
    fft_lines<double, MAXP, RS>(plane, px, N1, Strided{1}, PS, tx, sign);
    fft_lines<double, MAXP, RS>(plane, py, N0, Strided{PS}, 1, ty, sign);
  }
  for (int p = tid; p < np2; p += nthr) {
    const int x = p / N1, y = p - x * N1;
    base[p] = plane[x * PS + y];
  }
}

// ---------------------------------------------------------------------------
// plane pass with the lines in registers ("line kernels")
//
// For square planes N1 = N2 = N = G P (G a power of two, P <= 16) the plane
// work of a band pair runs on a pruned intermediate: only the nh = 2 hmax + 1
// rows |h| <= hmax ever hold data, so LDS holds nh x N values (not N x N).
//   y inverse : per row h, the length-N transform along k;
//   x phase   : per column y, the length-N transform along h (nh nonzero
//               inputs), the potential multiply (apply) or |u|^2 (density),
//               and for apply the forward transform, keeping rows |h| <= hmax;
//   y forward : per row, back along k (apply).
// Each line is owned by a group of G consecutive lanes, each lane holding P
// points in registers: the four-step split N = G x P, a length-P transform in
// registers, the twiddle exp(+-2 pi i t k / N), and a length-G transform
// across the group's lanes as a radix-2 network on lane shuffles (decimation
// in frequency: lane l ends with the outputs k + P bitrev(l)).  The forward
// transform is the exact conjugate transpose of the inverse (the network run
// backwards), so it takes its input in the order the inverse leaves it.  No
// stage barrier inside a line; three workgroup barriers per pair.
// ---------------------------------------------------------------------------
template <int P>
struct RegFac {
  // the first factor of a composite length: the largest of 8, 4, 2 dividing
  // it (3 or 5 for odd lengths)
  static constexpr int A = (P % 8 == 0 && P > 8) ? 8 : (P % 4 == 0 && P > 4) ? 4 : (P % 2 == 0 && P > 2) ? 2
                           : (P % 3 == 0 && P > 3) ? 3 : (P % 5 == 0 && P > 5) ? 5 : P;
};

// length-P DFT of v (kernel exp(s 2 pi i n k / P)) in registers; tw[m] =
// exp(-2 pi i m / Ntw) with Ntw = P * tws
template <typename R, int P, int A = RegFac<P>::A>
struct RegDft {
  static constexpr int B = P / A;
  static __device__ __forceinline__ void run(C2<R>* v, int s, const C2<R>* tw, int tws) {
    // n = B n1 + n2, k = k1 + A k2
    C2<R> y[B][A];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      C2<R> a[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) a[n1] = v[B * n1 + n2];
      RegDft<R, A>::run(a, s, tw, tws * B);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        C2<R> w = tw[(n2 * k1) * tws];
        if (s > 0) w.y = -w.y;
        y[n2][k1] = (n2 * k1 == 0) ? a[k1] : cmul<R>(a[k1], w);
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      C2<R> b[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) b[n2] = y[n2][k1];
      RegDft<R, B>::run(b, s, tw, tws * A);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = b[k2];
    }
  }
};
template <typename R, int P>
struct RegDft<R, P, P> {
  static __device__ __forceinline__ void run(C2<R>* v, int s, const C2<R>*, int) {
    if constexpr (P > 1) Dft<R, P>::run(v, s);
  }
};

// The lanes of a line group carry a logical index t (the butterfly
// position) that differs from the physical lane p: p = t0 ^ 2 t1 ^ 7 t2 ^
// 8 t3 for t = t0 + 2 t1 + 4 t2 + 8 t3 (a linear map over GF(2), so the
// partner of t along logical bit m is the physical lane p ^ mask(m), mask =
// 1, 2, 7, 8).  Each partner is then one DPP move per dword: quad
// permutations for 1 and 2, row_half_mirror (lane i reads 7 - i within its
// eight) for 7, row_ror:8 (lane i reads (i + 8) mod 16) for 8; the plain
// xor by 4 or 8 would take two moves with bank masks.
template <int G>
__device__ __forceinline__ int logical_lane(int p) {
  if constexpr (G >= 8) {
    const int c = (p >> 2) & 1;  // only mask 7 sets physical bit 2
    const int q = p ^ (c ? 7 : 0);
    return (q & 3) | (c << 2) | (q & 8);
  } else {
    return p;
  }
}

// the value held by the partner along logical bit m in {1, 2, 4, 8}
__device__ __forceinline__ int partner(int v, int m) {
  switch (m) {
    case 1: return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
    case 2: return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
    case 4: return __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    default: return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, true); // row_ror:8
  }
}
__device__ __forceinline__ float partner(float v, int m) {
  return __int_as_float(partner(__float_as_int(v), m));
}
__device__ __forceinline__ double partner(double v, int m) {
  const int lo = partner(__double2loint(v), m);
  const int hi = partner(__double2hiint(v), m);
  return __hiloint2double(hi, lo);
}
template <typename R>
__device__ __forceinline__ C2<R> partner2(C2<R> v, int m) {
  return mk<R>(partner(v.x, m), partner(v.y, m));
}

// one line of length N = G P over the G lanes of a group (t: lane in group)
template <typename R, int G, int P>
struct LineFft {
  static constexpr int N = G * P;
  // G->r, kernel exp(+2 pi i h x / N): on entry v[j] = in[t + G j]; on exit
  // v[k] = out[k + P bitrev(t)]
  static __device__ __forceinline__ void inv(C2<R>* v, int t, const C2<R>* tw0) {
    // the twiddles are re-read from LDS for every line (an opaque offset keeps
    // the compiler from holding all of them in registers across the pairs)
    int o = 0;
    asm volatile("" : "+v"(o));
    const C2<R>* tw = tw0 + o;
    RegDft<R, P>::run(v, +1, tw, G);
#pragma unroll
    for (int k = 1; k < P; ++k) {
      C2<R> w = tw[t * k];
      w.y = -w.y;
      v[k] = cmul<R>(v[k], w);
    }
    // radix-2 stages across the lanes, without branches: a lane with bit h
    // clear keeps v + p, one with it set (p - v) w, as (p + sg v) w' with
    // sg = +-1 and w' = 1 or w
#pragma unroll
    for (int h = G / 2; h >= 1; h /= 2) {
      const bool hi = (t & h) != 0;
      C2<R> w = tw[(t % h) * (G / (2 * h)) * P];
      w.y = -w.y;
      const R sg = hi ? (R)-1 : (R)1;
      const C2<R> wl = hi ? w : mk<R>(1, 0);
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const C2<R> p = partner2<R>(v[k], h);
        const C2<R> d = mk<R>(fma(sg, v[k].x, p.x), fma(sg, v[k].y, p.y));
        v[k] = cmul<R>(d, wl);
      }
    }
  }
  // r->G, kernel exp(-2 pi i h x / N), the conjugate transpose of inv: on
  // entry v[k] = in[k + P bitrev(t)]; on exit v[j] = out[t + G j]
  static __device__ __forceinline__ void fwd(C2<R>* v, int t, const C2<R>* tw0) {
    int o = 0;
    asm volatile("" : "+v"(o));
    const C2<R>* tw = tw0 + o;
    // the transposed stages: bit clear v + w p, bit set p - w v, as
    // al v + be p with (al, be) = (1, w) or (-w, 1)
#pragma unroll
    for (int h = 1; h < G; h *= 2) {
      const bool hi = (t & h) != 0;
      const C2<R> w = tw[(t % h) * (G / (2 * h)) * P];
      const C2<R> al = hi ? mk<R>(-w.x, -w.y) : mk<R>(1, 0);
      const C2<R> be = hi ? mk<R>(1, 0) : w;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const C2<R> p = partner2<R>(v[k], h);
        const C2<R> a = v[k];
        v[k] = mk<R>(fma(be.x, p.x, fma(-be.y, p.y, fma(al.x, a.x, -al.y * a.y))),
                     fma(be.x, p.y, fma(be.y, p.x, fma(al.x, a.y, al.y * a.x))));
      }
    }
#pragma unroll
    for (int k = 1; k < P; ++k) v[k] = cmul<R>(v[k], tw[t * k]);
    RegDft<R, P>::run(v, -1, tw, G);
  }
};

template <int G>
__device__ __forceinline__ int bitrev_lane(int t) {
  int r = 0;
#pragma unroll
  for (int b = 1; b < G; b <<= 1) r = (r << 1) | ((t & b) ? 1 : 0);
  return r;
}

constexpr int kModeApply = 0, kModeDensity = 1, kModeDensityOpen = 2;

struct LineGeom {
  int N3, PS, hmax, ncol;
};

// MODE apply: T is transformed in place (F: potential multiply of each band
// by its potential grid, potidx; nQ > 0 also accumulates <n|V^X|n>, X < nQ,
// into Qpart).  MODE density: pairs without an open-shell band, the closed
// shell's |u|^2 summed in registers into rho_part slice (chunk, 0), the open
// slices of the chunk zeroed.  MODE density-open (one chunk, run after it):
// the pairs holding an open-shell band, each band added into its shell's
// slice of chunk 0.
template <typename R, int G, int P, int MODE, int NT>
__global__ void __launch_bounds__(NT, 512 / NT) k_plane_lines(
    C2<R>* __restrict__ T, const int32_t* __restrict__ colidx, const int2* __restrict__ krange,
    LineGeom g, const C2<R>* __restrict__ twg, const R* __restrict__ pot, size_t ntot,
    const int32_t* __restrict__ potidx, int nvec, int nQ, double* __restrict__ Qpart,
    const int32_t* __restrict__ band_shell, int nsocc, double* __restrict__ rho_part, int pair0,
    int pair_end, int per_chunk) {
  constexpr int N = G * P;
  constexpr int NGRP = NT / G;        // line groups per workgroup
  constexpr int RHO = (N + NGRP - 1) / NGRP;    // x-phase columns per group
  constexpr int NW = NT / 64;
  extern __shared__ char smem_raw[];
  C2<R>* tw = reinterpret_cast<C2<R>*>(smem_raw);
  C2<R>* buf = tw + N;
  const int nh = 2 * g.hmax + 1;
  const int PS = g.PS;
  double* red = reinterpret_cast<double*>(buf + (size_t)nh * PS);  // [6][NW]
  int2* kr = reinterpret_cast<int2*>(red + 6 * NW);                 // [nh]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int t = logical_lane<G>(lane & (G - 1));
  const int grp = tid / G;
  const int brt = bitrev_lane<G>(t);
  const int z = blockIdx.x, chunk = blockIdx.y;
  const size_t zoff = (size_t)z * N * N;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  for (int i = tid; i < nh; i += NT) kr[i] = krange[i];
  const int p0 = pair0 + chunk * per_chunk;
  const int p1 = min(pair_end, p0 + per_chunk);
  double acc[MODE == kModeDensity ? RHO : 1][MODE == kModeDensity ? P : 1];  // closed-shell sum
  if constexpr (MODE == kModeDensity) {
#pragma unroll
    for (int q = 0; q < RHO; ++q)
#pragma unroll
      for (int k = 0; k < P; ++k) acc[q][k] = 0.0;
    for (int X = 1; X < nsocc; ++X) {
      double* out = rho_part + ((size_t)chunk * nsocc + X) * ntot + zoff;
      for (int pt = tid; pt < N * N; pt += NT) out[pt] = 0.0;
    }
  }
  C2<R>* Tprev = nullptr;
  for (int pair = p0; pair < p1; ++pair) {
    if constexpr (MODE == kModeDensity) {
      const int a = band_shell[2 * pair];
      const int b = 2 * pair + 1 < nvec ? band_shell[2 * pair + 1] : 99;
      if ((a >= 1 && a < nsocc) || (b >= 1 && b < nsocc)) continue;  // uniform
    }
    C2<R>* Tz = T + ((size_t)pair * g.N3 + z) * g.ncol;
    // the previous pair's result out, this pair's columns in (each position
    // belongs to one column, so one thread does both)
    for (int col = tid; col < g.ncol; col += NT) {
      const int at = colidx[col];
      if (MODE == kModeApply && Tprev) Tprev[col] = buf[at];
      buf[at] = Tz[col];
    }
    Tprev = Tz;
    __syncthreads();
    // y inverse, row r = h + hmax; positions outside the row's k range are zero
    for (int r = grp; r < nh; r += NGRP) {
      const int2 kk = kr[r];
      C2<R> v[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int k = t + G * j;
        const int ks = 2 * k > N ? k - N : k;
        const C2<R> b = buf[r * PS + k];
        const bool in = ks >= kk.x && ks <= kk.y;
        v[j] = mk<R>(in ? b.x : (R)0, in ? b.y : (R)0);
      }
      LineFft<R, G, P>::inv(v, t, tw);
#pragma unroll
      for (int k = 0; k < P; ++k) buf[r * PS + k + P * brt] = v[k];
    }
    __syncthreads();
    // x phase, column y
    const int n1 = 2 * pair, n2 = 2 * pair + 1;
    int s1 = 0, s2 = 0;
    if constexpr (MODE == kModeApply) {
      s1 = potidx[n1];
      s2 = n2 < nvec ? potidx[n2] : -1;
    } else {
      s1 = band_shell[n1];
      s2 = n2 < nvec ? band_shell[n2] : 99;
    }
    R q1[3] = {0, 0, 0}, q2[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < RHO; ++q) {
      const int y = grp + NGRP * q;
      if (RHO * NGRP == N || y < N) {
        C2<R> v[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const int h = t + G * j;
          const int hs = 2 * h > N ? h - N : h;
          const bool in = hs >= -g.hmax && hs <= g.hmax;
          const C2<R> b = buf[(in ? hs + g.hmax : 0) * PS + y];
          v[j] = mk<R>(in ? b.x : (R)0, in ? b.y : (R)0);
        }
        LineFft<R, G, P>::inv(v, t, tw);
        if constexpr (MODE == kModeApply) {
#pragma unroll
          for (int k = 0; k < P; ++k) {
            const int x = k + P * brt;
            const size_t pt = zoff + (size_t)x * N + y;
            const R u1 = v[k].x, u2 = v[k].y;
            const R a = s1 >= 0 ? pot[(size_t)s1 * ntot + pt] : (R)0;
            const R b = s2 >= 0 ? (s2 == s1 ? a : pot[(size_t)s2 * ntot + pt]) : (R)0;
            if (nQ > 0) {
#pragma unroll
              for (int X = 0; X < 3; ++X) {
                if (X < nQ) {
                  const R vx = X == s1 ? a : (X == s2 ? b : pot[(size_t)X * ntot + pt]);
                  q1[X] += vx * u1 * u1;
                  q2[X] += vx * u2 * u2;
                }
              }
            }
            v[k] = mk<R>(a * u1, b * u2);
          }
          LineFft<R, G, P>::fwd(v, t, tw);
#pragma unroll
          for (int j = 0; j < P; ++j) {
            const int h = t + G * j;
            const int hs = 2 * h > N ? h - N : h;
            if (hs >= -g.hmax && hs <= g.hmax) buf[(hs + g.hmax) * PS + y] = v[j];
          }
        } else if constexpr (MODE == kModeDensity) {
          const double w1 = s1 == 0 ? 1.0 : 0.0, w2 = s2 == 0 ? 1.0 : 0.0;
#pragma unroll
          for (int k = 0; k < P; ++k) {
            const double u1 = (double)v[k].x, u2 = (double)v[k].y;
            acc[q][k] += w1 * u1 * u1 + w2 * u2 * u2;
          }
        } else {
          // open pairs (one or two per system): every band of the pair adds
          // into its shell's slice of chunk 0 (after the closed-pair launch)
#pragma unroll
          for (int k = 0; k < P; ++k) {
            const int x = k + P * brt;
            const size_t pt = zoff + (size_t)x * N + y;
            const double u1 = (double)v[k].x, u2 = (double)v[k].y;
            if (s1 >= 0 && s1 < nsocc) rho_part[(size_t)s1 * ntot + pt] += u1 * u1;
            if (s2 >= 0 && s2 < nsocc) rho_part[(size_t)s2 * ntot + pt] += u2 * u2;
          }
        }
      }
      // one column at a time: interleaving the unrolled columns would hold
      // several lines in registers
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (MODE == kModeApply) {
      if (nQ > 0) {
#pragma unroll
        for (int X = 0; X < 3; ++X) {
          if (X < nQ) {
            const double t1 = wave_sum((double)q1[X]);
            const double t2 = wave_sum((double)q2[X]);
            if (lane == 0) {
              red[(2 * X) * NW + wid] = t1;
              red[(2 * X + 1) * NW + wid] = t2;
            }
          }
        }
      }
      __syncthreads();
      if (nQ > 0 && tid < 2 * nQ) {
        double s = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += red[tid * NW + w];
        const int X = tid >> 1, b = tid & 1;
        Qpart[(((size_t)pair * g.N3 + z) * 2 + b) * nQ + X] = s;
      }
      // y forward: the row as the inverse left it
      for (int r = grp; r < nh; r += NGRP) {
        C2<R> v[P];
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = buf[r * PS + k + P * brt];
        LineFft<R, G, P>::fwd(v, t, tw);
#pragma unroll
        for (int j = 0; j < P; ++j) buf[r * PS + t + G * j] = v[j];
      }
    }
    __syncthreads();
  }
  if constexpr (MODE == kModeApply) {
    if (Tprev)
      for (int col = tid; col < g.ncol; col += NT) Tprev[col] = buf[colidx[col]];
  } else if constexpr (MODE == kModeDensity) {
    if (nsocc > 0) {
      double* out = rho_part + ((size_t)chunk * nsocc) * ntot + zoff;
#pragma unroll
      for (int q = 0; q < RHO; ++q) {
        const int y = grp + NGRP * q;
        if (RHO * NGRP == N || y < N) {
#pragma unroll
          for (int k = 0; k < P; ++k) out[(size_t)(k + P * brt) * N + y] = acc[q][k];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
// 512 threads keep every thread at <= 8 (N <= 64) or <= 18 (N <= 96) points
// per FFT pass, so the butterfly registers fit without spilling
constexpr int kZThreads = 512;
int plane_threads(const Ctx& c) { return c.N[0] * c.N[1] > 1024 ? 512 : 256; }

int needed_points(int points, int nthr) { return (points + nthr - 1) / nthr; }

int pick_maxp(int need) {
  ROKS_CHECK(need <= 32, ROKS_ERR_SHAPE, "FFT plane too large for the LDS kernels");
  if (need <= 8) return 8;
  if (need <= 16) return 16;
  if (need <= 24) return 24;
  return 32;
}

// row stride of the LDS plane (complex elements): N2 plus a pad that spreads
// the strided column accesses of the x transforms over the LDS banks
constexpr int kPlanePad = 1;
int plane_stride(const Ctx& c) { return c.N[1] + kPlanePad; }

PlaneGeom geom(const Ctx& c) {
  PlaneGeom g;
  g.N1 = c.N[0];
  g.N2 = c.N[1];
  g.N3 = c.N[2];
  g.PS = plane_stride(c);
  g.hmax = c.hmax;
  g.ncol = c.ncol;
  g.p1 = c.plan[0];
  g.p2 = c.plan[1];
  return g;
}

size_t plane_lds(const Ctx& c, int nthr, size_t elem) {
  size_t b = (size_t)(c.N[0] + c.N[1] + c.N[0] * plane_stride(c) + 1) * elem;
  b += (size_t)2 * kMaxShell * (nthr / 64) * sizeof(double);
  return b;
}

int zchunk(const Ctx& c) {
  const int N3 = c.N[2];
  int CH = 32;
  while (CH > 1 && 2 * CH * N3 > kZThreads * 8) CH /= 2;
  return CH;
}

// Raise a kernel's dynamic LDS limit past the 64 KiB default.  The largest
// size set so far is remembered per (device, kernel), so steady-state
// launches make no runtime call for it.
std::mutex g_lds_mu;
std::map<std::pair<int, const void*>, size_t> g_lds_set;

template <typename K>
void allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return;
  int dev = 0;
  ROKS_HIP(hipGetDevice(&dev));
  const void* f = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lock(g_lds_mu);
  size_t& done = g_lds_set[{dev, f}];
  if (bytes <= done) return;
  ROKS_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  done = bytes;
}

template <typename R>
const C2<R>* twiddles(const Ctx& c, int d);
template <>
const double2* twiddles<double>(const Ctx& c, int d) { return c.d_tw[d]; }
template <>
const float2* twiddles<float>(const Ctx& c, int d) { return c.d_tw32[d]; }

// algorithmic HBM bytes: the column buffer of all pairs, the band arrays and
// real grids each move once per launch
double colbuf_bytes(const Ctx& c, int npairs) {
  return (double)npairs * c.N[2] * c.ncol * (c.prec == ROKS_FP32 ? sizeof(float2) : sizeof(double2));
}
double band_bytes(const Ctx& c, int nvec) { return (double)nvec * c.npw * sizeof(double2); }
// algorithmic flops of a complex line transform of length n (5 n log2 n)
double line_flops(int n) { return 5.0 * n * std::log2((double)n); }
// the plane passes' lines per band pair and z-plane: the rows |h| <= hmax
// along y and every column along x, once per direction
double plane_lines_flops(const Ctx& c, int directions) {
  return directions * ((2.0 * c.hmax + 1) * line_flops(c.N[1]) + (double)c.N[1] * line_flops(c.N[0]));
}
double grid_bytes(const Ctx& c) {
  return (double)c.ntot * (c.prec == ROKS_FP32 ? sizeof(float) : sizeof(double));
}

}  // namespace

void allow_dynamic_lds(const void* kernel, size_t bytes) { allow_lds(kernel, bytes); }

#define ROKS_DISPATCH_MAXP_RS(R, mp, RS, KER, ...)        \
  switch (mp) {                                           \
    case 8: KER<R, 8, RS>(__VA_ARGS__); break;            \
    case 16: KER<R, 16, RS>(__VA_ARGS__); break;          \
    case 24: KER<R, 24, RS>(__VA_ARGS__); break;          \
    default: KER<R, 32, RS>(__VA_ARGS__); break;          \
  }
#define ROKS_DISPATCH_MAXP(R, mp, rs, KER, ...)                              \
  if (rs == kLen64) {                                                       \
    ROKS_DISPATCH_MAXP_RS(R, mp, kLen64, KER, __VA_ARGS__)                  \
  } else {                                                                  \
    ROKS_DISPATCH_MAXP_RS(R, mp, kRadixAny, KER, __VA_ARGS__)               \
  }

// the plan class of one or two plans
int radix_set(const FftPlan1D& a) {
  return (a.n == 64 && a.nstages == 2 && a.radix[0] == 8 && a.radix[1] == 8) ? kLen64 : kRadixAny;
}
int radix_set(const FftPlan1D& a, const FftPlan1D& b) {
  return (radix_set(a) == kLen64 && radix_set(b) == kLen64) ? kLen64 : kRadixAny;
}

template <typename R, int MP, int RS>
static void run_zpass_bwd(Ctx& c, const double2* vecs, int nvec, void* T, int npairs, int CH,
                          const double* skip) {
  const size_t lds = (size_t)(c.N[2] + 2 * CH * (c.N[2] + 1)) * sizeof(C2<R>);
  allow_lds(k_zpass_bwd<R, MP, RS>, lds);
  dim3 grid(cdiv(c.nH + 1, CH), npairs);
  hipLaunchKernelGGL((k_zpass_bwd<R, MP, RS>), grid, dim3(kZThreads), lds, c.stream, vecs, nvec, c.npw,
                     c.d_cols, c.nH + 1, c.nH, c.plan[2], twiddles<R>(c, 2),
                     reinterpret_cast<C2<R>*>(T), c.ncol, CH, skip);
  ROKS_HIP(hipGetLastError());
}

void launch_zpass_bwd(Ctx& c, const double2* vecs, int nvec, void* T, int npairs, const double* skip) {
  c.T_src = nullptr;
  KernelTimer kt(c, "zpass_bwd", band_bytes(c, nvec) + colbuf_bytes(c, npairs),
                 (double)npairs * c.ncol * line_flops(c.N[2]));
  const int CH = zchunk(c);
  const int mp = pick_maxp(needed_points(2 * CH * c.N[2], kZThreads));
  if (c.prec == ROKS_FP32) {
    ROKS_DISPATCH_MAXP(float, mp, radix_set(c.plan[2]), run_zpass_bwd, c, vecs, nvec, T, npairs, CH, skip);
  } else {
    ROKS_DISPATCH_MAXP(double, mp, radix_set(c.plan[2]), run_zpass_bwd, c, vecs, nvec, T, npairs, CH, skip);
  }
}

template <typename R, int MP, int RS>
static void run_zpass_fwd(Ctx& c, const void* T, int npairs, const double2* vecs, int nvec,
                          const double* kinw, double2* Y, int CH) {
  const size_t lds = (size_t)(c.N[2] + 2 * CH * (c.N[2] + 1)) * sizeof(C2<R>);
  allow_lds(k_zpass_fwd<R, MP, RS>, lds);
  dim3 grid(cdiv(c.nH + 1, CH), npairs);
  hipLaunchKernelGGL((k_zpass_fwd<R, MP, RS>), grid, dim3(kZThreads), lds, c.stream,
                     reinterpret_cast<const C2<R>*>(T), c.ncol, c.d_cols, c.nH + 1, c.nH, c.plan[2],
                     twiddles<R>(c, 2), vecs, nvec, c.npw, kinw, c.d_g2, 1.0 / (double)c.ntot, Y, CH);
  ROKS_HIP(hipGetLastError());
}

void launch_zpass_fwd(Ctx& c, const void* T, int npairs, const double2* vecs, int nvec,
                      const double* kinw, double2* Y) {
  KernelTimer kt(c, "zpass_fwd", colbuf_bytes(c, npairs) + 2.0 * band_bytes(c, nvec),
                 (double)npairs * c.ncol * line_flops(c.N[2]));
  const int CH = zchunk(c);
  const int mp = pick_maxp(needed_points(2 * CH * c.N[2], kZThreads));
  if (c.prec == ROKS_FP32) {
    ROKS_DISPATCH_MAXP(float, mp, radix_set(c.plan[2]), run_zpass_fwd, c, T, npairs, vecs, nvec, kinw, Y, CH);
  } else {
    ROKS_DISPATCH_MAXP(double, mp, radix_set(c.plan[2]), run_zpass_fwd, c, T, npairs, vecs, nvec, kinw, Y, CH);
  }
}

template <typename R, int MP, int RS>
static void run_plane_apply(Ctx& c, void* T, int npairs, const void* pot, int npot,
                            const int32_t* potidx, int nvec, double* Qpart, int nQ) {
  const int nthr = plane_threads(c);
  const size_t lds = plane_lds(c, nthr, sizeof(C2<R>));
  allow_lds(k_plane_apply<R, MP, RS>, lds);
  const int nchunk = std::max(1, std::min(npairs, c.nchunk));
  const int per = cdiv(npairs, nchunk);
  dim3 grid(c.N[2], nchunk);
  hipLaunchKernelGGL((k_plane_apply<R, MP, RS>), grid, dim3(nthr), lds, c.stream,
                     reinterpret_cast<C2<R>*>(T), c.d_colpos, geom(c), twiddles<R>(c, 0),
                     twiddles<R>(c, 1), reinterpret_cast<const R*>(pot), npot, (size_t)c.ntot,
                     potidx, nvec, nQ, Qpart, npairs, per);
  ROKS_HIP(hipGetLastError());
}

// ---- line kernels ----
bool line_split(int n, int* G, int* P) {
  // the square sizes the line kernels are built for
  static const int table[][3] = {{16, 8, 2}, {24, 8, 3}, {32, 8, 4}, {40, 8, 5}, {48, 8, 6},
                                 {64, 8, 8}, {72, 8, 9}, {80, 16, 5}, {96, 16, 6}};
  for (const auto& e : table)
    if (e[0] == n) {
      *G = e[1];
      *P = e[2];
      return true;
    }
  return false;
}

// The density passes hold no potentials, so at 96 points they take the
// split with fewer cross-lane stages (8 lanes x 12 points: three radix-2
// lane stages instead of four, 16 % faster on the 96^3 oxide); the apply
// kept at 8 x 12 would spill.
bool line_split_density(int n, int* G, int* P) {
  if (n == 96) {
    *G = 8;
    *P = 12;
    return true;
  }
  return line_split(n, G, P);
}

size_t lines_lds(const Ctx& c, size_t elem, int nt) {
  const int n = c.N[0], nh = 2 * c.hmax + 1;
  return (size_t)(n + nh * (n + 1)) * elem + 6 * (nt / 64) * sizeof(double) +
         (size_t)nh * sizeof(int2);
}

LineGeom line_geom(const Ctx& c) {
  LineGeom g;
  g.N3 = c.N[2];
  g.PS = c.N[0] + 1;
  g.hmax = c.hmax;
  g.ncol = c.ncol;
  return g;
}

// apply: 256 threads, two or more workgroups per CU; density: 512 threads
// (the closed-shell sums of a lane's points stay in registers, half as many)
template <int MODE>
constexpr int line_threads() { return MODE == kModeApply ? 256 : 512; }

template <typename R, int G, int P, int MODE>
void run_lines_range(Ctx& c, void* T, int pair0, int pair_end, int nchunk, const void* pot,
                     const int32_t* potidx, int nvec, int nQ, double* Qpart, double* rho_part) {
  constexpr int NT = line_threads<MODE>();
  const size_t lds = lines_lds(c, sizeof(C2<R>), NT);
  allow_lds(k_plane_lines<R, G, P, MODE, NT>, lds);
  // every chunk runs (an empty one still writes its zero density slice)
  const int per = std::max(1, cdiv(pair_end - pair0, nchunk));
  dim3 grid(c.N[2], nchunk);
  hipLaunchKernelGGL((k_plane_lines<R, G, P, MODE, NT>), grid, dim3(NT), lds, c.stream,
                     reinterpret_cast<C2<R>*>(T), c.d_colidx,
                     reinterpret_cast<const int2*>(c.d_krange), line_geom(c), twiddles<R>(c, 0),
                     reinterpret_cast<const R*>(pot), (size_t)c.ntot, potidx, nvec, nQ, Qpart,
                     c.d_band_shell, c.nsocc, rho_part, pair0, pair_end, per);
  ROKS_HIP(hipGetLastError());
}

template <typename R, int G, int P, int MODE>
void run_lines(Ctx& c, void* T, int npairs, int nchunk, const void* pot, const int32_t* potidx,
               int nvec, int nQ, double* Qpart, double* rho_part) {
  if constexpr (MODE == kModeApply) {
    run_lines_range<R, G, P, kModeApply>(c, T, 0, npairs, nchunk, pot, potidx, nvec, nQ, Qpart,
                                         nullptr);
  } else {
    run_lines_range<R, G, P, kModeDensity>(c, T, 0, npairs, nchunk, nullptr, nullptr, nvec, 0,
                                           nullptr, rho_part);
    // the pairs that hold an open-shell band, one workgroup per plane
    int pa = -1, pb = -1;
    for (int n = 0; n < std::min(nvec, 2 * npairs); ++n) {
      const int X = c.band_shell[n];
      if (X >= 1 && X < c.nsocc) {
        if (pa < 0) pa = n / 2;
        pb = n / 2;
      }
    }
    if (pa >= 0)
      run_lines_range<R, G, P, kModeDensityOpen>(c, T, pa, pb + 1, 1, nullptr, nullptr, nvec, 0,
                                                 nullptr, rho_part);
  }
}

template <typename R, int MODE>
void dispatch_lines(Ctx& c, void* T, int npairs, int nchunk, const void* pot,
                    const int32_t* potidx, int nvec, int nQ, double* Qpart, double* rho_part) {
  const int LG = MODE == kModeApply ? c.lines_G : c.dlines_G;
  const int LP = MODE == kModeApply ? c.lines_P : c.dlines_P;
#define ROKS_LINES(GG, PP)                                                                         \
  if (LG == GG && LP == PP) {                                                                      \
    run_lines<R, GG, PP, MODE>(c, T, npairs, nchunk, pot, potidx, nvec, nQ, Qpart, rho_part);      \
    return;                                                                                        \
  }
  ROKS_LINES(8, 2) ROKS_LINES(8, 3) ROKS_LINES(8, 4) ROKS_LINES(8, 5) ROKS_LINES(8, 6)
  ROKS_LINES(8, 8) ROKS_LINES(8, 9) ROKS_LINES(16, 5) ROKS_LINES(16, 6)
  if constexpr (MODE != kModeApply) {
    ROKS_LINES(8, 12)
  }
#undef ROKS_LINES
  ROKS_CHECK(false, ROKS_ERR_SHAPE, "no line kernel for this plane");
}

void launch_plane_apply(Ctx& c, void* T, int npairs, const void* pot, int npot,
                        const int32_t* potidx, int nvec, double* Qpart, int nQ) {
  c.T_src = nullptr;  // the pass writes its result over the column buffer
  ROKS_CHECK(npot >= 1 && npot <= 3 && nQ <= npot, ROKS_ERR_ARG, "plane pass takes 1..3 potentials");
  KernelTimer kt(c, "plane_apply", 2.0 * colbuf_bytes(c, npairs) + npot * grid_bytes(c),
                 (double)npairs * c.N[2] * plane_lines_flops(c, 2));
  if (c.lines_G > 0) {
    // about two rounds of workgroups over the device
    const int nchunk = std::max(1, std::min(npairs, c.nchunk));
    if (c.prec == ROKS_FP32)
      dispatch_lines<float, kModeApply>(c, T, npairs, nchunk, pot, potidx, nvec, nQ, Qpart, nullptr);
    else
      dispatch_lines<double, kModeApply>(c, T, npairs, nchunk, pot, potidx, nvec, nQ, Qpart, nullptr);
    return;
  }
  const int mp = pick_maxp(needed_points(c.N[0] * c.N[1], plane_threads(c)));
  if (c.prec == ROKS_FP32) {
    ROKS_DISPATCH_MAXP(float, mp, radix_set(c.plan[0], c.plan[1]), run_plane_apply, c, T, npairs, pot, npot, potidx, nvec, Qpart, nQ);
  } else {
    ROKS_DISPATCH_MAXP(double, mp, radix_set(c.plan[0], c.plan[1]), run_plane_apply, c, T, npairs, pot, npot, potidx, nvec, Qpart, nQ);
  }
}

template <typename R, int MP, int RS>
static void run_plane_density(Ctx& c, const void* T, int npairs, double* rho_part, int nchunk) {
  const int nthr = plane_threads(c);
  const size_t lds = plane_lds(c, nthr, sizeof(C2<R>));
  allow_lds(k_plane_density<R, MP, RS>, lds);
  const int per = cdiv(npairs, nchunk);
  dim3 grid(c.N[2], nchunk);
  hipLaunchKernelGGL((k_plane_density<R, MP, RS>), grid, dim3(nthr), lds, c.stream,
                     reinterpret_cast<const C2<R>*>(T), c.d_colpos, geom(c), twiddles<R>(c, 0),
                     twiddles<R>(c, 1), c.d_band_shell, c.nb, c.nsocc, npairs, per, rho_part,
                     (size_t)c.ntot);
  ROKS_HIP(hipGetLastError());
}

// The FP32 tier's density planes: always with the line kernels (the square
// sizes of their table, 96^2 included); with the LDS-plane kernels only where
// they need at most 16 points per thread or are the length-64 build.  Beyond,
// the general-radix FP32 LDS-plane density kernel spills far more than the
// FP64 one (96^2 planes: 13.7 against 4.2 ms per all-band density), so such
// grids take the FP64 density.
bool fp32_density_planes(const Ctx& c) {
  if (c.lines_G > 0) return true;
  const int mp = pick_maxp(needed_points(c.N[0] * c.N[1], plane_threads(c)));
  return mp <= 16 || radix_set(c.plan[0], c.plan[1]) == kLen64;
}

void launch_plane_density(Ctx& c, const void* T, int npairs, double* rho_part, int nchunk) {
  KernelTimer kt(c, "plane_density",
                 colbuf_bytes(c, npairs) + (double)nchunk * c.nsocc * c.ntot * sizeof(double),
                 (double)npairs * c.N[2] * plane_lines_flops(c, 1));
  if (c.lines_G > 0) {
    void* Tm = const_cast<void*>(T);
    if (c.prec == ROKS_FP32)
      dispatch_lines<float, kModeDensity>(c, Tm, npairs, nchunk, nullptr, nullptr, c.nb, 0, nullptr, rho_part);
    else
      dispatch_lines<double, kModeDensity>(c, Tm, npairs, nchunk, nullptr, nullptr, c.nb, 0, nullptr, rho_part);
    return;
  }
  const int mp = pick_maxp(needed_points(c.N[0] * c.N[1], plane_threads(c)));
  if (c.prec == ROKS_FP32) {
    ROKS_DISPATCH_MAXP(float, mp, radix_set(c.plan[0], c.plan[1]), run_plane_density, c, T, npairs, rho_part, nchunk);
  } else {
    ROKS_DISPATCH_MAXP(double, mp, radix_set(c.plan[0], c.plan[1]), run_plane_density, c, T, npairs, rho_part, nchunk);
  }
}

constexpr int kAxisThreads = 256;
constexpr int kAxisPoints = 2048;  // points per workgroup at most (8 per thread)

template <typename R, int MP, int RS>
static void run_fft_axis(Ctx& c, double2* data, int sign, int axis, bool hartree) {
  const int n = c.N[axis];
  const int np2 = c.N[0] * c.N[1];
  // lines of this axis, their strides, and the batch (x lines: one z-plane each)
  int ncols, nbatch = 1;
  long estr, cstr, bstride = 0;
  if (axis == 1) {  // y: contiguous lines, one per (z, x)
    ncols = c.N[2] * c.N[0];
    estr = 1;
    cstr = c.N[1];
  } else if (axis == 0) {  // x: stride N2 within each z-plane
    ncols = c.N[1];
    estr = c.N[1];
    cstr = 1;
    nbatch = c.N[2];
    bstride = np2;
  } else {  // z: stride N1 N2
    ncols = np2;
    estr = np2;
    cstr = 1;
  }
  // ~1 000 workgroups per pass (several per CU, so their loads overlap), at
  // most kAxisPoints points each
  const int lines = ncols * nbatch;
  const int CH = std::max(1, std::min(kAxisPoints / n, cdiv(lines, 1024)));
  const size_t lds = (size_t)(n + CH * (n + 1)) * sizeof(double2);
  allow_lds(k_fft_axis<MP, RS>, lds);
  HartreeMul hm{};
  hm.on = 0;
  if (hartree) {
    ROKS_CHECK(axis == 2, ROKS_ERR_ARG, "the Hartree step rides on the z pass");
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) hm.b[i][j] = c.recip[i][j];
    for (int d = 0; d < 3; ++d) hm.N[d] = c.N[d];
    hm.inv = 1.0 / (double)c.ntot;
    hm.on = 1;
  }
  hipLaunchKernelGGL((k_fft_axis<MP, RS>), dim3(cdiv(ncols, CH), nbatch), dim3(kAxisThreads), lds, c.stream,
                     data, c.plan[axis], c.d_tw[axis], ncols, CH, estr, cstr, bstride, sign, hm);
  ROKS_HIP(hipGetLastError());
}

// one axis pass of the full-grid transform (hartree: the z pass with the
// Hartree multiply and the inverse z transform inside)
static void fft_axis_pass(Ctx& c, double2* data, int sign, int axis, bool hartree) {
  const int n = c.N[axis];
  const int pts = (kAxisPoints / n) * n;  // CH n at most
  const int mp = pick_maxp(needed_points(std::max(n, pts), kAxisThreads));
  ROKS_DISPATCH_MAXP(double, mp, radix_set(c.plan[axis]), run_fft_axis, c, data, sign, axis, hartree);
}

constexpr int kPlaneFftThreads = 512;

size_t fft_plane_lds(const Ctx& c) {
  return (size_t)(c.N[0] + c.N[1] + c.N[0] * plane_stride(c)) * sizeof(double2);
}

// the x-y plane fits the LDS of one workgroup (160 KiB) and needs at most 16
// points per thread (larger counts spill registers in the general-radix build,
// and two axis passes are then faster)
bool fft_plane_fits(const Ctx& c) {
  return fft_plane_lds(c) <= 160 * 1024 &&
         needed_points(c.N[0] * c.N[1], kPlaneFftThreads) <= 16;
}

template <typename R, int MP, int RS>
static void run_fft_plane(Ctx& c, double2* data, int sign, bool yfirst) {
  const size_t lds = fft_plane_lds(c);
  allow_lds(k_fft_plane<MP, RS>, lds);
  hipLaunchKernelGGL((k_fft_plane<MP, RS>), dim3(c.N[2]), dim3(kPlaneFftThreads), lds, c.stream, data,
                     c.plan[0], c.plan[1], c.d_tw[0], c.d_tw[1], plane_stride(c), sign, yfirst ? 1 : 0);
  ROKS_HIP(hipGetLastError());
}

// y and x transforms of the full grid: one plane pass when the plane fits the
// LDS, else two axis passes (same order of the axes either way)
static void fft_xy_pass(Ctx& c, double2* data, int sign, bool yfirst) {
  if (fft_plane_fits(c)) {
    const int mp = pick_maxp(needed_points(c.N[0] * c.N[1], kPlaneFftThreads));
    ROKS_DISPATCH_MAXP(double, mp, radix_set(c.plan[0], c.plan[1]), run_fft_plane, c, data, sign,
                       yfirst);
    return;
  }
  fft_axis_pass(c, data, sign, yfirst ? 1 : 0, false);
  fft_axis_pass(c, data, sign, yfirst ? 0 : 1, false);
}

// bytes moved: every pass reads and writes the grid once
void launch_fft3d(Ctx& c, double2* data, int sign) {
  const int passes = fft_plane_fits(c) ? 2 : 3;
  KernelTimer kt(c, "fft3d", 2.0 * passes * c.ntot * sizeof(double2),
                 5.0 * c.ntot * std::log2((double)c.ntot));
  fft_xy_pass(c, data, sign, true);
  fft_axis_pass(c, data, sign, 2, false);
}

void launch_hartree_fft(Ctx& c, double2* data) {
  const int passes = fft_plane_fits(c) ? 3 : 5;
  KernelTimer kt(c, "fft3d", 2.0 * passes * c.ntot * sizeof(double2),
                 10.0 * c.ntot * std::log2((double)c.ntot));
  fft_xy_pass(c, data, -1, true);
  fft_axis_pass(c, data, -1, 2, true);
  fft_xy_pass(c, data, +1, false);
}

}  // namespace roks
