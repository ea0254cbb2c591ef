// Hybrid exact exchange on PBE (Sec. III's PBE0 / DDH functionals): a
// fraction a of the Fock exchange of each configuration,
//   E_x^HF[L] = -1/2 sum_sigma sum_mn f_m f_n I_mn,  I_mn = int rho_mn V[rho_mn],
//   K^{sigma L}|v> = -sum_m f_m^{sigma L} psi_m V[psi_m v],
// rho_mn = psi_m psi_n (real Gamma-point orbitals), V[.] the Coulomb
// potential without its G = 0 term (the Hartree transform of the library,
// 4 pi / G^2 on the grid).  Orbitals live on the real-space grid as u =
// sum_G c(G) e^{iGr} (psi = u / sqrt(Omega)), two bands per complex
// transform; pair densities go through the Hartree transform two at a time
// (pair a in the real part, pair b in the imaginary part: both fields are
// real, so one complex transform carries both).  The cost is one Hartree
// transform per pair of bands and occupied orbital.
#include <cmath>
#include <vector>

#include "roks_internal.h"

namespace roks {

namespace {

constexpr int kExxBlocks = 64;

// block sum of two values per thread; the result in thread 0
__device__ void block_sum2(double (&v)[2], double* red) {
  const int tid = threadIdx.x, nw = blockDim.x >> 6, wid = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    double s = v[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[j * 16 + wid] = s;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[j * 16 + w];
      v[j] = s;
    }
  }
}

__global__ void k_exx_zero(double2* __restrict__ g, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    g[i] = make_double2(0.0, 0.0);
}

__device__ __forceinline__ size_t exx_index(int h, int k, int l, int N0, int N1, int N2) {
  const int x = ((h % N0) + N0) % N0, y = ((k % N1) + N1) % N1, z = ((l % N2) + N2) % N2;
  return ((size_t)z * N0 + x) * N1 + y;
}

// the full-grid spectrum of u_a + i u_b from the half-sphere coefficients
// (c(-G) = conj c(G)); G = 0 takes the real parts only
__global__ void k_exx_scatter(const double2* __restrict__ ca, const double2* __restrict__ cb, int npw,
                              const int32_t* __restrict__ miller, int N0, int N1, int N2,
                              double2* __restrict__ grid) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= npw) return;
  const int h = miller[3 * q], k = miller[3 * q + 1], l = miller[3 * q + 2];
  const double2 a = ca[q];
  const double2 b = cb ? cb[q] : make_double2(0.0, 0.0);
  if (q == 0) {
    grid[exx_index(0, 0, 0, N0, N1, N2)] = make_double2(a.x, b.x);
    return;
  }
  grid[exx_index(h, k, l, N0, N1, N2)] = make_double2(a.x - b.y, a.y + b.x);
  grid[exx_index(-h, -k, -l, N0, N1, N2)] = make_double2(a.x + b.y, b.x - a.y);
}

__global__ void k_exx_unpack(const double2* __restrict__ g, size_t n, double* __restrict__ ua,
                             double* __restrict__ ub) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = g[i];
    ua[i] = v.x;
    if (ub) ub[i] = v.y;
  }
}

// out = (ua ub s, uc ud s): two pair densities (the second may be absent)
__global__ void k_exx_pair2(const double* __restrict__ ua, const double* __restrict__ ub,
                            const double* __restrict__ uc, const double* __restrict__ ud, double s,
                            size_t n, double2* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = make_double2(ua[i] * ub[i] * s, uc ? uc[i] * ud[i] * s : 0.0);
}

// block partials of sum (ua ub s) Re V and sum (uc ud s) Im V
__global__ void __launch_bounds__(256) k_exx_int2(const double* __restrict__ ua,
                                                  const double* __restrict__ ub,
                                                  const double* __restrict__ uc,
                                                  const double* __restrict__ ud, double s,
                                                  const double2* __restrict__ V, size_t n,
                                                  double* __restrict__ part) {
  __shared__ double red[2 * 16];
  double acc[2] = {0.0, 0.0};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = V[i];
    acc[0] += ua[i] * ub[i] * s * v.x;
    if (uc) acc[1] += uc[i] * ud[i] * s * v.y;
  }
  block_sum2(acc, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = acc[0];
    part[2 * blockIdx.x + 1] = acc[1];
  }
}

// out = um (uv.x, uv.y) s: the pair densities of orbital m with two vectors
__global__ void k_exx_pack(const double* __restrict__ um, const double2* __restrict__ uv, size_t n,
                           double s, double2* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = uv[i];
    const double m = um[i] * s;
    out[i] = make_double2(m * v.x, m * v.y);
  }
}

// acc += (wa um Re V, wb um Im V); with part, the block partials of the pair
// integrals sum (um uv.x s) Re V and sum (um uv.y s) Im V
__global__ void __launch_bounds__(256) k_exx_acc(const double* __restrict__ um,
                                                 const double2* __restrict__ V, double wa, double wb,
                                                 const double2* __restrict__ uv, double s, size_t n,
                                                 double2* __restrict__ acc, double* __restrict__ part) {
  __shared__ double red[2 * 16];
  double sums[2] = {0.0, 0.0};
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const double2 v = V[i];
    const double m = um[i];
    double2 a = acc[i];
    a.x += wa * m * v.x;
    a.y += wb * m * v.y;
    acc[i] = a;
    if (part) {
      const double2 w = uv[i];
      sums[0] += m * w.x * s * v.x;
      sums[1] += m * w.y * s * v.y;
    }
  }
  if (!part) return;
  block_sum2(sums, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sums[0];
    part[2 * blockIdx.x + 1] = sums[1];
  }
}

// y_a(G) += scale (F(G) + conj F(-G)) / 2, y_b(G) += scale (F(G) - conj F(-G)) / 2i
__global__ void k_exx_gather(const double2* __restrict__ F, int npw, const int32_t* __restrict__ miller,
                             int N0, int N1, int N2, double scale, double2* __restrict__ ya,
                             double2* __restrict__ yb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= npw) return;
  const int h = miller[3 * q], k = miller[3 * q + 1], l = miller[3 * q + 2];
  const double2 p = F[exx_index(h, k, l, N0, N1, N2)];
  const double2 m = F[exx_index(-h, -k, -l, N0, N1, N2)];
  double2 a = ya[q];
  a.x += scale * 0.5 * (p.x + m.x);
  a.y += scale * 0.5 * (p.y - m.y);
  ya[q] = a;
  if (yb) {
    double2 b = yb[q];
    b.x += scale * 0.5 * (p.y + m.y);
    b.y -= scale * 0.5 * (p.x - m.x);
    yb[q] = b;
  }
}

// in-order sum of the kExxBlocks partials of `count` integral pairs, times dv
__global__ void k_exx_reduce(const double* __restrict__ part, int count, double dv,
                             double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * count) return;
  const int p = t >> 1, b = t & 1;
  double s = 0.0;
  for (int k = 0; k < kExxBlocks; ++k) s += part[((size_t)p * kExxBlocks + k) * 2 + b];
  out[t] = dv * s;
}

// Q[n][X] += a <n|K^X|n> = -a sum_m W[X][m] I[n][m] (m over the bands)
__global__ void k_exx_q(const double* __restrict__ I, const double* __restrict__ W, int nb, int nsocc,
                        double a, double* __restrict__ Q) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * nsocc) return;
  const int n = t / nsocc, X = t - n * nsocc;
  double s = 0.0;
  for (int m = 0; m < nb; ++m) s += W[(size_t)X * nb + m] * I[(size_t)n * nb + m];
  Q[(size_t)n * nsocc + X] -= a * s;
}

unsigned blocks_for(size_t n) { return (unsigned)std::min<size_t>(8192, (n + 255) / 256); }

void ensure_exx(Ctx& c) {
  if (c.d_exx_u) return;
  const size_t n = c.ntot;
  c.d_exx_u = dalloc<double>(c, (size_t)c.nb * n);
  c.d_exx_g = dalloc<double2>(c, 3 * n);
  c.d_exx_I = dalloc<double>(c, 2 * (size_t)c.nb * (c.nb + 1));
  c.d_exx_part = dalloc<double>(c, 2 * (size_t)kExxBlocks * c.nb * (size_t)c.nb);
  // W[X][m] = sum_L c_L sum_sigma f_X^{sigma L} f_m^{sigma L}
  std::vector<double> W((size_t)c.nsocc * c.nb, 0.0);
  for (int X = 0; X < c.nsocc; ++X)
    for (int m = 0; m < c.nb; ++m) {
      const int Y = c.band_shell[m];
      double w = 0.0;
      for (int L = 0; L < c.nconf; ++L)
        for (int s = 0; s < 2; ++s) w += c.cL[L] * c.shell_f[X][L][s] * (Y < c.nsocc ? c.shell_f[Y][L][s] : 0.0);
      W[(size_t)X * c.nb + m] = w;
    }
  c.d_exx_W = dalloc<double>(c, W.size());
  ROKS_HIP(hipMemcpyAsync(c.d_exx_W, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
  ROKS_HIP(hipStreamSynchronize(c.stream));
}

// the real-space grids u_a + i u_b of bands a, b (b may be -1) of vecs into g
void to_grid(Ctx& c, const double2* vecs, int a, int b, double2* g) {
  const size_t n = c.ntot;
  hipLaunchKernelGGL(k_exx_zero, dim3(blocks_for(n)), dim3(256), 0, c.stream, g, n);
  hipLaunchKernelGGL(k_exx_scatter, dim3(cdiv(c.npw, 256)), dim3(256), 0, c.stream, vecs + (size_t)a * c.npw,
                     b >= 0 ? vecs + (size_t)b * c.npw : nullptr, c.npw, c.d_miller, c.N[0], c.N[1], c.N[2], g);
  ROKS_HIP(hipGetLastError());
  launch_fft3d(c, g, +1);
}

bool occupied(const Ctx& c, int m) { return !c.shell_virtual[c.band_shell[m]]; }

}  // namespace

void exx_orbitals(Ctx& c, const double2* orb) {
  ensure_exx(c);
  const size_t n = c.ntot;
  for (int a = 0; a < c.nb; a += 2) {
    const int b = a + 1 < c.nb ? a + 1 : -1;
    to_grid(c, orb, a, b, c.d_exx_g);
    hipLaunchKernelGGL(k_exx_unpack, dim3(blocks_for(n)), dim3(256), 0, c.stream, c.d_exx_g, n,
                       c.d_exx_u + (size_t)a * n, b >= 0 ? c.d_exx_u + (size_t)b * n : nullptr);
    ROKS_HIP(hipGetLastError());
  }
}

void exx_energies(Ctx& c) {
  const size_t n = c.ntot;
  const double s = 1.0 / c.omega, dv = c.omega / (double)n;
  std::vector<int> occ;
  for (int m = 0; m < c.nb; ++m)
    if (occupied(c, m)) occ.push_back(m);
  std::vector<std::pair<int, int>> pairs;
  for (size_t i = 0; i < occ.size(); ++i)
    for (size_t j = i; j < occ.size(); ++j) pairs.emplace_back(occ[i], occ[j]);
  const int np2 = (int)((pairs.size() + 1) / 2);
  double2* g = c.d_exx_g;
  for (int p = 0; p < np2; ++p) {
    const auto P0 = pairs[2 * p];
    const bool two = 2 * p + 1 < (int)pairs.size();
    const auto P1 = two ? pairs[2 * p + 1] : P0;
    const double* ua = c.d_exx_u + (size_t)P0.first * n;
    const double* ub = c.d_exx_u + (size_t)P0.second * n;
    const double* uc = two ? c.d_exx_u + (size_t)P1.first * n : nullptr;
    const double* ud = two ? c.d_exx_u + (size_t)P1.second * n : nullptr;
    hipLaunchKernelGGL(k_exx_pair2, dim3(blocks_for(n)), dim3(256), 0, c.stream, ua, ub, uc, ud, s, n, g);
    ROKS_HIP(hipGetLastError());
    launch_hartree_fft(c, g);
    hipLaunchKernelGGL(k_exx_int2, dim3(kExxBlocks), dim3(256), 0, c.stream, ua, ub, uc, ud, s, g, n,
                       c.d_exx_part + (size_t)p * 2 * kExxBlocks);
    ROKS_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_exx_reduce, dim3(cdiv(2 * np2, 256)), dim3(256), 0, c.stream, c.d_exx_part, np2, dv,
                     c.d_exx_I);
  ROKS_HIP(hipGetLastError());
  std::vector<double> I(2 * (size_t)np2);
  to_host(c, I.data(), c.d_exx_I, I.size() * sizeof(double));
  for (int L = 0; L < kMaxConf; ++L) c.exx_E[L] = 0.0;
  for (size_t k = 0; k < pairs.size(); ++k) {
    const int m = pairs[k].first, nn = pairs[k].second;
    const double Imn = I[k];
    for (int L = 0; L < c.nconf; ++L) {
      double w = 0.0;
      for (int sp = 0; sp < 2; ++sp)
        w += (double)c.occ[(L * 2 + sp) * c.nb + m] * (double)c.occ[(L * 2 + sp) * c.nb + nn];
      c.exx_E[L] -= (m == nn ? 0.5 : 1.0) * w * Imn;
    }
  }
}

void exx_apply(Ctx& c, const double2* vecs, int nvec, const double* rowW, double2* out, double* Iout) {
  const size_t n = c.ntot;
  const double s = 1.0 / c.omega, dv = c.omega / (double)n;
  double2* uv = c.d_exx_g;
  double2* pd = c.d_exx_g + n;
  double2* acc = c.d_exx_g + 2 * n;
  const int npair = (nvec + 1) / 2;
  for (int p = 0; p < npair; ++p) {
    const int a = 2 * p, b = a + 1 < nvec ? a + 1 : -1;
    to_grid(c, vecs, a, b, uv);
    hipLaunchKernelGGL(k_exx_zero, dim3(blocks_for(n)), dim3(256), 0, c.stream, acc, n);
    for (int m = 0; m < c.nb; ++m) {
      const double wa = rowW[(size_t)a * c.nb + m], wb = b >= 0 ? rowW[(size_t)b * c.nb + m] : 0.0;
      if (wa == 0.0 && wb == 0.0 && !Iout) continue;
      if (!occupied(c, m)) continue;
      const double* um = c.d_exx_u + (size_t)m * n;
      hipLaunchKernelGGL(k_exx_pack, dim3(blocks_for(n)), dim3(256), 0, c.stream, um, uv, n, s, pd);
      ROKS_HIP(hipGetLastError());
      launch_hartree_fft(c, pd);
      hipLaunchKernelGGL(k_exx_acc, dim3(kExxBlocks), dim3(256), 0, c.stream, um, pd, wa, wb, uv, s, n, acc,
                         Iout ? c.d_exx_part + ((size_t)p * c.nb + m) * 2 * kExxBlocks : nullptr);
      ROKS_HIP(hipGetLastError());
    }
    launch_fft3d(c, acc, -1);
    hipLaunchKernelGGL(k_exx_gather, dim3(cdiv(c.npw, 256)), dim3(256), 0, c.stream, acc, c.npw, c.d_miller,
                       c.N[0], c.N[1], c.N[2], c.exx / (double)n, out + (size_t)a * c.npw,
                       b >= 0 ? out + (size_t)b * c.npw : nullptr);
    ROKS_HIP(hipGetLastError());
  }
  if (Iout) {
    // I[a][m], I[b][m] of every vector pair: partial index (p nb + m), the
    // two entries of a partial pair are bands a and b
    ROKS_CHECK(nvec == c.nb, ROKS_ERR_ARG, "pair integrals need all bands");
    hipLaunchKernelGGL(k_exx_reduce, dim3(cdiv(2 * npair * c.nb, 256)), dim3(256), 0, c.stream,
                       c.d_exx_part, npair * c.nb, dv, Iout + (size_t)c.nb * c.nb);
    ROKS_HIP(hipGetLastError());
  }
}

void exx_shell_expectations(Ctx& c) {
  // the reduced pairs sit at d_exx_I + nb^2 in (pair p, m, band of the pair)
  // order; I[n][m] with n = 2p + b
  const int nb = c.nb, npair = (nb + 1) / 2;
  std::vector<double> red(2 * (size_t)npair * nb), I((size_t)nb * nb, 0.0);
  to_host(c, red.data(), c.d_exx_I + (size_t)nb * nb, red.size() * sizeof(double));
  for (int p = 0; p < npair; ++p)
    for (int m = 0; m < nb; ++m)
      for (int b = 0; b < 2; ++b) {
        const int row = 2 * p + b;
        if (row < nb && occupied(c, m)) I[(size_t)row * nb + m] = red[((size_t)p * nb + m) * 2 + b];
      }
  ROKS_HIP(hipMemcpyAsync(c.d_exx_I, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice, c.stream));
  hipLaunchKernelGGL(k_exx_q, dim3(cdiv(nb * c.nsocc, 256)), dim3(256), 0, c.stream, c.d_exx_I, c.d_exx_W,
                     nb, c.nsocc, c.exx, c.d_Q);
  ROKS_HIP(hipGetLastError());
  ROKS_HIP(hipStreamSynchronize(c.stream));  // I goes out of scope
}

}  // namespace roks
