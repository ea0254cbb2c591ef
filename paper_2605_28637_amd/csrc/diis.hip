// DIIS on the ROKS residual (Sec. II A, Eq. residual_frank; the method of
// Hutter, Luthi and Parrinello named there), reusing the hot path: the
// energy and F^n|n> of the CG step, its band products, the Teter
// preconditioner and the Cholesky orthonormalisation.  Steps (the oracle's
// readings D1-D5):
//   r_n = F^n|n> - sum_m S|m> Lambda_mn,
//         Lambda_mn = theta_mn - lambda_mn (theta_mn - theta_nm),
//         lambda = 1/2, or 1/2 / -1/2 for the open pair (a, b) / (b, a);
//   e_n = K_n r_n (Teter, E_ref from r_n, no projection);
//   c = argmin c^T B c, sum c = 1, B_ij = sum_n <e^i_n|e^j_n> over the kept
//       iterates (the oldest dropped while the bordered system is singular);
//   psi = orth(sum_i c_i (psi^i + step e^i)) (in the metric of S).
// The kept orbitals and error vectors live in device arrays of the context
// (2 x 8 band arrays, allocated on the first step); B is kept on the host,
// one new row per step, each entry a band-ordered sum of per-band dots.
#include <cmath>
#include <cstring>

#include "roks_internal.h"

namespace roks {

namespace {

// Lambda[m][n] = theta[m][n] - lambda_mn (theta[m][n] - theta[n][m])
__global__ void k_diis_lambda(const double* __restrict__ theta, int nb, int a, int b,
                              double* __restrict__ Lam) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * nb) return;
  const int m = t / nb, n = t - m * nb;
  double lam = 0.5;
  if (m == b && n == a) lam = -0.5;  // lambda_ba; lambda_ab stays 1/2
  const double th = theta[t];
  Lam[t] = th - lam * (th - theta[n * nb + m]);
}

struct Combine {
  const double* psi[kDiisMaxHistory];
  const double* e[kDiisMaxHistory];
  double c[kDiisMaxHistory];
  int k;
};

// out = sum_j c_j (psi_j + step e_j), the terms added in iterate order
__global__ void __launch_bounds__(256) k_diis_combine(Combine cb, double step, size_t n,
                                                      double* __restrict__ out) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < cb.k; ++j) s += cb.c[j] * (cb.psi[j][i] + step * cb.e[j][i]);
  out[i] = s;
}

// the bordered DIIS system [B 1; 1^T 0] [c; mu] = [0; 1] by Gaussian
// elimination with partial pivoting; false when a pivot vanishes against
// the scale of B
bool solve_bordered(const std::vector<double>& B, int k, std::vector<double>& c) {
  const int n = k + 1;
  std::vector<double> A((size_t)n * n, 0.0), x(n, 0.0);
  double scale = 0.0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      A[(size_t)i * n + j] = B[(size_t)i * k + j];
      scale = std::max(scale, std::fabs(B[(size_t)i * k + j]));
    }
  for (int i = 0; i < k; ++i) A[(size_t)i * n + k] = A[(size_t)k * n + i] = 1.0;
  x[k] = 1.0;
  const double tiny = 1e-14 * std::max(scale, 1e-300);
  for (int col = 0; col < n; ++col) {
    int p = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + col]) > std::fabs(A[(size_t)p * n + col])) p = r;
    // the border column holds ones: compare its pivots with 1, the rest with B
    const double ref = col == k ? 1e-14 : tiny;
    if (!(std::fabs(A[(size_t)p * n + col]) > ref)) return false;
    if (p != col) {
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)p * n + j], A[(size_t)col * n + j]);
      std::swap(x[p], x[col]);
    }
    for (int r = col + 1; r < n; ++r) {
      const double f = A[(size_t)r * n + col] / A[(size_t)col * n + col];
      if (f == 0.0) continue;
      for (int j = col; j < n; ++j) A[(size_t)r * n + j] -= f * A[(size_t)col * n + j];
      x[r] -= f * x[col];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = x[r];
    for (int j = r + 1; j < n; ++j) s -= A[(size_t)r * n + j] * x[j];
    x[r] = s / A[(size_t)r * n + r];
  }
  c.assign(x.begin(), x.begin() + k);
  for (double v : c)
    if (!std::isfinite(v)) return false;
  return true;
}

}  // namespace

void reset_diis(Ctx& c) {
  c.diis_order.clear();
}

void diis_step(Ctx& c, const roks_diis_params& p, roks_diis_info* info) {
  ROKS_CHECK(c.have_orbitals, ROKS_ERR_STATE, "no orbitals set");
  ROKS_CHECK(p.history >= 1 && p.history <= kDiisMaxHistory, ROKS_ERR_ARG,
             "history must be 1 .. ROKS_DIIS_MAX_HISTORY");
  ROKS_CHECK(p.step > 0.0 && std::isfinite(p.step), ROKS_ERR_ARG, "step must be > 0");
  const int nb = c.nb, K = 2 * c.npw;
  const size_t band = (size_t)nb * c.npw;
  if (!c.d_diis) {
    c.d_diis = dalloc<double2>(c, 2 * (size_t)kDiisMaxHistory * band);
    c.d_diis_dots = dalloc<double>(c, (size_t)(kDiisMaxHistory + 1) * nb);
    c.diis_B.assign((size_t)kDiisMaxHistory * kDiisMaxHistory, 0.0);
  }
  // a new history length or coupling starts a new history
  if (p.history != c.diis_hist || (p.asymmetric != 0) != c.diis_asym) reset_diis(c);
  c.diis_hist = p.history;
  c.diis_asym = p.asymmetric != 0;
  // open pair (two open bands, band order)
  int a = -1, b = -1, no = 0;
  for (int n = 0; n < nb; ++n) {
    const int X = c.band_shell[n];
    if (!c.shell_closed[X] && !c.shell_virtual[X]) {
      if (no == 0) a = n;
      else if (no == 1) b = n;
      ++no;
    }
  }
  const bool pair = no == 2;
  roks_energies e0;
  energy_gradient(c, &e0);
  // D1: Lambda (in d_m1), r = Y - Lambda^T psi (in d_p)
  hipLaunchKernelGGL(k_diis_lambda, dim3(cdiv(nb * nb, 256)), dim3(256), 0, c.stream, c.d_theta, nb,
                     (pair && c.diis_asym) ? a : -1, (pair && c.diis_asym) ? b : -1, c.d_m1);
  ROKS_HIP(hipGetLastError());
  double2* r = c.d_p;
  gemm_expand_to(c, nb, K, nb, c.d_m1, nb, false, dbl(overlap_psi(c)), K, dbl(c.d_Y), K, dbl(r), K,
                 -1.0, 1.0);
  // the slot of the new iterate (the oldest is dropped at full history)
  if ((int)c.diis_order.size() == p.history) c.diis_order.erase(c.diis_order.begin());
  int slot = 0;
  for (;; ++slot) {
    bool used = false;
    for (int s : c.diis_order) used = used || s == slot;
    if (!used) break;
  }
  double2* ps = c.d_diis + (size_t)(2 * slot) * band;
  double2* es = ps + band;
  // D2: e = K r (Teter, E_ref = 1.5 <r|T|r> / <r|r> per band)
  double* rr = c.d_diis_dots;
  band_dots2(c, r, r, nb, rr, c.d_bandv);
  launch_teter(c, c.d_bandv, rr, r, nullptr, es);
  copy_dev(c, ps, c.d_psi, band * sizeof(double2));
  c.diis_order.push_back(slot);
  // D3: the new row of B, per-band dots summed in band order on the host
  const int k = (int)c.diis_order.size();
  for (int j = 0; j < k; ++j) {
    const double2* ej = c.d_diis + (size_t)(2 * c.diis_order[j] + 1) * band;
    band_dots2(c, es, ej, nb, c.d_diis_dots + (size_t)(1 + j) * nb, nullptr);
  }
  std::vector<double> dots((size_t)(k + 1) * nb);
  to_host(c, dots.data(), c.d_diis_dots, dots.size() * sizeof(double));
  double oc = 0.0;
  if (pair) {
    double tab = 0.0, tba = 0.0;
    to_host(c, &tab, c.d_theta + (size_t)a * nb + b, sizeof(double));
    to_host(c, &tba, c.d_theta + (size_t)b * nb + a, sizeof(double));
    oc = tab - tba;
  }
  double rnorm2 = 0.0;
  for (int n = 0; n < nb; ++n) rnorm2 += dots[n];
  const int H = kDiisMaxHistory;
  for (int j = 0; j < k; ++j) {
    double s = 0.0;
    for (int n = 0; n < nb; ++n) s += dots[(size_t)(1 + j) * nb + n];
    c.diis_B[(size_t)slot * H + c.diis_order[j]] = s;
    c.diis_B[(size_t)c.diis_order[j] * H + slot] = s;
  }
  std::vector<double> coef;
  for (;;) {
    const int kk = (int)c.diis_order.size();
    std::vector<double> Bk((size_t)kk * kk);
    for (int i = 0; i < kk; ++i)
      for (int j = 0; j < kk; ++j)
        Bk[(size_t)i * kk + j] = c.diis_B[(size_t)c.diis_order[i] * H + c.diis_order[j]];
    if (solve_bordered(Bk, kk, coef)) break;
    if (kk == 1) {
      coef.assign(1, 1.0);
      break;
    }
    c.diis_order.erase(c.diis_order.begin());
  }
  // D4: psi = sum_i c_i (psi^i + step e^i), then D5
  Combine cb{};
  cb.k = (int)c.diis_order.size();
  for (int j = 0; j < cb.k; ++j) {
    cb.psi[j] = dbl(c.d_diis + (size_t)(2 * c.diis_order[j]) * band);
    cb.e[j] = dbl(c.d_diis + (size_t)(2 * c.diis_order[j] + 1) * band);
    cb.c[j] = coef[j];
  }
  const size_t nreal = 2 * band;
  hipLaunchKernelGGL(k_diis_combine, dim3((unsigned)((nreal + 255) / 256)), dim3(256), 0, c.stream, cb,
                     p.step, nreal, dbl(c.d_psi));
  ROKS_HIP(hipGetLastError());
  c.potentials_valid = false;
  reset_cg(c);  // carried CG directions do not belong to these orbitals
  try {
    orthonormalize(c, c.d_psi);
  } catch (const Error&) {
    // a combination without full rank: the step's input orbitals stay
    copy_dev(c, c.d_psi, ps, band * sizeof(double2));
    reset_diis(c);
    throw;
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->E = e0.E;
    info->rnorm2 = rnorm2;
    info->open_coupling = oc;
    info->used = cb.k;
    for (int j = 0; j < cb.k; ++j) info->coeffs[j] = coef[j];
  }
}

}  // namespace roks
