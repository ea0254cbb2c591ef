// The C ABI (include/roks.h): argument checks, error translation, host <->
// device copies.  Every entry point catches the library's exceptions and
// returns a status; the message is kept per context.
#include <cmath>
#include <cstring>
#include <string>

#include "roks_internal.h"

struct roks_mlp_s {
  roks::Mlp m;
};

namespace {

thread_local std::string g_create_error;

template <typename F>
roks_status guard(roks_ctx ctx, F&& f) {
  if (!ctx) return ROKS_ERR_ARG;
  try {
    f(ctx->c);
    return ROKS_OK;
  } catch (const roks::Error& e) {
    ctx->c.last_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    ctx->c.last_error = e.what();
    return ROKS_ERR_HIP;
  }
}

template <typename F>
roks_status guard_mlp(roks_mlp mlp, F&& f) {
  if (!mlp) return ROKS_ERR_ARG;
  try {
    f(mlp->m);
    return ROKS_OK;
  } catch (const roks::Error& e) {
    mlp->m.last_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    mlp->m.last_error = e.what();
    return ROKS_ERR_HIP;
  }
}

// release one allocation of the context (stream-synchronised)
void dfree(roks::Ctx& c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c.allocations.size(); ++i)
    if (c.allocations[i].p == p) {
      ROKS_HIP(hipStreamSynchronize(c.stream));
      ROKS_HIP(hipFree(p));
      c.allocations.erase(c.allocations.begin() + (long)i);
      return;
    }
}

void drop_records(roks::Ctx& c) {
  dfree(c, c.d_rec_psi);
  dfree(c, c.d_rec_kg);
  dfree(c, c.d_rec_feat);
  dfree(c, c.d_rec_valid);
  dfree(c, c.d_rec_ekin);
  c.d_rec_ekin = nullptr;
  c.d_rec_psi = c.d_rec_kg = nullptr;
  c.d_rec_feat = nullptr;
  c.d_rec_valid = nullptr;
  c.rec_max = 0;
  c.rec_count = 0;
}

void upload_bands(roks::Ctx& c, double2* dst, const double* src) {
  ROKS_HIP(hipMemcpyAsync(dst, src, (size_t)c.nb * c.npw * sizeof(double2), hipMemcpyHostToDevice,
                          c.stream));
}

void check_finite_host(const roks::Ctx& c, const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    ROKS_CHECK(std::isfinite(v[i]), ROKS_ERR_NAN, "non-finite input coefficient");
}

// c(-G) = conj(c(G)) makes c(0) real: a nonzero Im c_n(0) is no real orbital
void check_g0_real_host(const roks::Ctx& c, const double* v) {
  for (int n = 0; n < c.nb; ++n)
    ROKS_CHECK(v[(size_t)n * c.npw * 2 + 1] == 0.0, ROKS_ERR_ARG,
               "Im c_n(G = 0) must be zero (real orbitals)");
}

}  // namespace

extern "C" {

const char* roks_version(void) { return "roks-gfx950 0.2"; }

roks_status roks_grid_rule(const double cell[3][3], double ecut, int32_t grid[3]) {
  if (!cell || !grid || !(ecut > 0) || !std::isfinite(ecut)) return ROKS_ERR_ARG;
  int g[3];
  roks::grid_rule(cell, ecut, g);
  for (int d = 0; d < 3; ++d) grid[d] = g[d];
  return ROKS_OK;
}

roks_status roks_create(const roks_system* sys, void* hip_stream, roks_ctx* out) {
  if (!out) return ROKS_ERR_ARG;
  *out = nullptr;
  roks_ctx ctx = new (std::nothrow) roks_ctx_s;
  if (!ctx) return ROKS_ERR_OOM;
  try {
    roks::build_problem(ctx->c, sys);
    roks::build_sphere(ctx->c);
    roks::build_projectors(ctx->c);
    roks::init_device(ctx->c, hip_stream);
    roks::upload_static(ctx->c);
  } catch (const roks::Error& e) {
    g_create_error = e.msg;
    roks::free_device(ctx->c);
    delete ctx;
    return e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    roks::free_device(ctx->c);
    delete ctx;
    return ROKS_ERR_HIP;
  }
  *out = ctx;
  return ROKS_OK;
}

roks_status roks_destroy(roks_ctx ctx) {
  if (!ctx) return ROKS_ERR_ARG;
  roks::free_device(ctx->c);
  delete ctx;
  return ROKS_OK;
}

const char* roks_last_error(roks_ctx ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->c.last_error.c_str();
}

roks_status roks_sizes(roks_ctx ctx, int32_t* npw, int32_t grid[3], int32_t* nproj, int32_t* nbands) {
  return guard(ctx, [&](roks::Ctx& c) {
    if (npw) *npw = c.npw;
    if (grid)
      for (int d = 0; d < 3; ++d) grid[d] = c.N[d];
    if (nproj) *nproj = c.nproj;
    if (nbands) *nbands = c.nb;
  });
}

roks_status roks_gvectors(roks_ctx ctx, int32_t* miller) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(miller, ROKS_ERR_ARG, "miller is NULL");
    std::memcpy(miller, c.miller.data(), c.miller.size() * sizeof(int32_t));
  });
}

roks_status roks_set_coeffs(roks_ctx ctx, const double* cf, int32_t orthonormalize) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(cf, ROKS_ERR_ARG, "coefficients are NULL");
    check_finite_host(c, cf, (size_t)c.nb * c.npw * 2);
    check_g0_real_host(c, cf);
    upload_bands(c, c.d_psi, cf);
    if (orthonormalize) roks::orthonormalize(c, c.d_psi);
    ROKS_HIP(hipStreamSynchronize(c.stream));
    c.have_orbitals = true;
    c.potentials_valid = false;
    roks::reset_cg(c);
    roks::reset_diis(c);
  });
}

roks_status roks_set_coeffs_d(roks_ctx ctx, const void* cf, int32_t orthonormalize) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(cf, ROKS_ERR_ARG, "coefficients are NULL");
    ROKS_HIP(hipMemcpyAsync(c.d_psi, cf, (size_t)c.nb * c.npw * sizeof(double2),
                            hipMemcpyDeviceToDevice, c.stream));
    roks::launch_zero_g0_imag(c, c.d_psi, c.nb);
    if (orthonormalize) roks::orthonormalize(c, c.d_psi);
    c.have_orbitals = true;
    c.potentials_valid = false;
    roks::reset_cg(c);
    roks::reset_diis(c);
  });
}

roks_status roks_get_coeffs(roks_ctx ctx, double* cf) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(cf, ROKS_ERR_ARG, "output is NULL");
    ROKS_CHECK(c.have_orbitals, ROKS_ERR_STATE, "no orbitals set");
    ROKS_HIP(hipMemcpyAsync(cf, c.d_psi, (size_t)c.nb * c.npw * sizeof(double2),
                            hipMemcpyDeviceToHost, c.stream));
    ROKS_HIP(hipStreamSynchronize(c.stream));
  });
}

roks_status roks_get_coeffs_d(roks_ctx ctx, void* cf) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(cf, ROKS_ERR_ARG, "output is NULL");
    ROKS_CHECK(c.have_orbitals, ROKS_ERR_STATE, "no orbitals set");
    ROKS_HIP(hipMemcpyAsync(cf, c.d_psi, (size_t)c.nb * c.npw * sizeof(double2),
                            hipMemcpyDeviceToDevice, c.stream));
  });
}

roks_status roks_set_positions(roks_ctx ctx, const double* pos) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(pos, ROKS_ERR_ARG, "positions are NULL");
    for (int i = 0; i < 3 * c.natoms; ++i)
      ROKS_CHECK(std::isfinite(pos[i]), ROKS_ERR_ARG, "non-finite position");
    c.pos.assign(pos, pos + 3 * (size_t)c.natoms);
    roks::upload_positions(c);
    ROKS_HIP(hipStreamSynchronize(c.stream));
    roks::reset_cg(c);
    roks::reset_diis(c);
    if (c.has_q && c.have_orbitals) {
      // S moves with the atoms: the orbitals become S-orthonormal again
      c.potentials_valid = false;
      roks::orthonormalize(c, c.d_psi);
    }
  });
}

static uint32_t channel_count(const roks::Ctx& c, uint32_t mask) {
  ROKS_CHECK((mask >> (2 * c.nconf)) == 0, ROKS_ERR_ARG, "channel mask selects a missing configuration");
  uint32_t n = 0;
  for (int b = 0; b < 2 * c.nconf; ++b) n += (mask >> b) & 1u;
  return n;
}

roks_status roks_apply_h(roks_ctx ctx, const double* c_in, uint32_t mask, double* h_out) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(h_out, ROKS_ERR_ARG, "output is NULL");
    const uint32_t nch = mask ? channel_count(c, mask) : 1u;
    roks::ensure_potentials(c);
    const double2* src = c.d_psi;
    if (c_in) {
      check_finite_host(c, c_in, (size_t)c.nb * c.npw * 2);
      check_g0_real_host(c, c_in);
      upload_bands(c, c.d_in, c_in);
      src = c.d_in;
    }
    const size_t band = (size_t)c.nb * c.npw;
    double2* out = c.d_Y;
    if (nch > 1) {
      if (!c.d_hch) c.d_hch = roks::dalloc<double2>(c, 4 * band);
      out = c.d_hch;
    }
    roks::apply_operator(c, src, mask, out, false);
    ROKS_HIP(hipMemcpyAsync(h_out, out, nch * band * sizeof(double2), hipMemcpyDeviceToHost, c.stream));
    ROKS_HIP(hipStreamSynchronize(c.stream));
  });
}

roks_status roks_apply_h_d(roks_ctx ctx, const void* c_in, uint32_t mask, void* h_out) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(h_out, ROKS_ERR_ARG, "output is NULL");
    if (mask) channel_count(c, mask);
    roks::ensure_potentials(c);
    const double2* src = c_in ? reinterpret_cast<const double2*>(c_in) : c.d_psi;
    roks::apply_operator(c, src, mask, reinterpret_cast<double2*>(h_out), false);
  });
}

roks_status roks_apply_h_noalloc_d(roks_ctx ctx, const void* c_in, uint32_t mask, void* h_out) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(h_out, ROKS_ERR_ARG, "output is NULL");
    if (mask) channel_count(c, mask);
    roks::apply_noalloc(c, reinterpret_cast<const double2*>(c_in), mask,
                        reinterpret_cast<double2*>(h_out));
  });
}

roks_status roks_energy_gradient(roks_ctx ctx, roks_energies* e, double* grad, double* theta) {
  return guard(ctx, [&](roks::Ctx& c) {
    roks_energies en;
    roks::energy_gradient(c, &en);
    if (e) *e = en;
    if (grad)
      ROKS_HIP(hipMemcpyAsync(grad, c.d_gI, (size_t)c.nb * c.npw * sizeof(double2),
                              hipMemcpyDeviceToHost, c.stream));
    if (theta)
      ROKS_HIP(hipMemcpyAsync(theta, c.d_theta, (size_t)c.nb * c.nb * sizeof(double),
                              hipMemcpyDeviceToHost, c.stream));
    ROKS_HIP(hipStreamSynchronize(c.stream));
  });
}

roks_status roks_subspace(roks_ctx ctx, double* R, double* kappa, double* A) {
  return guard(ctx, [&](roks::Ctx& c) {
    roks::energy_gradient(c, nullptr, nullptr, true);
    const size_t nn = (size_t)c.nb * c.nb * sizeof(double);
    if (R) ROKS_HIP(hipMemcpyAsync(R, c.d_R, nn, hipMemcpyDeviceToHost, c.stream));
    if (kappa) ROKS_HIP(hipMemcpyAsync(kappa, c.d_kappa, nn, hipMemcpyDeviceToHost, c.stream));
    if (A) ROKS_HIP(hipMemcpyAsync(A, c.d_A, nn, hipMemcpyDeviceToHost, c.stream));
    ROKS_HIP(hipStreamSynchronize(c.stream));
  });
}

roks_status roks_pcg_step(roks_ctx ctx, roks_step_info* info) {
  return guard(ctx, [&](roks::Ctx& c) { roks::pcg_step(c, info); });
}

roks_status roks_graph_steps(roks_ctx ctx, int32_t k, roks_step_info* info, int32_t* accepted) {
  return guard(ctx, [&](roks::Ctx& c) {
    const int a = roks::graph_steps(c, k, info);
    if (accepted) *accepted = a;
  });
}

roks_status roks_diis_step(roks_ctx ctx, const roks_diis_params* params, roks_diis_info* info) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(params, ROKS_ERR_ARG, "params is NULL");
    roks::diis_step(c, *params, info);
  });
}

roks_status roks_diis_solve(roks_ctx ctx, const roks_diis_params* params, double tol, int32_t maxiter,
                            roks_diis_info* last, int32_t* iterations) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(params, ROKS_ERR_ARG, "params is NULL");
    ROKS_CHECK(tol > 0 && maxiter > 0, ROKS_ERR_ARG, "tol and maxiter must be > 0");
    roks_diis_info info{}, prev{};
    int it = 0, hits = 0;
    while (it < maxiter) {
      roks::diis_step(c, *params, &info);
      if (it > 0 && std::fabs(info.E - prev.E) < tol) ++hits;
      else hits = 0;
      prev = info;
      ++it;
      if (hits >= 2) break;
    }
    if (last) *last = info;
    if (iterations) *iterations = it;
  });
}

roks_status roks_diis_reset(roks_ctx ctx) {
  return guard(ctx, [&](roks::Ctx& c) { roks::reset_diis(c); });
}

roks_status roks_reset_cg(roks_ctx ctx) {
  return guard(ctx, [&](roks::Ctx& c) { roks::reset_cg(c); });
}

roks_status roks_set_restart(roks_ctx ctx, int32_t period) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(period >= 0, ROKS_ERR_ARG, "period must be >= 0");
    c.restart_period = period;
  });
}

roks_status roks_set_precision(roks_ctx ctx, int32_t precision) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(precision == ROKS_FP64 || precision == ROKS_FP32 || precision == ROKS_FP32_BF16X3,
               ROKS_ERR_ARG, "unknown precision");
    // the FFT tier and the projector-product tier
    const int fft = precision == ROKS_FP64 ? ROKS_FP64 : ROKS_FP32;
    const bool bf3 = precision == ROKS_FP32_BF16X3;
    if (fft == ROKS_FP32 && !c.d_vsh32) {
      c.d_vsh32 = roks::dalloc<float>(c, (size_t)c.nsocc * c.ntot);
      c.d_vloc32 = roks::dalloc<float>(c, (size_t)2 * c.nconf * c.ntot);
    }
    if (fft != c.prec || bf3 != c.bf3) c.potentials_valid = false;
    const bool left_bf3 = c.bf3 && !bf3;
    c.prec = fft;
    c.bf3 = bf3;
    if (left_bf3 && c.has_q && c.have_orbitals) {
      // the BF16x3 products left the S-Gram's q part at their rounding
      roks::reset_cg(c);
      roks::orthonormalize(c, c.d_psi);
    }
  });
}

roks_status roks_solve(roks_ctx ctx, double tol, int32_t maxiter, roks_step_info* last,
                       int32_t* iterations) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(tol > 0 && maxiter > 0, ROKS_ERR_ARG, "tol and maxiter must be > 0");
    int hits = 0, it = 0;
    bool retried = false, linesearch_failed = false, done = false;
    roks_step_info info{};
    constexpr int kChunk = 8;
    roks_step_info recs[kChunk];
    while (it < maxiter && !done) {
      if ((c.flags & ROKS_FLAG_GRAPH) && it + kChunk <= maxiter && roks::graph_eligible(c)) {
        // graph mode: the accepted iterations of one replay, in order; after
        // a rejected one the host step below takes over
        const int acc = roks::graph_steps(c, kChunk, recs);
        for (int i = 0; i < acc; ++i) {
          info = recs[i];
          ++it;
          retried = false;
          hits = std::fabs(info.E1 - info.E0) < tol ? hits + 1 : 0;
          if (hits >= 2) done = true;
        }
        if (done || acc == kChunk) continue;
      }
      roks::pcg_step(c, &info);
      ++it;
      if (info.stalled) {
        // a stall moves nothing: drop the carried directions and retry once
        // from the preconditioned gradient before judging it
        if (!retried) {
          roks::reset_cg(c);
          retried = true;
          continue;
        }
        // the energy resolution of the tier
        const double rel = c.bf3 ? 2e-5 : c.prec == ROKS_FP32 ? 2e-6 : 1e-12;
        const double resolution = rel * std::max(1.0, std::fabs(info.E0));
        if (std::fabs(info.dE0) * roks::smallest_trial_step(c) >= std::max(tol, resolution))
          linesearch_failed = true;
        break;
      }
      retried = false;
      hits = std::fabs(info.E1 - info.E0) < tol ? hits + 1 : 0;
      if (hits >= 2) break;
    }
    ROKS_HIP(hipStreamSynchronize(c.stream));
    if (last) *last = info;
    if (iterations) *iterations = it;
    ROKS_CHECK(!linesearch_failed, ROKS_ERR_LINESEARCH,
               "no energy decrease found although the gradient predicts one above the tolerance");
  });
}

roks_status roks_forces(roks_ctx ctx, double* f) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(f || c.natoms == 0, ROKS_ERR_ARG, "output is NULL");
    roks::forces(c, f);
  });
}

roks_status roks_synchronize(roks_ctx ctx) {
  return guard(ctx, [&](roks::Ctx& c) { ROKS_HIP(hipStreamSynchronize(c.stream)); });
}

}  // extern "C"

extern "C" {

roks_status roks_timing_enable(roks_ctx ctx, int32_t enable) {
  return guard(ctx, [&](roks::Ctx& c) {
    roks::clear_timing(c);
    c.timing = enable != 0;
  });
}

roks_status roks_timing_only(roks_ctx ctx, const char* kernel) {
  return guard(ctx, [&](roks::Ctx& c) { c.timing_only = kernel ? kernel : ""; });
}

roks_status roks_timing_read(roks_ctx ctx, const char* kernel, double* total_ms, int32_t* launches,
                             double* bytes, double* flops) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(kernel, ROKS_ERR_ARG, "kernel name is NULL");
    ROKS_HIP(hipStreamSynchronize(c.stream));
    double ms = 0.0, by = 0.0, fl = 0.0;
    int32_t n = 0;
    for (auto& t : c.timed) {
      if (t.name != kernel) continue;
      float e = 0.f;
      ROKS_HIP(hipEventElapsedTime(&e, t.a, t.b));
      ms += e;
      by += t.bytes;
      fl += t.flops;
      ++n;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
  });
}

// ---------------------------------------------------------------------------
// learned rescaling of the preconditioner
// ---------------------------------------------------------------------------
roks_status roks_mlp_create(const float* theta, uint64_t seed, void* hip_stream, roks_mlp* out) {
  if (!out) return ROKS_ERR_ARG;
  *out = nullptr;
  roks_mlp mlp = new (std::nothrow) roks_mlp_s;
  if (!mlp) return ROKS_ERR_OOM;
  try {
    if (hip_stream) {
      mlp->m.stream = static_cast<hipStream_t>(hip_stream);
    } else {
      ROKS_HIP(hipStreamCreate(&mlp->m.stream));
      mlp->m.own_stream = true;
    }
    roks::mlp_init(mlp->m, theta, seed);
  } catch (const roks::Error& e) {
    g_create_error = e.msg;
    roks::mlp_free(mlp->m);
    delete mlp;
    return e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    roks::mlp_free(mlp->m);
    delete mlp;
    return ROKS_ERR_HIP;
  }
  *out = mlp;
  return ROKS_OK;
}

roks_status roks_mlp_destroy(roks_mlp mlp) {
  if (!mlp) return ROKS_ERR_ARG;
  roks::mlp_free(mlp->m);
  delete mlp;
  return ROKS_OK;
}

const char* roks_mlp_last_error(roks_mlp mlp) {
  if (!mlp) return g_create_error.c_str();
  return mlp->m.last_error.c_str();
}

roks_status roks_mlp_set_params(roks_mlp mlp, const float* theta) {
  return guard_mlp(mlp, [&](roks::Mlp& m) {
    ROKS_CHECK(theta != nullptr, ROKS_ERR_ARG, "theta is NULL");
    roks::mlp_set_params(m, theta);
  });
}

roks_status roks_mlp_get_params(roks_mlp mlp, float* theta) {
  return guard_mlp(mlp, [&](roks::Mlp& m) {
    ROKS_CHECK(theta != nullptr, ROKS_ERR_ARG, "theta is NULL");
    ROKS_HIP(hipMemcpyAsync(theta, m.d_p, ROKS_MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost,
                            m.stream));
    ROKS_HIP(hipStreamSynchronize(m.stream));
  });
}

roks_status roks_mlp_forward(roks_mlp mlp, const float* x, int64_t nsamples, float* o) {
  return guard_mlp(mlp, [&](roks::Mlp& m) {
    ROKS_CHECK(x && o, ROKS_ERR_ARG, "x and o must not be NULL");
    ROKS_CHECK(nsamples > 0 && nsamples <= (int64_t)1 << 30, ROKS_ERR_SHAPE,
               "nsamples must be in 1 .. 2^30");
    for (int64_t i = 0; i < 3 * nsamples; ++i)
      ROKS_CHECK(std::isfinite(x[i]), ROKS_ERR_NAN, "non-finite feature");
    float* dx = nullptr;
    float* dout = nullptr;
    ROKS_HIP(hipMalloc(&dx, (size_t)nsamples * 3 * sizeof(float)));
    if (hipMalloc(&dout, (size_t)nsamples * sizeof(float)) != hipSuccess) {
      (void)hipFree(dx);
      throw roks::Error{ROKS_ERR_OOM, "hipMalloc failed"};
    }
    hipError_t e = hipMemcpyAsync(dx, x, (size_t)nsamples * 3 * sizeof(float),
                                  hipMemcpyHostToDevice, m.stream);
    if (e == hipSuccess) {
      try {
        roks::mlp_forward(m, dx, (int)nsamples, dout, nullptr, m.stream);
      } catch (...) {
        e = hipErrorLaunchFailure;
      }
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(o, dout, (size_t)nsamples * sizeof(float), hipMemcpyDeviceToHost, m.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m.stream);
    (void)hipFree(dx);
    (void)hipFree(dout);
    ROKS_HIP(e);
  });
}

roks_status roks_mlp_num_samples(roks_mlp mlp, int64_t* nsamples, int32_t* nsegments) {
  return guard_mlp(mlp, [&](roks::Mlp& m) {
    if (nsamples) *nsamples = m.S;
    if (nsegments) *nsegments = m.nseg;
  });
}

roks_status roks_mlp_get_samples(roks_mlp mlp, float* x, double* moments,
                                 int32_t* segment_offsets) {
  return guard_mlp(mlp, [&](roks::Mlp& m) {
    if (m.S > 0) {
      if (x)
        ROKS_HIP(hipMemcpyAsync(x, m.d_X, (size_t)m.S * 3 * sizeof(float), hipMemcpyDeviceToHost,
                                m.stream));
      if (moments)
        for (int r = 0; r < 3; ++r)
          ROKS_HIP(hipMemcpyAsync(moments + (size_t)r * m.S, m.d_abg + (size_t)r * m.Scap,
                                  (size_t)m.S * sizeof(double), hipMemcpyDeviceToHost, m.stream));
      ROKS_HIP(hipStreamSynchronize(m.stream));
    }
    if (segment_offsets)
      std::memcpy(segment_offsets, m.band_off.data(), m.band_off.size() * sizeof(int32_t));
  });
}

roks_status roks_mlp_clear_samples(roks_mlp mlp) {
  return guard_mlp(mlp, [&](roks::Mlp& m) { roks::mlp_clear_samples(m); });
}

roks_status roks_mlp_loss_grad(roks_mlp mlp, double* loss, float* grad) {
  return guard_mlp(mlp, [&](roks::Mlp& m) {
    roks::mlp_loss_grad(m, m.d_loss);
    double h[2] = {0.0, 0.0};
    ROKS_HIP(hipMemcpyAsync(h, m.d_loss, sizeof(h), hipMemcpyDeviceToHost, m.stream));
    if (grad)
      ROKS_HIP(hipMemcpyAsync(grad, m.d_g, ROKS_MLP_PARAMS * sizeof(float), hipMemcpyDeviceToHost,
                              m.stream));
    ROKS_HIP(hipStreamSynchronize(m.stream));
    if (loss) *loss = h[0];
  });
}

roks_status roks_mlp_train(roks_mlp mlp, int32_t steps, double lr, double* loss_history) {
  return guard_mlp(mlp, [&](roks::Mlp& m) {
    ROKS_CHECK(steps >= 0, ROKS_ERR_ARG, "steps must be >= 0");
    ROKS_CHECK(lr > 0 && std::isfinite(lr), ROKS_ERR_ARG, "lr must be > 0");
    ROKS_CHECK(m.S > 0 && m.nseg > 0, ROKS_ERR_STATE, "the network has no training samples");
    if (steps == 0) return;
    double* hist = nullptr;
    ROKS_HIP(hipMalloc(&hist, (size_t)steps * 2 * sizeof(double)));
    hipError_t e = hipSuccess;
    try {
      for (int k = 0; k < steps; ++k) {
        roks::mlp_loss_grad(m, hist + 2 * k);
        roks::mlp_adam(m, lr);
      }
    } catch (...) {
      e = hipErrorLaunchFailure;
    }
    std::vector<double> h((size_t)steps * 2);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h.data(), hist, h.size() * sizeof(double), hipMemcpyDeviceToHost, m.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m.stream);
    (void)hipFree(hist);
    ROKS_HIP(e);
    if (loss_history)
      for (int k = 0; k < steps; ++k) loss_history[k] = h[2 * (size_t)k];
  });
}

roks_status roks_record(roks_ctx ctx, int32_t max_records, int32_t stride) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(max_records >= 0 && stride >= 1, ROKS_ERR_ARG,
               "max_records must be >= 0 and stride >= 1");
    drop_records(c);
    if (max_records == 0) return;
    roks::build_gshells(c);
    const size_t band = (size_t)c.nb * c.npw;
    c.d_rec_psi = roks::dalloc<double2>(c, band * max_records);
    c.d_rec_kg = roks::dalloc<double2>(c, band * max_records);
    c.d_rec_feat = roks::dalloc<float>(c, 3 * (size_t)c.nb * c.nsh * max_records);
    c.d_rec_valid = roks::dalloc<int32_t>(c, (size_t)c.nb * max_records);
    c.d_rec_ekin = roks::dalloc<double>(c, (size_t)c.nb * max_records);
    if (!c.d_rec_sel) c.d_rec_sel = roks::dalloc<int32_t>(c, c.nb);
    c.rec_max = max_records;
    c.rec_stride = stride;
    c.rec_count = 0;
    ROKS_HIP(hipStreamSynchronize(c.stream));
  });
}

roks_status roks_mlp_collect(roks_mlp mlp, roks_ctx ctx, int32_t* used, int32_t* skipped) {
  if (!mlp) return ROKS_ERR_ARG;
  return guard(ctx, [&](roks::Ctx& c) {
    int u = 0, k = 0;
    roks::collect_records(c, mlp->m, &u, &k);
    if (used) *used = u;
    if (skipped) *skipped = k;
  });
}

roks_status roks_set_mlp(roks_ctx ctx, roks_mlp mlp) {
  return guard(ctx, [&](roks::Ctx& c) {
    if (mlp) {
      roks::build_gshells(c);
      ROKS_HIP(hipStreamSynchronize(mlp->m.stream));
      c.mlp = &mlp->m;
    } else {
      c.mlp = nullptr;
    }
  });
}

}  // extern "C"
