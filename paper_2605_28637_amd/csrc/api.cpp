// The C ABI (include/roks.h): argument checks, error translation, host <->
// device copies.  Every entry point catches the library's exceptions and
// returns a status; the message is kept per context.
#include <cmath>
#include <cstring>
#include <string>

#include "roks_internal.h"

struct roks_ctx_s {
  roks::Ctx c;
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

void upload_bands(roks::Ctx& c, double2* dst, const double* src) {
  ROKS_HIP(hipMemcpyAsync(dst, src, (size_t)c.nb * c.npw * sizeof(double2), hipMemcpyHostToDevice,
                          c.stream));
}

void check_finite_host(const roks::Ctx& c, const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    ROKS_CHECK(std::isfinite(v[i]), ROKS_ERR_NAN, "non-finite input coefficient");
}

}  // namespace

extern "C" {

const char* roks_version(void) { return "roks-gfx950 0.1 (fp64 tier)"; }

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
    upload_bands(c, c.d_psi, cf);
    if (orthonormalize) roks::orthonormalize(c, c.d_psi);
    ROKS_HIP(hipStreamSynchronize(c.stream));
    c.have_orbitals = true;
    c.potentials_valid = false;
    roks::reset_cg(c);
  });
}

roks_status roks_set_coeffs_d(roks_ctx ctx, const void* cf, int32_t orthonormalize) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(cf, ROKS_ERR_ARG, "coefficients are NULL");
    ROKS_HIP(hipMemcpyAsync(c.d_psi, cf, (size_t)c.nb * c.npw * sizeof(double2),
                            hipMemcpyDeviceToDevice, c.stream));
    if (orthonormalize) roks::orthonormalize(c, c.d_psi);
    c.have_orbitals = true;
    c.potentials_valid = false;
    roks::reset_cg(c);
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
    roks::energy_gradient(c, nullptr);
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

roks_status roks_reset_cg(roks_ctx ctx) {
  return guard(ctx, [&](roks::Ctx& c) { roks::reset_cg(c); });
}

roks_status roks_set_precision(roks_ctx ctx, int32_t precision) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(precision == ROKS_FP64 || precision == ROKS_FP32, ROKS_ERR_ARG, "unknown precision");
    if (precision == ROKS_FP32 && !c.d_vsh32) {
      c.d_vsh32 = roks::dalloc<float>(c, (size_t)c.nsocc * c.ntot);
      c.d_vloc32 = roks::dalloc<float>(c, (size_t)2 * c.nconf * c.ntot);
    }
    if (precision != c.prec) c.potentials_valid = false;
    c.prec = precision;
  });
}

roks_status roks_solve(roks_ctx ctx, double tol, int32_t maxiter, roks_step_info* last,
                       int32_t* iterations) {
  return guard(ctx, [&](roks::Ctx& c) {
    ROKS_CHECK(tol > 0 && maxiter > 0, ROKS_ERR_ARG, "tol and maxiter must be > 0");
    int hits = 0, it = 0;
    roks_step_info info{};
    while (it < maxiter) {
      roks::pcg_step(c, &info);
      ++it;
      hits = std::fabs(info.E1 - info.E0) < tol ? hits + 1 : 0;
      if (hits >= 2) break;
    }
    if (last) *last = info;
    if (iterations) *iterations = it;
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

}  // extern "C"
