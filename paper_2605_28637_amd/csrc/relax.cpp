// Geometry relaxation and the Franck-Condon cycle of Sec. IV B, host-side
// drivers over the library's own entry points (the electronic solve, the
// Hellmann-Feynman forces of Eq. force_hf, new positions), with the same
// steps as the oracle's readings G0-G4:
//   G0 total energy = electronic E + sum_{I<J} sum_t B exp(-|R_I - R_J - t| / rho)
//      over the 27 nearest cell translations t (the ions' repulsion, which
//      the synthetic Gaussian-well atoms lack);
//   G1 BFGS on the Cartesian positions, H_0 = h0 I, s = H F capped at
//      max_step per atom, the BFGS update of H when s.y > 0 (y = F_old -
//      F_new), else H = h0 I;
//   G2 each geometry's orbitals by the CG solve from the previous ones
//      (S-orthonormalised first with overlap coefficients, S moving with
//      the atoms), restarted every scf_restart iterations;
//   G3 a step that raises the energy is halved (at most four times, H reset);
//   G4 stop at max_I |F_I| < fmax or after maxsteps.
#include <cmath>
#include <cstring>
#include <vector>

#include "roks_internal.h"

namespace {

struct PairTerm {
  double E = 0.0;
  std::vector<double> F;
};

PairTerm pair_repulsion(const roks::Ctx& c, double B, double rho) {
  PairTerm p;
  const int nat = c.natoms;
  p.F.assign(3 * (size_t)nat, 0.0);
  if (B == 0.0) return p;
  for (int I = 0; I < nat; ++I)
    for (int J = I + 1; J < nat; ++J)
      for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j)
          for (int k = -1; k <= 1; ++k) {
            double d[3];
            for (int a = 0; a < 3; ++a)
              d[a] = c.pos[3 * I + a] - c.pos[3 * J + a] -
                     (i * c.cell[0][a] + j * c.cell[1][a] + k * c.cell[2][a]);
            const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double e = B * std::exp(-r / rho);
            p.E += e;
            for (int a = 0; a < 3; ++a) {
              const double f = (e / rho) * d[a] / r;
              p.F[3 * I + a] += f;
              p.F[3 * J + a] -= f;
            }
          }
  return p;
}

void check(roks_status s) {
  if (s != ROKS_OK) throw roks::Error{s, "relaxation: an electronic step failed"};
}

struct Geometry {
  double E = 0.0;              // total energy (G0)
  std::vector<double> F;       // total forces
  int iterations = 0;          // CG iterations of the solve
};

// G2 + G0 at the context's current positions
Geometry electrons(roks_ctx ctx, const roks_relax_params& p, bool want_forces) {
  roks::Ctx& c = ctx->c;
  Geometry g;
  roks_step_info info{};
  int32_t it = 0;
  // a search that stalls at the arithmetic's resolution ends the solve
  // there; the context's restart period is restored afterwards
  if (c.has_q) {
    c.potentials_valid = false;
    roks::reset_cg(c);
    roks::orthonormalize(c, c.d_psi);
  }
  const int keep_period = c.restart_period;
  c.restart_period = p.scf_restart;
  c.since_restart = 0;
  const roks_status st = roks_solve(ctx, p.scf_tol, p.scf_maxiter, &info, &it);
  c.restart_period = keep_period;
  if (st != ROKS_ERR_LINESEARCH) check(st);
  const PairTerm pr = pair_repulsion(c, p.pair_B, p.pair_rho);
  g.E = info.E1 + pr.E;
  g.iterations = it;
  if (want_forces) {
    g.F.assign(3 * (size_t)c.natoms, 0.0);
    if (c.natoms > 0) check(roks_forces(ctx, g.F.data()));
    for (size_t i = 0; i < g.F.size(); ++i) g.F[i] += pr.F[i];
  }
  return g;
}

double max_force(const std::vector<double>& F) {
  double m = 0.0;
  for (size_t I = 0; 3 * I + 2 < F.size(); ++I)
    m = std::max(m, std::sqrt(F[3 * I] * F[3 * I] + F[3 * I + 1] * F[3 * I + 1] + F[3 * I + 2] * F[3 * I + 2]));
  return m;
}

void set_positions(roks_ctx ctx, const std::vector<double>& x) { check(roks_set_positions(ctx, x.data())); }

void relax_impl(roks_ctx ctx, const roks_relax_params& p, roks_relax_info* out) {
  roks::Ctx& c = ctx->c;
  const int n = 3 * c.natoms;
  std::vector<double> x = c.pos;
  Geometry g = electrons(ctx, p, true);
  int nscf = g.iterations, steps = 0;
  std::vector<double> H((size_t)n * n, 0.0);
  auto reset_h = [&]() {
    std::fill(H.begin(), H.end(), 0.0);
    for (int i = 0; i < n; ++i) H[(size_t)i * n + i] = p.h0;
  };
  reset_h();
  std::vector<double> s(n), xn(n), y(n), Hy(n);
  // the orbitals of the accepted geometry: every trial solve starts from them
  std::vector<double> keep((size_t)c.nb * c.npw * 2);
  while (steps < p.maxsteps && max_force(g.F) >= p.fmax) {
    check(roks_get_coeffs(ctx, keep.data()));
    for (int i = 0; i < n; ++i) {
      double v = 0.0;
      for (int j = 0; j < n; ++j) v += H[(size_t)i * n + j] * g.F[j];
      s[i] = v;
    }
    const double big = max_force(s);
    if (big > p.max_step)
      for (double& v : s) v *= p.max_step / big;
    Geometry gn;
    for (int halving = 0; halving < 5; ++halving) {
      for (int i = 0; i < n; ++i) xn[i] = x[i] + s[i];
      set_positions(ctx, xn);
      gn = electrons(ctx, p, false);
      nscf += gn.iterations;
      if (gn.E <= g.E || halving == 4) break;
      for (double& v : s) v *= 0.5;
      reset_h();
      check(roks_set_coeffs(ctx, keep.data(), 0));
    }
    gn.F.assign(n, 0.0);
    if (c.natoms > 0) check(roks_forces(ctx, gn.F.data()));
    const PairTerm pr = pair_repulsion(c, p.pair_B, p.pair_rho);
    for (int i = 0; i < n; ++i) gn.F[i] += pr.F[i];
    double sy = 0.0;
    for (int i = 0; i < n; ++i) {
      y[i] = g.F[i] - gn.F[i];
      sy += s[i] * y[i];
    }
    if (sy > 0.0) {
      // H <- (I - r s y^T) H (I - r y s^T) + r s s^T, r = 1 / s.y
      const double r = 1.0 / sy;
      for (int i = 0; i < n; ++i) {
        double v = 0.0;
        for (int j = 0; j < n; ++j) v += H[(size_t)i * n + j] * y[j];
        Hy[i] = v;
      }
      double yHy = 0.0;
      for (int i = 0; i < n; ++i) yHy += y[i] * Hy[i];
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          H[(size_t)i * n + j] += -r * (s[i] * Hy[j] + Hy[i] * s[j]) + (r * r * yHy + r) * s[i] * s[j];
    } else {
      reset_h();
    }
    x = xn;
    g = gn;
    ++steps;
  }
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->E = g.E;
    out->fmax = max_force(g.F);
    out->steps = steps;
    out->scf_iterations = nscf;
    out->converged = max_force(g.F) < p.fmax ? 1 : 0;
  }
}

void check_params(const roks_relax_params* p) {
  ROKS_CHECK(p, ROKS_ERR_ARG, "params is NULL");
  ROKS_CHECK(p->fmax > 0 && p->scf_tol > 0 && p->scf_maxiter > 0 && p->scf_restart >= 0 &&
                 p->maxsteps >= 0 &&
                 p->max_step > 0 && p->h0 > 0 && p->pair_B >= 0 && p->pair_rho > 0,
             ROKS_ERR_ARG, "relaxation parameters out of range");
}

template <typename F>
roks_status guarded(roks_ctx ctx, F&& f) {
  if (!ctx) return ROKS_ERR_ARG;
  try {
    f();
    return ROKS_OK;
  } catch (const roks::Error& e) {
    ctx->c.last_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    ctx->c.last_error = e.what();
    return ROKS_ERR_HIP;
  }
}

}  // namespace

extern "C" {

roks_status roks_get_positions(roks_ctx ctx, double* pos) {
  return guarded(ctx, [&]() {
    ROKS_CHECK(pos || ctx->c.natoms == 0, ROKS_ERR_ARG, "output is NULL");
    std::copy(ctx->c.pos.begin(), ctx->c.pos.end(), pos);
  });
}

roks_status roks_relax(roks_ctx ctx, const roks_relax_params* params, roks_relax_info* info) {
  return guarded(ctx, [&]() {
    check_params(params);
    ROKS_CHECK(ctx->c.have_orbitals, ROKS_ERR_STATE, "no orbitals set");
    relax_impl(ctx, *params, info);
  });
}

roks_status roks_franck_condon(roks_ctx gs, roks_ctx ex, const roks_relax_params* params,
                               const double* masses, roks_fc_result* out) {
  if (!gs || !ex) return ROKS_ERR_ARG;
  return guarded(gs, [&]() {
    check_params(params);
    roks::Ctx& cg = gs->c;
    roks::Ctx& ce = ex->c;
    ROKS_CHECK(masses && out, ROKS_ERR_ARG, "masses or output is NULL");
    ROKS_CHECK(cg.natoms == ce.natoms && cg.nb == ce.nb && cg.npw == ce.npw, ROKS_ERR_SHAPE,
               "the two contexts describe different systems");
    ROKS_CHECK(cg.have_orbitals, ROKS_ERR_STATE, "no ground-state orbitals set");
    std::memset(out, 0, sizeof(*out));
    // ground-state relaxation: R_gs, E^gs(R_gs)
    roks_relax_info ig{};
    relax_impl(gs, *params, &ig);
    const std::vector<double> Rgs = cg.pos;
    // the excited state at R_gs from the ground-state orbitals: E^ex(R_gs)
    std::vector<double> cbuf((size_t)cg.nb * cg.npw * 2);
    check(roks_get_coeffs(gs, cbuf.data()));
    set_positions(ex, Rgs);
    check(roks_set_coeffs(ex, cbuf.data(), ce.has_q ? 1 : 0));
    const Geometry eg = electrons(ex, *params, false);
    // excited-state relaxation from there: R_ex, E^ex(R_ex)
    roks_relax_info ie{};
    relax_impl(ex, *params, &ie);
    const std::vector<double> Rex = ce.pos;
    // the ground state at R_ex from its relaxed orbitals: E^gs(R_ex)
    set_positions(gs, Rex);
    check(roks_set_coeffs(gs, cbuf.data(), cg.has_q ? 1 : 0));
    const Geometry ge = electrons(gs, *params, false);
    out->E_gs_at_gs = ig.E;
    out->E_ex_at_gs = eg.E;
    out->E_ex_at_ex = ie.E;
    out->E_gs_at_ex = ge.E;
    out->E_abs = eg.E - ig.E;
    out->E_FC_ex = eg.E - ie.E;
    out->E_FC_gs = ge.E - ig.E;
    out->E_emi = out->E_abs - out->E_FC_ex - out->E_FC_gs;
    double q = 0.0;
    for (int I = 0; I < cg.natoms; ++I)
      for (int a = 0; a < 3; ++a) {
        const double d = Rex[3 * I + a] - Rgs[3 * I + a];
        q += masses[I] * d * d;
      }
    out->dQ = std::sqrt(q);
    out->gs_steps = ig.steps;
    out->ex_steps = ie.steps;
    out->converged = (ig.converged && ie.converged) ? 1 : 0;
  });
}

}  // extern "C"
