"""Pins of the relaxation oracle (oracle/relax.py) on the CPU:

* the pair repulsion's forces (reading G0) are minus the central finite
  differences of its energy, in a non-cubic cell;
* the BFGS driver (G1, G3, G4) reaches the exact minimiser of a convex
  quadratic, a textbook property of the method;
* the Franck-Condon cycle of Sec. IV B on the dimer: both relaxed
  geometries are stationary (forces below the threshold), the two shifts
  are non-negative (each equilibrium minimises its own surface), the
  emission energy equals E^ex(R_ex) - E^gs(R_ex) (the paper's definitions
  combined), and Delta Q is the mass-weighted distance of the geometries."""
import numpy as np

from oracle import relax as orl
from oracle import roks as orc
from paper_2605_28637_amd import inputs


def test_pair_forces_are_minus_the_energy_gradient():
    rng = np.random.default_rng(5)
    cell = np.array([[6.0, 0.3, 0.0], [0.0, 7.0, 0.4], [0.2, 0.0, 6.5]])
    pos = rng.uniform(0, 6, size=(4, 3))
    B, rho = 1.3, 0.9
    E, F = orl.pair_repulsion(pos, cell, B, rho)
    h = 1e-5
    for I in range(4):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[I, a] += h
            pm[I, a] -= h
            d = (orl.pair_repulsion(pp, cell, B, rho)[0] - orl.pair_repulsion(pm, cell, B, rho)[0]) / (2 * h)
            assert abs(F[I, a] + d) < 1e-8 * max(1.0, abs(d)), (I, a)


def test_bfgs_reaches_the_minimiser_of_a_quadratic():
    rng = np.random.default_rng(3)
    Q = rng.normal(size=(6, 6))
    A = Q @ Q.T + 0.5 * np.eye(6)
    xs = rng.normal(size=6)

    def evaluate(x, state):
        d = x - xs
        return 0.5 * d @ A @ d, -(A @ d), state, 1

    p = orl.RelaxParams(fmax=1e-10, maxsteps=200, max_step=0.5, h0=0.1)
    x, E, F, _, steps, work, hist = orl.bfgs(evaluate, np.zeros(6), None, p)
    assert np.abs(x - xs).max() < 1e-9
    assert steps < 60
    assert all(hist[i + 1]["E"] <= hist[i]["E"] + 1e-15 for i in range(len(hist) - 1))


def test_franck_condon_cycle_identities():
    gs = inputs.dimer(configuration="gs")
    ex = inputs.dimer()
    m = orc.Model(gs)
    psi0 = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, gs["seed"]))
    p = orl.RelaxParams()
    masses = np.array([24.3, 16.0])
    fc = orl.franck_condon(gs, ex, psi0, masses, p)
    assert fc["gs_converged"] and fc["ex_converged"]
    assert fc["E_FC_ex"] > -1e-9 and fc["E_FC_gs"] > -1e-9
    assert abs(fc["E_emi"] - (fc["E_ex_at_ex"] - fc["E_gs_at_ex"])) < 1e-12
    assert fc["E_emi"] < fc["E_abs"]
    dQ = np.sqrt((masses[:, None] * (fc["R_ex"] - fc["R_gs"]) ** 2).sum())
    assert abs(fc["dQ"] - dQ) < 1e-12 and fc["dQ"] > 0.01
    # the excited equilibrium is stationary on the excited surface
    me = orc.Model(ex)
    me.set_positions(fc["R_ex"])
    st, h = orc.solve(me, psi0, tol=1e-11, maxiter=800, restart_period=20)
    F = orl.total_forces(me, st.psi, p)
    assert np.linalg.norm(F, axis=1).max() < 3 * p.fmax
