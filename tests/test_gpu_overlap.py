"""The general overlap S = 1 + sum q |beta><beta| (Sec. II A; reading R27 of
the oracle) on the GPU against the oracle beyond the per-call parity cases
of test_gpu_parity.py: the S-orthonormalisation after a move of the atoms,
DIIS steps, a converged ground state against the dense generalised
eigenproblem, the forces with their overlap term at convergence, the first
relaxation steps, and the checks of q at creation.  FP64 bar as in the other
parity tests."""
import numpy as np
import pytest

from helpers import SphereMap, band_rel, ensure_built, small_molecule
from oracle import dense, diis as od, relax as orl, roks as orc
from paper_2605_28637_amd import inputs

pytestmark = pytest.mark.gpu


def _pair(system):
    rb = ensure_built()
    print("case", system.get("name"), system["grid"], system["nbands"], flush=True)
    g = rb.Roks(system)
    m = orc.Model(system)
    mp = SphereMap(g.miller(), m.miller)
    g.set_coeffs(inputs.random_coefficients(g.miller(), system["cell"], g.nb, system["seed"]), True)
    psi = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, system["seed"]), m)
    return rb, g, m, mp, psi


def test_moved_atoms_reorthonormalise_in_the_new_metric():
    rb, g, m, mp, psi = _pair(inputs.with_overlap(inputs.tiny_cell(), 0.5))
    pos = m.pos + np.array([[0.3, -0.2, 0.1], [-0.1, 0.25, 0.0]])
    g.set_positions(pos)
    m.set_positions(pos)
    want = orc.orthonormalize(psi, m)
    assert band_rel(mp.to_full(g.get_coeffs()), want) < 1e-12
    e, _, _ = g.energy_gradient()
    assert abs(e["E"] - orc.energy(m, want)) < 1e-10 * max(1.0, abs(e["E"]))
    g.close()


@pytest.mark.parametrize("asym", [False, True])
def test_diis_steps_with_overlap_match_the_oracle(asym):
    rb, g, m, mp, psi = _pair(inputs.with_overlap(small_molecule(), 0.4))
    st = od.DiisState(psi)
    for i in range(4):
        gi = g.diis_step(history=4, step=0.3, asymmetric=asym)
        oi = od.diis_step(m, st, history=4, step=0.3, asymmetric=asym)
        print(i, gi["E"], oi.E, gi["rnorm2"], oi.rnorm2, flush=True)
        assert abs(gi["E"] - oi.E) < 1e-10 * max(1.0, abs(oi.E)), i
        assert abs(gi["rnorm2"] - oi.rnorm2) < 1e-8 * oi.rnorm2, i
        assert gi["used"] == oi.used, i
    assert band_rel(mp.to_full(g.get_coeffs()), st.psi) < 1e-8
    g.close()


def test_ground_state_with_overlap_solves_the_generalised_problem():
    """CG on the GPU reaches the energy of the dense SCF over H c = eps S c;
    the forces there match the oracle's (with the overlap term of Eq.
    force_hf)."""
    s = inputs.with_overlap(inputs.with_configuration(inputs.tiny_cell(), "gs"), 0.5)
    rb, g, m, mp, psi = _pair(s)
    info, it = g.solve(tol=1e-12, maxiter=800)
    E_scf, _, _ = dense.scf_closed_shell(m, 5)
    print("GPU", info["E1"], it, "dense", E_scf, flush=True)
    assert abs(info["E1"] - E_scf) < 1e-9
    F = g.forces()
    Fo = orc.forces(m, mp.to_full(g.get_coeffs()))
    T = orc.overlap_force_term(m, mp.to_full(g.get_coeffs()))
    assert np.abs(F - Fo).max() < 1e-8 * max(1.0, np.abs(Fo).max())
    assert np.abs(T).max() > 1e-4
    g.close()


def test_singlet_forces_with_overlap_at_convergence():
    s = inputs.with_overlap(inputs.tiny_cell(), 0.5)
    rb, g, m, mp, psi = _pair(s)
    g.solve(tol=1e-12, maxiter=800)
    c = mp.to_full(g.get_coeffs())
    F = g.forces()
    Fo = orc.forces(m, c)
    print(F, Fo, flush=True)
    assert np.abs(F - Fo).max() < 1e-8 * max(1.0, np.abs(Fo).max())
    g.close()


def test_relax_first_steps_with_overlap_match_the_oracle():
    s = inputs.with_overlap(inputs.dimer(configuration="gs"), 0.3)
    rb, g, m, mp, psi = _pair(s)
    info = g.relax(maxsteps=2)
    r = orl.relax(m, psi, orl.RelaxParams(maxsteps=2))
    print(info, r.E, r.steps, flush=True)
    assert info["steps"] == r.steps == 2
    assert abs(info["E"] - r.E) < 1e-9
    assert np.abs(g.get_positions() - r.pos).max() < 1e-7
    g.close()


@pytest.mark.parametrize("bad", ["asymmetric", "mixed_l", "nonfinite"])
def test_overlap_coefficients_are_checked(bad):
    rb = ensure_built()
    s = inputs.with_overlap(small_molecule(), 0.4)
    sp = [dict(x) for x in s["species"]]
    q = np.array(sp[0]["q"], dtype=float)
    if bad == "asymmetric":
        q = np.array([[0.4, 0.0], [0.0, 0.24]])
        sp[0]["proj"] = [(0, 0.6), (0, 1.0)]
        q[0, 1] = 0.1
    elif bad == "mixed_l":
        q[0, 1] = q[1, 0] = 0.1  # s and p channels
    else:
        q[0, 0] = np.nan
    sp[0]["q"] = q
    s = dict(s, species=sp)
    with pytest.raises(rb.RoksError) as ei:
        rb.Roks(s)
    assert ei.value.status == 1
