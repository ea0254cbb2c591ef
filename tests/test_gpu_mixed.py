"""FP32 tier (FFTs, plane arithmetic and potentials in FP32; orbitals, kinetic
terms, band-space matrices, Gram / Cholesky / rotation, energies and line
search in FP64) against the FP64 oracle.

Per-call tolerances follow from the arithmetic: an FP32 transform of N^3
points carries ~1e-7 log2(N^3) relative error, an H-apply chains four of them
and a multiply, so 2e-6 relative (Frobenius) bounds apply and gradient; energy
terms come from FP32 densities summed in FP64, 2e-6 relative to the largest
term.  End-to-end targets: excitation energy within 1 meV (3.67e-5 Ha) and
forces within 1e-4 Ha/bohr of FP64.
"""
import numpy as np
import pytest

from helpers import SphereMap, ensure_built, rel, small_molecule
from oracle import roks as orc
from paper_2605_28637_amd import inputs

pytestmark = pytest.mark.gpu

MEV = 1.0 / 27211.386


def _pair(system, precision):
    rb = ensure_built()
    print("case", system.get("name"), system["grid"], system["nbands"], "prec", precision, flush=True)
    g = rb.Roks(system, precision=precision)
    m = orc.Model(system)
    mp = SphereMap(g.miller(), m.miller)
    g.set_coeffs(inputs.random_coefficients(g.miller(), system["cell"], g.nb, system["seed"]), True)
    psi = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, system["seed"]))
    return g, m, mp, psi


@pytest.mark.parametrize("case", ["tiny", "small_odd_bands", "molecule_box"])
def test_fp32_energies_apply_gradient(case):
    rb = ensure_built()
    s = {"tiny": inputs.tiny_cell, "small_odd_bands": small_molecule,
         "molecule_box": inputs.molecule_box}[case]()
    g, m, mp, psi = _pair(s, rb.FP32)
    e, gi, th = g.energy_gradient()
    gr = orc.gradient(m, psi)
    scale = max(1.0, max(abs(v) for t in gr.pot.terms.values() for v in t))
    assert abs(e["E"] - gr.pot.E) < 2e-6 * scale
    Y = mp.to_full(g.apply_h())
    assert rel(Y, gr.Y) < 2e-6
    assert np.linalg.norm(mp.to_full(gi) - gr.gI) < 2e-6 * np.linalg.norm(gr.Y)
    assert np.abs(th - gr.theta).max() < 2e-6 * np.abs(gr.theta).max()
    g.close()


def test_fp32_ladder_reaches_fp64_minimum_tiny():
    """FP32 iterations to 1e-6 Ha, then FP64 polish to 1e-10 Ha: the same
    energy as the FP64 oracle from the same start, for the ground state (one
    minimum).  From a random start the tiny singlet has several stationary
    points (E = -0.14627, -0.14762, -0.16252 Ha): FP64 runs pass the first
    and leave it along a direction whose energy change is below the FP32
    tier's rounding, so which one a ladder reaches is not a property of the
    arithmetic; the singlet is tested from the ground-state orbitals below."""
    rb = ensure_built()
    s = inputs.with_configuration(inputs.tiny_cell(), "gs")
    g, m, mp, psi = _pair(s, rb.FP32)
    i32, n32 = g.solve(tol=1e-6, maxiter=400)
    g.set_precision(rb.FP64)
    i64, n64 = g.solve(tol=1e-10, maxiter=600)
    st, hist = orc.solve(m, psi, tol=1e-10, maxiter=600, orthonormalize_start=False)
    assert abs(i64["E1"] - hist[-1].E1) < 1e-9
    assert i64["E1"] <= i32["E1"] + 1e-9
    g.close()


def _ladder(rb, r, precision, switch_tol, tol):
    """FP32 iterations until |dE| < switch_tol, then FP64 to tol (a pure
    FP64 run when precision is FP64)."""
    if precision == rb.FP32:
        r.solve(tol=switch_tol, maxiter=800)
        r.set_precision(rb.FP64)
    info, _ = r.solve(tol=tol, maxiter=800)
    return info


def _gs_then_singlet_gpu(rb, system, precision, tol, switch_tol=1e-5):
    gs = inputs.with_configuration(system, "gs")
    g = rb.Roks(gs, precision=precision)
    g.set_coeffs(inputs.random_coefficients(g.miller(), gs["cell"], g.nb, gs["seed"]), True)
    ig = _ladder(rb, g, precision, switch_tol, tol)
    c = g.get_coeffs()
    g.close()
    r = rb.Roks(system, precision=precision)
    r.set_coeffs(c, True)
    ie = _ladder(rb, r, precision, switch_tol, tol)
    F = r.forces()
    r.close()
    return ig["E1"], ie["E1"], F


def _gs_then_singlet_oracle(system, tol):
    gs = inputs.with_configuration(system, "gs")
    mg = orc.Model(gs)
    st, hg = orc.solve(mg, inputs.random_coefficients(mg.miller, mg.cell, mg.nb, gs["seed"]),
                       tol=tol, maxiter=800)
    m = orc.Model(system)
    st2, he = orc.solve(m, st.psi, tol=tol, maxiter=800)
    return hg[-1].E1, he[-1].E1, orc.forces(m, st2.psi)


@pytest.mark.parametrize("case", ["tiny", "small_molecule"])
def test_fp32_ladder_excitation_energy_and_forces(case):
    """Ground state, then the singlet from the ground-state orbitals (the
    paper's protocol), with the precision ladder (FP32 to |dE| < 1e-5 Ha, FP64
    polish), against the FP64 oracle running the same protocol: excitation
    energy within 1 meV; singlet forces within 1e-4 Ha/bohr on the
    well-conditioned 12-band molecule (the tiny cell's flat valley leaves
    energy-converged states 1e-4 apart in force on both sides)."""
    rb = ensure_built()
    s = inputs.tiny_cell() if case == "tiny" else small_molecule(nb=12)
    tol = 1e-10 if case == "tiny" else 1e-12
    eg32, es32, F32 = _gs_then_singlet_gpu(rb, s, rb.FP32, tol)
    eg64, es64, F64 = _gs_then_singlet_oracle(s, tol)
    exc32, exc64 = es32 - eg32, es64 - eg64
    print("excitation ladder %.9f FP64 oracle %.9f Ha, diff %.2e Ha; max force diff %.2e"
          % (exc32, exc64, exc32 - exc64, np.abs(F32 - F64).max()))
    assert abs(exc32 - exc64) < MEV
    if case != "tiny":
        assert np.abs(F32 - F64).max() < 1e-4
