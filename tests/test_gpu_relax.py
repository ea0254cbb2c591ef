"""roks_relax / roks_franck_condon (Sec. IV B) against the relaxation
oracle (oracle/relax.py, readings G0-G4) on the dimer workload: the first
BFGS steps from the same start (positions to 1e-7 bohr, energies to 1e-9
Ha: the forces agree to the FP64 bar, so the steps do), then the whole
cycle -- E_abs, both Franck-Condon shifts and E_emi to 1e-8 Ha, Delta Q and
the two equilibrium geometries to 1e-5 (both runs stop at the same force
threshold along the same path)."""
import numpy as np
import pytest

from helpers import ensure_built
from oracle import relax as orl
from oracle import roks as orc
from paper_2605_28637_amd import inputs

pytestmark = pytest.mark.gpu

MASSES = np.array([24.3, 16.0])


def _start(system):
    rb = ensure_built()
    g = rb.Roks(system)
    g.set_coeffs(inputs.random_coefficients(g.miller(), system["cell"], g.nb, system["seed"]), True)
    m = orc.Model(system)
    psi = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, system["seed"]))
    return rb, g, m, psi


def test_relax_first_steps_match_the_oracle():
    s = inputs.dimer(configuration="gs")
    print("dimer gs relax 2 steps", flush=True)
    rb, g, m, psi = _start(s)
    info = g.relax(maxsteps=2)
    r = orl.relax(m, psi, orl.RelaxParams(maxsteps=2))
    print(info, r.E, r.steps)
    assert info["steps"] == r.steps == 2
    assert abs(info["E"] - r.E) < 1e-9
    assert np.abs(g.get_positions() - r.pos).max() < 1e-7
    g.close()


def test_franck_condon_cycle_matches_the_oracle():
    gs, ex = inputs.dimer(configuration="gs"), inputs.dimer()
    print("dimer Franck-Condon cycle", flush=True)
    rb, g, m, psi = _start(gs)
    e = rb.Roks(ex)
    out = rb.franck_condon(g, e, MASSES)
    Rex = g.get_positions()
    want = orl.franck_condon(gs, ex, psi, MASSES, orl.RelaxParams())
    print({k: out[k] for k in ("E_abs", "E_FC_ex", "E_FC_gs", "E_emi", "dQ", "gs_steps", "ex_steps")})
    print({k: want[k] for k in ("E_abs", "E_FC_ex", "E_FC_gs", "E_emi", "dQ", "gs_steps", "ex_steps")})
    assert out["converged"] == 1
    for k in ("E_gs_at_gs", "E_ex_at_gs", "E_ex_at_ex", "E_gs_at_ex", "E_abs", "E_FC_ex", "E_FC_gs",
              "E_emi"):
        assert abs(out[k] - want[k]) < 1e-8, k
    assert abs(out["dQ"] - want["dQ"]) < 1e-5
    assert np.abs(Rex - want["R_ex"]).max() < 1e-5
    assert np.abs(e.get_positions() - want["R_ex"]).max() < 1e-5
    g.close()
    e.close()


def test_relax_rejects_bad_parameters():
    rb, g, m, psi = _start(inputs.dimer(configuration="gs"))
    for bad in ({"fmax": 0.0}, {"max_step": -1.0}, {"h0": 0.0}, {"pair_rho": 0.0},
                {"pair_B": -1.0}, {"scf_restart": -1}):
        with pytest.raises(rb.RoksError) as ei:
            g.relax(**bad)
        assert ei.value.status == 1
    g.close()
