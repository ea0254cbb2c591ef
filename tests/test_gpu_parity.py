"""GPU (gfx950, FP64 tier) against the CPU oracle on the same seeded inputs.

Both sides start from the same counter-based random coefficients (keyed on
Miller indices) and orthonormalise them independently; results are compared
after matching plane waves by Miller index.  FP64 tolerance: 1e-10 per call, band by band (the largest
error of a band relative to that band's norm), the bar stated for the FP64
tier.
"""
import numpy as np
import pytest

from helpers import SphereMap, band_rel, ensure_built, orthorhombic_cell, rel, small_molecule
from oracle import roks as orc
from paper_2605_28637_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-10

CASES = {
    "tiny": lambda: inputs.tiny_cell(),
    "small_odd_bands": lambda: small_molecule(),
    "orthorhombic": lambda: orthorhombic_cell(),
    "ground_state": lambda: inputs.with_configuration(inputs.tiny_cell(), "gs"),
    "triplet": lambda: inputs.with_configuration(small_molecule(), "triplet"),
    "exchange_only": lambda: dict(inputs.tiny_cell(), xc="x"),
    # an odd grid (45^3 = 3^2 5): no Nyquist plane, the LDS-plane kernels
    "odd_grid": lambda: inputs.molecule_box(seed=2007, natoms=4, nb=9, N=45, L=14.0),
    # PBE (ROKS_XC_PBE): spectral gradients with the Nyquist planes of an even
    # grid, and on an odd grid without them
    "pbe": lambda: dict(inputs.tiny_cell(), xc="pbe"),
    "pbe_molecule": lambda: dict(small_molecule(), xc="pbe"),
    "pbe_odd_grid": lambda: dict(inputs.molecule_box(seed=2007, natoms=4, nb=9, N=45, L=14.0), xc="pbe"),
    # hybrids: a quarter (PBE0) and 0.36 (the dielectric-dependent fraction
    # the paper takes for MgO) of exact exchange
    "pbe0": lambda: dict(inputs.tiny_cell(), xc="pbe", exx=0.25),
    "ddh_molecule": lambda: dict(small_molecule(), xc="pbe", exx=0.36),
    # the overlap S = 1 + sum q |beta><beta|: one s channel, s + p channels,
    # and two coupled s channels (q_01 != 0) in the one-cell oxide
    "overlap": lambda: inputs.with_overlap(inputs.tiny_cell(), 0.5),
    "overlap_molecule": lambda: inputs.with_overlap(small_molecule(), 0.4),
    "overlap_oxide_cell": lambda: inputs.with_overlap(
        inputs.oxide_vacancy(reps=1, N=24, nb=16), 0.3),
    # the overlap with the other functionals: PBE, and a hybrid on PBE
    "overlap_pbe": lambda: dict(inputs.with_overlap(small_molecule(), 0.4), xc="pbe"),
    "overlap_pbe0": lambda: dict(inputs.with_overlap(inputs.tiny_cell(), 0.5), xc="pbe", exx=0.25),
}


class Pair:
    def __init__(self, system):
        rb = ensure_built()
        print("case", system.get("name"), system["grid"], system["nbands"], flush=True)
        self.s = system
        self.gpu = rb.Roks(system)
        self.m = orc.Model(system)
        self.map = SphereMap(self.gpu.miller(), self.m.miller)
        seed = system["seed"]
        self.gpu.set_coeffs(inputs.random_coefficients(self.gpu.miller(), system["cell"],
                                                       self.gpu.nb, seed), True)
        self.psi = orc.orthonormalize(inputs.random_coefficients(self.m.miller, self.m.cell,
                                                                 self.m.nb, seed), self.m)


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    p = Pair(CASES[request.param]())
    yield p
    p.gpu.close()


def test_sphere_matches_oracle(pair):
    gm = pair.gpu.miller()
    assert len(gm) * 2 - 1 == pair.m.npw
    assert tuple(gm[0]) == (0, 0, 0)
    full = set(map(tuple, gm)) | set(map(tuple, -gm))
    assert full == set(map(tuple, pair.m.miller))


def test_orthonormalised_start(pair):
    c = pair.map.to_full(pair.gpu.get_coeffs())
    assert band_rel(c, pair.psi) < 1e-12


def test_energies(pair):
    e, _, _ = pair.gpu.energy_gradient()
    pot = orc.potentials(pair.m, pair.psi)
    scale = max(1.0, max(abs(v) for t in pot.terms.values() for v in t))
    assert abs(e["E"] - pot.E) < TOL * scale
    for k in ("kinetic", "nonlocal", "external", "hartree", "xc"):
        np.testing.assert_allclose(e[k], pot.terms["nl" if k == "nonlocal" else
                                                   {"kinetic": "kin", "external": "ext"}.get(k, k)],
                                   rtol=0, atol=TOL * scale)
    np.testing.assert_allclose(e["E_L"], pot.E_L, rtol=0, atol=TOL * scale)


def test_apply_shell_mode(pair):
    Y = pair.map.to_full(pair.gpu.apply_h())
    pot = orc.potentials(pair.m, pair.psi)
    ref = orc.apply_shells(pair.m, pot, pair.psi)
    assert band_rel(Y, ref) < TOL


def test_apply_channels_on_arbitrary_vectors(pair):
    nconf = pair.m.nconf
    mask = (1 << (2 * nconf)) - 1
    v = inputs.random_coefficients(pair.gpu.miller(), pair.s["cell"], pair.gpu.nb, 77)
    H = pair.gpu.apply_h(v, mask)
    pot = orc.potentials(pair.m, pair.psi)
    vf = pair.map.to_full(v)
    k = 0
    for L in range(nconf):
        for s in range(2):
            ref = orc.apply_channel(pair.m, pot, L, s, vf)
            assert band_rel(pair.map.to_full(H[k]), ref) < TOL, (L, s)
            k += 1


def test_gradient_and_theta(pair):
    _, g, th = pair.gpu.energy_gradient()
    gr = orc.gradient(pair.m, pair.psi)
    assert band_rel(th, gr.theta) < TOL
    assert band_rel(pair.map.to_full(g), gr.gI) < TOL


def test_subspace_matrices(pair):
    R, kap, A = pair.gpu.subspace()
    gr = orc.gradient(pair.m, pair.psi)
    scale = max(1.0, np.abs(gr.R).max())
    # every block, the virtual one (<m|F^c|n>) included
    assert np.abs(R - gr.R).max() < TOL * scale
    assert np.abs(kap - gr.kappa).max() < TOL * max(1.0, np.abs(gr.kappa).max())
    assert np.abs(A - gr.A).max() < 1e-9


def test_three_cg_steps_and_forces(pair):
    st = orc.CGState(psi=pair.psi.copy())
    # one step from the shared start: the orbitals at the FP64 per-call bar
    gi = pair.gpu.pcg_step()
    oi = orc.pcg_step(pair.m, st)
    assert abs(gi["E1"] - oi.E1) < TOL * max(1.0, abs(oi.E0))
    assert band_rel(pair.map.to_full(pair.gpu.get_coeffs()), st.psi) < TOL
    for i in range(1, 3):
        gi = pair.gpu.pcg_step()
        oi = orc.pcg_step(pair.m, st)
        scale = max(1.0, abs(oi.E0))
        assert abs(gi["E0"] - oi.E0) < TOL * scale, i
        assert abs(gi["E1"] - oi.E1) < TOL * scale, i
        assert abs(gi["delta"] - oi.delta) < 1e-8 * max(1.0, oi.delta), i
        assert abs(gi["beta"] - oi.beta) < 1e-8 * max(1.0, abs(oi.beta)), i
        assert gi["E1"] < gi["E0"]
    assert band_rel(pair.map.to_full(pair.gpu.get_coeffs()), st.psi) < 1e-8
    F = pair.gpu.forces()
    Fo = orc.forces(pair.m, st.psi)
    assert np.abs(F - Fo).max() < 1e-8 * max(1.0, np.abs(Fo).max())


@pytest.mark.parametrize("nb", [90, 140])
def test_cg_steps_with_many_bands(nb):
    """Band counts past the single-workgroup rotation (nb > 78) and, at 140,
    past the LDS Cholesky (nb > 128): the multi-kernel exponential and the
    global-memory factorisation in the line search."""
    rb = ensure_built()
    s = small_molecule(nb=nb)
    print("many-band case", nb, flush=True)
    m = orc.Model(s)
    g = rb.Roks(s)
    g.set_coeffs(inputs.random_coefficients(g.miller(), s["cell"], g.nb, s["seed"]), True)
    st = orc.CGState(psi=orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"])),
                     dt=orc.DT_INIT)
    for i in range(2):
        gi = g.pcg_step()
        oi = orc.pcg_step(m, st)
        scale = max(1.0, abs(oi.E0))
        assert abs(gi["E0"] - oi.E0) < TOL * scale, i
        assert abs(gi["E1"] - oi.E1) < TOL * scale, i
        assert abs(gi["delta"] - oi.delta) < 1e-8 * max(1.0, oi.delta), i
    mp = SphereMap(g.miller(), m.miller)
    assert band_rel(mp.to_full(g.get_coeffs()), st.psi) < 1e-8
    g.close()


def test_periodic_restart_matches_oracle():
    """Reading R23 on both sides: 12 steps with a restart every 5."""
    rb = ensure_built()
    s = inputs.tiny_cell()
    print("restart case tiny", flush=True)
    m = orc.Model(s)
    g = rb.Roks(s)
    g.set_coeffs(inputs.random_coefficients(g.miller(), s["cell"], g.nb, s["seed"]), True)
    g.set_restart(5)
    st = orc.CGState(psi=orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"])),
                     dt=orc.DT_INIT, restart_period=5)
    flags = []
    for i in range(12):
        gi = g.pcg_step()
        oi = orc.pcg_step(m, st)
        flags.append(gi["restarted"])
        assert bool(gi["restarted"]) == bool(oi.restarted), i
        assert (gi["beta"] == 0.0) == (oi.beta == 0.0), i
        assert abs(gi["E1"] - oi.E1) < 1e-9 * max(1.0, abs(oi.E0)), i
    assert flags[5] == 1 and flags[10] == 1
    g.close()


def test_device_pointer_entry_points_match_host_ones():
    """roks_set_coeffs_d / roks_get_coeffs_d / roks_apply_h_d on torch device
    buffers give the host entry points' results bit for bit."""
    import torch
    rb = ensure_built()
    s = small_molecule()
    g = rb.Roks(s)
    c = inputs.random_coefficients(g.miller(), s["cell"], g.nb, s["seed"])
    g.set_coeffs(c, True)
    yh = g.apply_h()
    yc = g.apply_h(mask=0b1010)
    ch = g.get_coeffs()
    dev = torch.from_numpy(np.stack([ch.real, ch.imag], -1)).cuda().contiguous()
    out = torch.empty((g.nb, g.npw, 2), dtype=torch.float64, device="cuda")
    out2 = torch.empty((2, g.nb, g.npw, 2), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g2 = rb.Roks(s)
    g2.set_coeffs_d(dev.data_ptr(), False)
    g2.apply_h_d(None, 0, out.data_ptr())
    g2.apply_h_d(dev.data_ptr(), 0b1010, out2.data_ptr())
    back = torch.empty_like(dev)
    g2.get_coeffs_d(back.data_ptr())
    g2.synchronize()
    y = out.cpu().numpy()
    y2 = out2.cpu().numpy()
    np.testing.assert_array_equal(y[..., 0] + 1j * y[..., 1], yh)
    np.testing.assert_array_equal(y2[..., 0] + 1j * y2[..., 1], yc)
    np.testing.assert_array_equal(back.cpu().numpy(), dev.cpu().numpy())
    g.close()
    g2.close()


def test_state_errors():
    rb = ensure_built()
    r = rb.Roks(inputs.tiny_cell())
    with pytest.raises(rb.RoksError) as e:
        r.apply_h()
    assert e.value.status == 8
    c = inputs.random_coefficients(r.miller(), np.eye(3) * 8, r.nb, 5)
    c[1] = c[0]
    with pytest.raises(rb.RoksError) as e:
        r.set_coeffs(c, True)
    assert e.value.status == 5
    # a complex G = 0 coefficient is no real orbital
    c = inputs.random_coefficients(r.miller(), np.eye(3) * 8, r.nb, 5)
    c[2, 0] += 0.1j
    with pytest.raises(rb.RoksError) as e:
        r.set_coeffs(c, True)
    assert e.value.status == 1
    r.close()


@pytest.mark.parametrize("nb,dup", [(24, (3, 17)), (140, (3, 100))])
def test_dependent_bands_are_not_positive_definite(nb, dup):
    """A band equal to an earlier one: ROKS_ERR_NOT_PD from the one-workgroup
    Cholesky (<= 128 bands) and from the blocked one (band 100 repeats band 3
    of the first 64-column panel: its pivot is tested against its Gram
    diagonal, not against the updated block's)."""
    rb = ensure_built()
    s = small_molecule(nb=nb)
    r = rb.Roks(s)
    c = inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"])
    c[dup[1]] = c[dup[0]]
    with pytest.raises(rb.RoksError) as e:
        r.set_coeffs(c, True)
    assert e.value.status == 5
    c = inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"])
    r.set_coeffs(c, True)  # independent bands pass
    r.close()


def test_canonicalisation_rotates_every_shell_like_the_oracle():
    """ROKS_FLAG_CANONICALIZE: the Jacobi angles of the closed and virtual
    blocks (F^c in the virtual one) and three CG steps against the oracle."""
    rb = ensure_built()
    s = small_molecule()
    print("canonicalise case", flush=True)
    g = rb.Roks(s, flags=rb.FLAG_CANONICALIZE)
    m = orc.Model(s)
    fl = orc.Flags(canonicalize=True)
    g.set_coeffs(inputs.random_coefficients(g.miller(), s["cell"], g.nb, s["seed"]), True)
    psi = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"]))
    R, kap, A = g.subspace()
    gr = orc.gradient(m, psi, fl)
    assert np.abs(R - gr.R).max() < TOL * max(1.0, np.abs(gr.R).max())
    assert np.abs(kap - gr.kappa).max() < TOL * max(1.0, np.abs(gr.kappa).max())
    assert np.abs(A - gr.A).max() < 1e-9
    virt = [n for n in range(m.nb) if m.shell_virtual[m.band_shell[n]]]
    assert len(virt) == 2 and abs(A[virt[0], virt[1]]) > 0
    st = orc.CGState(psi=psi)
    for i in range(3):
        gi = g.pcg_step()
        oi = orc.pcg_step(m, st, fl)
        assert abs(gi["E1"] - oi.E1) < TOL * max(1.0, abs(oi.E0)), i
    mp = SphereMap(g.miller(), m.miller)
    assert band_rel(mp.to_full(g.get_coeffs()), st.psi) < 1e-8
    g.close()


def test_converged_singlet_tiny():
    """PCG to 1e-10 Ha on both sides from the same start: same E_S and forces."""
    s = inputs.tiny_cell()
    p = Pair(s)
    info, it = p.gpu.solve(tol=1e-10, maxiter=400)
    st, hist = orc.solve(p.m, p.psi, tol=1e-10, maxiter=400, orthonormalize_start=False)
    assert abs(info["E1"] - hist[-1].E1) < 1e-9
    F = p.gpu.forces()
    Fo = orc.forces(p.m, st.psi)
    assert np.abs(F - Fo).max() < 1e-5
    p.gpu.close()


def test_molecule_box_full_size():
    """The 24 bohr / 64^3 / 20-atom / 40-band molecule-in-box at full size:
    energies, every band's F^n|n>, theta, g_I, the subspace matrices, one CG
    step from the shared start and the forces after it."""
    s = inputs.molecule_box()
    p = Pair(s)
    e, g, th = p.gpu.energy_gradient()
    gr = orc.gradient(p.m, p.psi)
    scale = max(1.0, max(abs(v) for t in gr.pot.terms.values() for v in t))
    assert abs(e["E"] - gr.pot.E) < TOL * scale
    Y = p.map.to_full(p.gpu.apply_h())
    assert band_rel(Y, gr.Y) < TOL
    assert band_rel(th, gr.theta) < TOL
    assert band_rel(p.map.to_full(g), gr.gI) < TOL
    R, kap, A = p.gpu.subspace()
    assert np.abs(R - gr.R).max() < TOL * max(1.0, np.abs(gr.R).max())
    assert np.abs(kap - gr.kappa).max() < TOL * max(1.0, np.abs(gr.kappa).max())
    assert np.abs(A - gr.A).max() < 1e-9
    st = orc.CGState(psi=p.psi.copy())
    gi = p.gpu.pcg_step()
    oi = orc.pcg_step(p.m, st)
    assert abs(gi["E1"] - oi.E1) < TOL * max(1.0, abs(oi.E0))
    assert abs(gi["delta"] - oi.delta) < 1e-8 * max(1.0, oi.delta)
    assert band_rel(p.map.to_full(p.gpu.get_coeffs()), st.psi) < TOL
    F = p.gpu.forces()
    Fo = orc.forces(p.m, st.psi)
    assert np.abs(F - Fo).max() < 1e-9 * max(1.0, np.abs(Fo).max())
    p.gpu.close()


def test_largest_batch_member():
    """The largest member of the uneven batch (58 atoms x 4 projectors, 116
    bands, 80^3): energies, sampled F^n|n> and one CG step against the
    oracle (the expansions past 128 inner rows on the tiled product)."""
    rb = ensure_built()
    s = max(inputs.batch_systems(), key=lambda x: x["nbands"])
    print("batch member", s["name"], s["grid"], s["nbands"], flush=True)
    assert s["nbands"] >= 100
    p = Pair(s)
    assert p.gpu.nproj == 4 * len(s["pos"]) >= 200
    e, g, th = p.gpu.energy_gradient()
    pot = orc.potentials(p.m, p.psi)
    assert abs(e["E"] - pot.E) < TOL * max(1.0, max(abs(v) for t in pot.terms.values() for v in t))
    Y = p.map.to_full(p.gpu.apply_h())
    for n in (0, s["nbands"] // 2, s["nbands"] - 4, s["nbands"] - 3):
        X = p.m.band_shell[n]
        ref = orc.apply_shell_operator(p.m, pot, X, p.psi[n:n + 1])[0]
        assert band_rel(Y[n], ref) < TOL, n
    st = orc.CGState(psi=p.psi.copy())
    gi = p.gpu.pcg_step()
    oi = orc.pcg_step(p.m, st)
    assert abs(gi["E1"] - oi.E1) < TOL * max(1.0, abs(oi.E0))
    assert band_rel(p.map.to_full(p.gpu.get_coeffs()), st.psi) < TOL
    p.gpu.close()
