"""Pins of the learned-preconditioner oracle (oracle/mlp.py)."""
import math

import numpy as np
import scipy.linalg

from oracle import mlp, roks
from paper_2605_28637_amd import inputs


def test_param_count():
    assert mlp.NPARAM == 4481


def test_gelu_closed_forms_and_derivative():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(mlp.gelu(np.array([8.0])), [8.0], rtol=1e-12)
    np.testing.assert_allclose(mlp.gelu(np.array([-8.0])), [0.0], atol=1e-12)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_prime(z), fd, atol=1e-8)


def test_p18_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    th = rng.normal(0, 0.3, mlp.NPARAM)
    X = rng.normal(size=(7, 3))
    do = rng.normal(size=7)
    g = mlp.backward(th, mlp.forward(th, X)[1], do)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (do @ mlp.forward(tp, X)[0] - do @ mlp.forward(tm, X)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g[i])), i


def test_loss_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    th = rng.normal(0, 0.3, mlp.NPARAM)
    nb, nsh = 3, 5
    X = rng.normal(size=(nb, nsh, 3))
    a, b, c = rng.normal(size=(nb, nsh)), rng.uniform(0.1, 1, (nb, nsh)), rng.uniform(0.1, 1, (nb, nsh))
    L, g = mlp.loss_and_grad(th, X, a, b, c)
    h = 1e-6
    for i in rng.choice(mlp.NPARAM, 40, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, a, b, c)[0] - mlp.loss_and_grad(tm, X, a, b, c)[0]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g[i]))


def test_band_loss_limits():
    # a parallel to delta -> 0; orthogonal -> 1 (per band, shell moments)
    beta = np.array([[1.0, 4.0]])
    gamma = np.array([[1.0, 4.0]])
    alpha = np.array([[1.0, 4.0]])  # Kg = delta
    L, _ = mlp.band_loss(np.ones((1, 2)), alpha, beta, gamma)
    assert abs(L) < 1e-15
    L, _ = mlp.band_loss(np.ones((1, 2)), np.zeros((1, 2)), beta, gamma)
    assert abs(L - 1.0) < 1e-15


def test_alignment_recovers_rotated_subspace_exactly():
    m = roks.Model(inputs.molecule_box(natoms=2, nb=8, N=16, L=8.0))
    psi = roks.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, 3))
    rng = np.random.default_rng(2)
    rot = np.zeros((m.nb, m.nb))
    for X in range(m.nshell):
        sel = np.where(m.band_shell == X)[0]
        Q, _ = np.linalg.qr(rng.normal(size=(len(sel), len(sel))))
        rot[np.ix_(sel, sel)] = Q
    psi_inf = rot.T @ psi  # a rotation within every shell: nothing to correct
    d = mlp.aligned_correction(m, psi, psi_inf)
    assert np.abs(d).max() < 1e-12
    # plus an out-of-span component: recovered as the correction of band 0
    extra = inputs.random_coefficients(m.miller, m.cell, 1, 9)[0]
    extra = extra - roks.overlap(psi, extra[None])[:, 0] @ psi
    extra *= 1e-3 / math.sqrt(roks.dot(extra, extra))
    psi2 = psi_inf.copy()
    psi2[0] = psi2[0] + extra
    d2 = mlp.aligned_correction(m, psi, psi2)
    # extra is orthogonal to the span, so O = <inf|psi> is still rot^T, the
    # alignment undoes the rotation exactly and delta_n = rot[n, 0] * extra
    assert np.abs(d2 - np.outer(rot[:, 0], extra)).max() < 1e-12


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 1e-2)
    np.testing.assert_allclose(th, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.140625], dtype=np.float32)
    r = mlp.bf16_round(vals)
    np.testing.assert_array_equal(r, [1.0, 1.0, 1.0 + 2 ** -7, -2.5, 3.140625])


def test_untrained_network_is_near_plain_teter():
    th = mlp.init_params(5)
    X = np.random.default_rng(3).normal(size=(100, 3))
    s = mlp.scale_of(mlp.forward(th, X)[0])
    assert np.abs(s - 1).max() < 0.1


def test_normalized_scale_keeps_the_plain_first_order_decrease():
    m = roks.Model(inputs.molecule_box(natoms=2, nb=8, N=16, L=8.0))
    psi = roks.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, 4))
    gr = roks.gradient(m, psi)
    g2sh, shell_of = mlp.g_shells(0.5 * m.g2)
    rng = np.random.default_rng(5)
    s_shell = np.exp(rng.uniform(-2, 2, size=(m.nb, len(g2sh))))
    s_shell[0] = np.nan  # a band without features keeps s = 1
    sc = mlp.normalized_scale(m, gr.gI, s_shell, shell_of)
    p1 = roks.precondition(m, psi, gr.gI, scale=sc)
    p0 = roks.precondition(m, psi, gr.gI)
    d1 = sum(roks.dot(p1[n], gr.gI[n]) for n in range(1, m.nb))
    d0 = sum(roks.dot(p0[n], gr.gI[n]) for n in range(1, m.nb))
    assert abs(d1 - d0) <= 1e-12 * abs(d0)
    assert abs(roks.dot(p1[0], gr.gI[0]) - roks.dot(p0[0], gr.gI[0])) <= 1e-12 * abs(d0)
    np.testing.assert_allclose(sc[0], 1.0)
    occupied = [n for n in range(1, m.nb) if roks.dot(gr.gI[n], gr.gI[n]) > 0]
    assert len(occupied) >= 3
    # per band the first-order change is redistributed, not kept
    per = [roks.dot(p1[n], gr.gI[n]) / roks.dot(p0[n], gr.gI[n]) for n in occupied]
    assert max(per) / min(per) > 1.1
    # a factor constant over all bands and shells is removed entirely
    sc2 = mlp.normalized_scale(m, gr.gI, np.full((m.nb, len(g2sh)), 3.7), shell_of)
    np.testing.assert_allclose(sc2, 1.0, rtol=1e-13)


def test_moments_are_energy_norm_products_split_by_shell():
    m = roks.Model(inputs.molecule_box(natoms=2, nb=6, N=16, L=8.0))
    x = inputs.random_coefficients(m.miller, m.cell, m.nb, 21)
    y = inputs.random_coefficients(m.miller, m.cell, m.nb, 22)
    ekin = np.linspace(0.5, 2.0, m.nb)
    g2sh, shell_of = mlp.g_shells(0.5 * m.g2)
    a, b, c = mlp.moments(m, x, y, shell_of, len(g2sh), ekin)
    # summed over shells: <x|T|y> + ekin <x|y> from the model's own kinetic operator
    xTy = np.real(np.sum(np.conj(x) * (0.5 * m.g2) * y, axis=1))
    np.testing.assert_allclose(a.sum(1), xTy + ekin * np.array([roks.dot(x[n], y[n]) for n in range(m.nb)]),
                               rtol=1e-12)
    np.testing.assert_allclose(b.sum(1), roks.band_kinetic(m, x) + ekin * np.sum(np.abs(x) ** 2, 1), rtol=1e-12)
    np.testing.assert_allclose(c.sum(1), roks.band_kinetic(m, y) + ekin * np.sum(np.abs(y) ** 2, 1), rtol=1e-12)
    # each shell holds only its own |G|^2: moving one G's weight to another
    # shell changes exactly those two entries
    k = shell_of[5]
    assert np.all(np.isclose(g2sh[shell_of], 0.5 * m.g2, rtol=0, atol=1e-9))
    assert b[0, k] > 0
