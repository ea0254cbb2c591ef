"""Learned rescaling of the Teter preconditioner on the GPU against the FP64
oracle (oracle/mlp.py), which evaluates the network with the same BF16
rounding of the weights.

Tolerances follow from the arithmetic:
* forward: a running error bound of the FP32 evaluation (gamma_n = n u/(1 - n u),
  u = 2^-24, per dot product; activation values carry 8 u (|z| + 1) for erf
  and the product), propagated through |GELU'| <= 1.13;
* training pairs: features are FP64 values rounded to FP32 (2 u relative);
  moments (energy-norm products per (band, |G|^2 shell)) are FP64 sums over iterates that agree to 1e-12, with the polar
  factor by Newton-Schulz on the GPU and by SVD in the oracle: 1e-9 relative;
* loss: s in FP32 (a few u relative) enters A^2/(BC) to second order: 1e-5;
* gradient: per parameter, a sum over samples of FP32 products, chunks of
  1 024 in sequence: gamma_1024 (6.1e-5) plus the per-sample error, against
  the sum of the terms' magnitudes: 2e-4 of that sum.
"""
import math

import numpy as np
import pytest

from helpers import SphereMap, ensure_built, rel, small_molecule
from oracle import mlp as om
from oracle import roks as orc
from paper_2605_28637_amd import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _gamma(n):
    return n * U / (1 - n * U)


def _forward_bound(theta, X):
    """Worst-case |o_fp32 - o_exact| of the FP32 forward pass."""
    p = om.unpack(theta)
    o, (X_, z1, h1, z2, h2) = om.forward(theta, X)
    aW1, aW2, aw3 = np.abs(p["W1"]), np.abs(p["W2"]), np.abs(p["w3"])
    e_z1 = _gamma(3) * (np.abs(p["b1"]) + np.abs(X) @ aW1.T)
    e_h1 = 1.13 * e_z1 + 8 * U * (np.abs(z1) + 1)
    e_z2 = _gamma(64) * (np.abs(p["b2"]) + np.abs(h1) @ aW2.T) + e_h1 @ aW2.T
    e_h2 = 1.13 * e_z2 + 8 * U * (np.abs(z2) + 1)
    return _gamma(64) * (abs(p["b3"][0]) + np.abs(h2) @ aw3) + e_h2 @ aw3


def _theta(seed, out_scale):
    """Oracle-initialised parameters with the output layer scaled so that
    s = exp(2 tanh(o)) spans a visible range."""
    th = om.init_params(seed)
    u = om.unpack(th)
    u["w3"][:] *= out_scale
    u["b3"][:] = 0.1
    return th.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("S", [1, 255, 1000, 4099])
def test_forward_matches_oracle(S):
    rb = ensure_built()
    print("mlp forward S", S, flush=True)
    th = _theta(7, 300.0)
    X = np.random.default_rng(S).normal(0, 2, size=(S, 3)).astype(np.float32).astype(np.float64)
    net = rb.Mlp(th)
    o = net.forward(X).astype(np.float64)
    thb = om.bf16_round(th)
    ref, _ = om.forward(thb, X)
    bound = _forward_bound(thb, X)
    assert np.all(np.abs(o - ref) <= 2 * bound + 1e-30), np.max(np.abs(o - ref) / bound)
    # parameters come back unrounded (FP32 master copy)
    np.testing.assert_array_equal(net.get_params(), th.astype(np.float32))
    net.close()


def test_seeded_initialisation_is_near_plain_teter():
    rb = ensure_built()
    net = rb.Mlp(seed=11)
    th = net.get_params().astype(np.float64)
    assert np.all(np.isfinite(th)) and th[-1] == 0.0
    p = om.unpack(th)
    assert np.abs(p["W1"]).max() <= 1 / math.sqrt(3) and np.abs(p["W2"]).max() <= 1 / 8
    assert np.abs(p["w3"]).max() <= 1e-2 / 8
    o = net.forward(np.random.default_rng(0).normal(size=(500, 3)))
    assert np.abs(om.scale_of(o.astype(np.float64)) - 1).max() < 0.1
    net.close()


# ---------------------------------------------------------------------------
# training pairs from recorded iterates
# ---------------------------------------------------------------------------
def _oracle_pairs(m, psi_list, psi_inf):
    """Oracle features [nseg][len][3] and moments [nseg][3][len] of the
    occupied bands with a gradient, one segment per recorded iterate, in the
    library's order (band-major, shells in ascending |G|^2); shorter segments
    are padded with zero moments, which add nothing to a segment's sums."""
    g2sh, shell_of = om.g_shells(0.5 * m.g2)
    segs = []
    for psi in psi_list:
        gr = orc.gradient(m, psi)
        F = om.band_features(m, psi, gr.gI, g2sh)
        Kg = om.plain_teter_Kg(m, gr.gI)
        d = om.aligned_correction(m, psi, psi_inf)
        a, b, c = om.moments(m, Kg, d, shell_of, len(g2sh), orc.band_kinetic(m, psi))
        sel = [n for n in range(m.nb)
               if not m.shell_virtual[m.band_shell[n]] and not np.isnan(F[n, 0, 0])]
        segs.append((F[sel].reshape(-1, 3), np.stack([a[sel].ravel(), b[sel].ravel(), c[sel].ravel()])))
    L = max(len(x) for x, _ in segs)
    X = np.zeros((len(segs), L, 3))
    M = np.zeros((len(segs), 3, L))
    lens = []
    for j, (x, mo) in enumerate(segs):
        X[j, :len(x)] = x
        M[j, :, :len(x)] = mo
        lens.append(len(x))
    return X, M, lens


@pytest.fixture(scope="module")
def pairs():
    """Two recorded iterates of a small molecule (11 bands, ragged band pair)
    and an unrelated orthonormal set as psi_inf, on both sides."""
    rb = ensure_built()
    s = small_molecule()
    print("mlp pairs", s["grid"], s["nbands"], flush=True)
    m = orc.Model(s)
    g = rb.Roks(s)
    mp = SphereMap(g.miller(), m.miller)
    c0 = inputs.random_coefficients(g.miller(), s["cell"], g.nb, s["seed"])
    c1 = inputs.random_coefficients(g.miller(), s["cell"], g.nb, s["seed"] + 77)
    g.set_coeffs(c0, True)
    g.record(4, 1)
    g.pcg_step()
    g.pcg_step()
    g.set_coeffs(c0 + 0.3 * c1, True)
    net = rb.Mlp(_theta(3, 300.0))
    used, skipped = net.collect(g)
    assert (used, skipped) == (2, 0)
    # the oracle's own iterates from the same start
    psi0 = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"]))
    st = orc.CGState(psi=psi0.copy())
    orc.pcg_step(m, st)
    psi1 = st.psi.copy()
    full0 = inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"])
    full1 = inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"] + 77)
    psi_inf = orc.orthonormalize(full0 + 0.3 * full1)
    Xo, Mo, lens = _oracle_pairs(m, [psi0, psi1], psi_inf)
    yield rb, g, net, m, Xo, Mo, lens
    g.close()
    net.close()


def test_collected_pairs_match_oracle(pairs):
    rb, g, net, m, Xo, Mo, lens = pairs
    S, nseg = net.num_samples()
    assert nseg == 2 and S == sum(lens)
    x, mom, off = net.get_samples()
    np.testing.assert_array_equal(off, np.r_[0, np.cumsum(lens)])
    for j in range(nseg):
        xg = x[off[j]:off[j + 1]].astype(np.float64)
        xo = Xo[j, :lens[j]]
        assert np.all(np.abs(xg - xo) <= 4 * U * np.abs(xo) + 1e-7), j
        mg = mom[:, off[j]:off[j + 1]]
        mo = Mo[j, :, :lens[j]]
        B, C = mo[1].sum(), mo[2].sum()
        assert np.abs(mg[0] - mo[0]).max() <= 1e-9 * math.sqrt(B * C), j
        assert np.abs(mg[1] - mo[1]).max() <= 1e-9 * B, j
        assert np.abs(mg[2] - mo[2]).max() <= 1e-9 * C, j


def _abs_grad_magnitude(theta, X, do):
    """Per parameter, the sum over samples of |term| of the gradient sum."""
    p = om.unpack(theta)
    _, (X_, z1, h1, z2, h2) = om.forward(theta, X)
    ado = np.abs(do)
    adz2 = np.outer(ado, np.abs(p["w3"])) * np.abs(om.gelu_prime(z2))
    adz1 = (adz2 @ np.abs(p["W2"])) * np.abs(om.gelu_prime(z1))
    parts = {"W1": adz1.T @ np.abs(X), "b1": adz1.sum(0), "W2": adz2.T @ np.abs(h1),
             "b2": adz2.sum(0), "w3": np.abs(h2).T @ ado, "b3": np.array([ado.sum()])}
    return np.concatenate([parts[k].ravel() for k in ("W1", "b1", "W2", "b2", "w3", "b3")])


def test_loss_and_gradient_match_oracle(pairs):
    rb, g, net, m, Xo, Mo, lens = pairs
    th = net.get_params().astype(np.float64)
    L, grad = net.loss_grad()
    thb = om.bf16_round(th)
    Lo, go = om.loss_and_grad(thb, Xo, Mo[:, 0], Mo[:, 1], Mo[:, 2])
    print("loss gpu %.9f oracle %.9f" % (L, Lo))
    assert abs(L - Lo) < 1e-5
    # the per-sample dL/do of the oracle, for the magnitude of every sum
    nb, nsh, _ = Xo.shape
    o, _ = om.forward(thb, Xo.reshape(-1, 3))
    t = np.tanh(o)
    s = np.exp(2 * t).reshape(nb, nsh)
    _, dlds = om.band_loss(s, Mo[:, 0], Mo[:, 1], Mo[:, 2])
    do = dlds.ravel() * s.ravel() * 2 * (1 - t * t)
    mag = _abs_grad_magnitude(thb, Xo.reshape(-1, 3), do)
    err = np.abs(grad.astype(np.float64) - go)
    assert np.all(err <= 2e-4 * mag + 1e-12 * np.abs(go).max()), np.max(err / (mag + 1e-300))


def test_adam_step_matches_oracle(pairs):
    rb, g, net, m, Xo, Mo, lens = pairs
    th = _theta(5, 300.0)
    net.set_params(th)
    lr = 1e-3
    hist = net.train(1, lr)
    th1 = net.get_params().astype(np.float64)
    Lo, go = om.loss_and_grad(om.bf16_round(th), Xo, Mo[:, 0], Mo[:, 1], Mo[:, 2])
    assert abs(hist[0] - Lo) < 1e-5
    tho, _, _ = om.adam_step(th, np.zeros_like(th), np.zeros_like(th), go, 1, lr)
    # the first Adam step is lr g/(|g| + eps): insensitive to the gradient's
    # rounding except where |g| is at its noise level
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    assert big.sum() > 100
    np.testing.assert_allclose(th1[big], tho[big], rtol=0, atol=1e-3 * lr + 4 * U * np.abs(th).max())
    assert np.all(np.abs(th1 - th) <= lr * 1.0001 + 4 * U * np.abs(th).max())


def test_training_lowers_the_loss(pairs):
    rb, g, net, m, Xo, Mo, lens = pairs
    net.set_params(_theta(5, 300.0))
    hist = net.train(200, 3e-3)
    L_end, _ = net.loss_grad()
    print("loss %.6f -> %.6f" % (hist[0], L_end))
    assert L_end < hist[0] - 1e-3
    assert np.all(np.isfinite(hist))
    # training is deterministic: the same run gives the same parameters
    th_a = net.get_params()
    net.set_params(_theta(5, 300.0))
    net.train(200, 3e-3)
    np.testing.assert_array_equal(net.get_params(), th_a)


# ---------------------------------------------------------------------------
# inference inside the CG step
# ---------------------------------------------------------------------------
def test_learned_pcg_steps_match_oracle():
    rb = ensure_built()
    s = small_molecule()
    print("learned pcg", s["grid"], s["nbands"], flush=True)
    m = orc.Model(s)
    g = rb.Roks(s)
    mp = SphereMap(g.miller(), m.miller)
    g.set_coeffs(inputs.random_coefficients(g.miller(), s["cell"], g.nb, s["seed"]), True)
    th = _theta(9, 300.0)
    om.unpack(th)["W1"][:, 0] *= 4.0  # a strong dependence on |G|^2
    th = th.astype(np.float32).astype(np.float64)
    net = rb.Mlp(th)
    g.set_mlp(net)
    thb = om.bf16_round(th)
    g2sh, shell_of = om.g_shells(0.5 * m.g2)
    st = orc.CGState(psi=orc.orthonormalize(
        inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"])))
    spread = []
    for i in range(3):
        gr = orc.gradient(m, st.psi)
        F = om.band_features(m, st.psi, gr.gI, g2sh)
        s_shell = np.full(F.shape[:2], np.nan)
        for n in range(m.nb):
            if not np.isnan(F[n, 0, 0]):
                s_shell[n] = om.scale_of(om.forward(thb, F[n])[0])
        sc = om.normalized_scale(m, gr.gI, s_shell, shell_of)
        spread.append(max(sc[n].max() / sc[n].min() for n in range(m.nb)))
        oi = orc.pcg_step(m, st, scale=sc)
        gi = g.pcg_step()
        assert gi["learned"] == 1 and gi["fallback"] == 0
        dE = abs(oi.E0 - oi.E1)
        print("step", i, "E1 gpu %.12f oracle %.12f, s spread %.3f" % (gi["E1"], oi.E1, spread[-1]))
        assert abs(gi["E0"] - oi.E0) < 1e-5 * dE + 1e-10 * abs(oi.E0), i
        assert abs(gi["E1"] - oi.E1) < 1e-5 * dE + 1e-10 * abs(oi.E0), i
    assert min(spread) > 1.2  # within a band the rescaling is not a no-op
    assert rel(mp.to_full(g.get_coeffs()), st.psi) < 1e-5
    g.set_mlp(None)
    assert g.pcg_step()["learned"] == 0
    g.close()
    net.close()
