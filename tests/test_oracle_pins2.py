"""More pins of the CPU oracle, each against something other than the
oracle's own formula:

* the local well on the grid against the real-space Gaussian summed over
  periodic images (the amplitude and width of v(r) = -A exp(-r^2/(2 sigma^2)));
* the pair curvature kappa (reading R3) and R (Eq. r_matrix_singlet) of every
  pair class against finite differences of the frozen-potential energy
  along the rotation exp(t E_mn), with the shell operators applied by the
  oracle's FFT path;
* the Teter reference energy (reading R1) of a single plane wave in closed
  form, and the preconditioned vector it gives (Eq. prec_k);
* P9: SciPy's L-BFGS, minimising E_S over Cholesky-orthonormalised
  coefficients (a different optimiser, none of the paper's CG, rotation or
  preconditioner), reaches the CG minimum of the tiny cell.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.optimize

from oracle import roks
from paper_2605_28637_amd import inputs


# ---------------------------------------------------------------------------
# the local well: amplitude and width in real space
# ---------------------------------------------------------------------------
def test_vext_is_periodic_sum_of_gaussian_wells():
    s = dict(inputs.tiny_cell())
    L = 10.0
    A, sigma = 1.7, 0.7
    s["cell"] = np.eye(3) * L
    s["grid"] = (48, 48, 48)
    s["ecut"] = 2.0  # the sphere does not matter for V_ext (full grid)
    s["species"] = [{"A": A, "sigma": sigma, "proj": [], "D": np.zeros((0, 0))}]
    s["species_of_atom"] = np.array([0])
    R = np.array([3.1, 4.6, 5.35])
    s["pos"] = R[None, :]
    m = roks.Model(s)
    frac = np.stack(np.meshgrid(*[np.arange(n) / n for n in m.grid], indexing="ij"), -1)
    r = frac @ m.cell
    v = np.zeros(m.grid)
    for img in itertools.product((-1, 0, 1), repeat=3):
        d = r - (R + np.array(img) @ m.cell)
        v += -A * np.exp(-(d * d).sum(-1) / (2 * sigma * sigma))
    assert np.abs(m.vext_r - v).max() < 1e-8 * A
    # two atoms of different species superpose
    s2 = dict(s)
    s2["species"] = [s["species"][0], {"A": 0.9, "sigma": 1.1, "proj": [], "D": np.zeros((0, 0))}]
    s2["species_of_atom"] = np.array([0, 1])
    R2 = np.array([7.0, 2.2, 8.1])
    s2["pos"] = np.stack([R, R2])
    m2 = roks.Model(s2)
    v2 = v.copy()
    for img in itertools.product((-1, 0, 1), repeat=3):
        d = r - (R2 + np.array(img) @ m.cell)
        v2 += -0.9 * np.exp(-(d * d).sum(-1) / (2 * 1.1 * 1.1))
    assert np.abs(m2.vext_r - v2).max() < 1e-8


# ---------------------------------------------------------------------------
# kappa (R3) and R (Eq. r_matrix_singlet) by finite differences
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_roks():
    # 7 closed + 2 open + 2 virtual bands: every pair class
    s = inputs.molecule_box(seed=2001, natoms=6, nb=11, N=24, L=12.0)
    m = roks.Model(s)
    psi = roks.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, 2001))
    return m, psi


def _frozen_energy(m, pot, psi):
    """sum_k <psi_k|F^{X(k)}|psi_k> with the operators of fixed potentials."""
    E = 0.0
    for X in range(m.nshell):
        if m.shell_virtual[X]:
            continue
        sel = np.where(m.band_shell == X)[0]
        FX = roks.apply_shell_operator(m, pot, X, psi[sel])
        E += float(np.sum(np.real(np.conj(psi[sel]) * FX)))
    return E


@pytest.mark.parametrize("pair", [(2, 7), (1, 8), (4, 9), (7, 8), (7, 10), (8, 9), (8, 10)])
def test_kappa_and_R_are_frozen_pair_derivatives(small_roks, pair):
    """With psi'_m = cos t psi_m - sin t psi_n, psi'_n = sin t psi_m + cos t psi_n
    (U = exp(t E_mn), psi' = U^T psi), the frozen-potential energy has
    dE/dt = -2 R_mn and d^2E/dt^2 = 2 kappa_mn at t = 0 for pairs of
    different shells (closed-open, closed-virtual, open-open, open-virtual)."""
    m, psi = small_roks
    gr = roks.gradient(m, psi)
    a, b = pair
    assert m.band_shell[a] != m.band_shell[b]
    pot = gr.pot

    def rotated(t):
        E = np.zeros((m.nb, m.nb))
        E[a, b], E[b, a] = 1.0, -1.0
        U = scipy.linalg.expm(t * E)
        return U.T @ psi

    h = 1e-3
    Ep, E0, Em = (_frozen_energy(m, pot, rotated(t)) for t in (h, 0.0, -h))
    d1 = (Ep - Em) / (2 * h)
    d2 = (Ep - 2 * E0 + Em) / (h * h)
    scale = max(1.0, abs(gr.kappa[a, b]))
    assert abs(d1 + 2 * gr.R[a, b]) < 1e-6 * scale, (d1, gr.R[a, b])
    assert abs(d2 - 2 * gr.kappa[a, b]) < 1e-5 * scale, (d2, gr.kappa[a, b])
    # the generator is a descent direction of the frozen model and its angle
    # the frozen model's minimiser for kappa > 0 (reading R2)
    if gr.kappa[a, b] > 0:
        ts = np.linspace(-0.8, 0.8, 3201)
        Es = [E0 - 2 * gr.R[a, b] * 0.5 * math.sin(2 * t)
              + gr.kappa[a, b] * 0.5 * (1 - math.cos(2 * t)) for t in ts]
        # the exact frozen energy is a trigonometric polynomial of degree 2 in t;
        # check the model at the predicted angle against the oracle's rotation
        t = gr.A[a, b]
        Ef = _frozen_energy(m, pot, rotated(t))
        assert Ef <= E0 + 1e-12
        assert abs(ts[int(np.argmin(Es))] - t) < 1e-3


import scipy.linalg  # noqa: E402  (used above through the module name)


# ---------------------------------------------------------------------------
# Teter reference energy of one plane wave (reading R1, Eq. prec_k)
# ---------------------------------------------------------------------------
def test_teter_reference_energy_of_one_plane_wave():
    m = roks.Model(inputs.tiny_cell())
    # one plane-wave pair +-G (the largest |G| of the sphere)
    j = int(np.argmax(m.g2))
    g = np.zeros(m.npw, complex)
    g[j] = 0.3 + 0.4j
    g[m.minus[j]] = np.conj(g[j])
    Er = roks.teter_reference_energy(m, g)
    assert abs(Er - 1.5 * 0.5 * m.g2[j]) < 1e-14 * Er
    # the preconditioned vector: x = 2/3, K = -(2/E_ref) P(x)/(P(x) + 16 x^4),
    # P(x) = 27 + 18 x + 12 x^2 + 8 x^3 (coefficients printed in Eq. prec_k);
    # psi a different plane wave, so the projection removes nothing
    x = 2.0 / 3.0
    P = 27 + 18 * x + 12 * x * x + 8 * x ** 3
    K = -(2.0 / Er) * P / (P + 16 * x ** 4)
    k = int(np.where((m.miller == [1, 0, 0]).all(axis=1))[0][0])
    assert k not in (j, m.minus[j])
    psi = np.zeros((1, m.npw), complex)
    psi[0, k] = psi[0, m.minus[k]] = 1 / math.sqrt(2)
    mm = roks.Model(inputs.with_configuration(inputs.tiny_cell(n_closed=0), "triplet"))
    assert mm.nb == 2
    gI = np.stack([g, g])
    ps = np.stack([psi[0], np.zeros(m.npw, complex)])
    z = int(np.where((m.miller == 0).all(axis=1))[0][0])
    ps[1, z] = 1.0  # G = 0: orthogonal to both plane waves
    p = roks.precondition(mm, ps, gI)
    np.testing.assert_allclose(p[0], K * g, rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# P9: an independent optimiser reaches the CG minimum
# ---------------------------------------------------------------------------
class _RealEmbedding:
    """Real coordinates y of conjugate-symmetric full-sphere vectors with
    <a|b> = y_a . y_b (G = 0 real part, sqrt 2 (Re, Im) of one of each +-G)."""

    def __init__(self, m):
        self.m = m
        self.zero = int(np.where((m.miller == 0).all(axis=1))[0][0])
        half = [i for i in range(m.npw) if i != self.zero and i < m.minus[i]]
        self.half = np.array(half)
        self.dim = 1 + 2 * len(half)

    def to_full(self, y):
        y = y.reshape(-1, self.dim)
        c = np.zeros((len(y), self.m.npw), complex)
        c[:, self.zero] = y[:, 0]
        z = (y[:, 1::2] + 1j * y[:, 2::2]) / math.sqrt(2)
        c[:, self.half] = z
        c[:, self.m.minus[self.half]] = np.conj(z)
        return c

    def to_real(self, c):
        y = np.zeros((len(c), self.dim))
        y[:, 0] = c[:, self.zero].real
        y[:, 1::2] = math.sqrt(2) * c[:, self.half].real
        y[:, 2::2] = math.sqrt(2) * c[:, self.half].imag
        return y


def _energy_and_grad(m, emb, x):
    """E_S(Psi(X)) with Psi = L^-1 X, X X^T = L L^T (Cholesky in band order),
    and its gradient by the chain rule: dE = 2 sum_n <F^n psi_n|d psi_n>
    (P7 pins it by finite differences), through the orthonormalisation."""
    X = x.reshape(m.nb, emb.dim)
    G = X @ X.T
    Lc = np.linalg.cholesky(G)
    Li = scipy.linalg.solve_triangular(Lc, np.eye(m.nb), lower=True)
    Y = Li @ X
    psi = emb.to_full(Y)
    pot = roks.potentials(m, psi)
    Fpsi = roks.apply_shells(m, pot, psi)
    Ybar = 2.0 * emb.to_real(Fpsi)
    # Psi = L^-1 X: Xbar = L^-T Ybar + (through L) ...
    Lbar = -Li.T @ Ybar @ Y.T
    Pm = Lc.T @ Lbar
    Phi = np.tril(Pm) - 0.5 * np.diag(np.diag(Pm))
    Gbar = Li.T @ Phi @ Li
    Gbar = 0.5 * (Gbar + Gbar.T)
    Xbar = Li.T @ Ybar + 2.0 * Gbar @ X
    return pot.E, Xbar.ravel()


def test_p9_lbfgs_reaches_cg_minimum():
    m = roks.Model(inputs.tiny_cell())
    emb = _RealEmbedding(m)
    psi0 = roks.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, 1000))
    st, hist = roks.solve(m, psi0, tol=1e-12, maxiter=600, orthonormalize_start=False)
    E_cg = hist[-1].E1
    # the chain-rule gradient against central differences
    x0 = emb.to_real(psi0).ravel()
    E, g = _energy_and_grad(m, emb, x0)
    rng = np.random.default_rng(3)
    d = rng.normal(size=x0.shape)
    h = 1e-5
    fd = (_energy_and_grad(m, emb, x0 + h * d)[0] - _energy_and_grad(m, emb, x0 - h * d)[0]) / (2 * h)
    assert abs(fd - g @ d) < 1e-7 * abs(fd)
    # L-BFGS from the CG minimum perturbed by ~3 % per coefficient: returns to
    # the same energy (a local minimum of E_S over orthonormal sets)
    xs = emb.to_real(st.psi).ravel()
    x1 = xs * (1.0 + 0.03 * rng.normal(size=xs.shape))
    E1 = _energy_and_grad(m, emb, x1)[0]
    assert E1 - E_cg > 1e-4
    res = scipy.optimize.minimize(lambda v: _energy_and_grad(m, emb, v), x1, jac=True,
                                  method="L-BFGS-B",
                                  options={"maxiter": 5000, "maxcor": 30, "ftol": 1e-16,
                                           "gtol": 1e-10})
    assert abs(res.fun - E_cg) < 1e-9, (res.fun, E_cg, res.message)
