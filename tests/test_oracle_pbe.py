"""Pins of the oracle's PBE exchange-correlation (oracle/xc.py, reading R25
of oracle/roks.py) on the CPU:

* with zero gradients PBE is the spin LDA (Slater + PW92) exactly, energy
  and potentials;
* the complex-step partial derivatives agree with central differences;
* at a huge gradient the exchange enhancement tends to 1 + kappa (the
  Lieb-Oxford bound of the construction) and the correlation energy density
  to zero;
* the grid potential is the derivative of the grid energy: perturbing one
  spin density at one grid point changes E_xc by v_xc^sigma(r) dV (this pins
  the divergence term's sign and factors)."""
import numpy as np

from oracle import roks as orc
from oracle import xc
from paper_2605_28637_amd import inputs


def test_zero_gradient_is_the_lda():
    rng = np.random.default_rng(0)
    ru = rng.uniform(1e-4, 0.5, 200)
    rd = rng.uniform(1e-4, 0.5, 200)
    z = np.zeros(200)
    e, fu, fd, fuu, fud, fdd = xc.pbe_point_derivatives(ru, rd, z, z, z)
    el, vu, vd = xc.lda(ru, rd)
    assert np.abs(e - el).max() < 1e-14
    assert np.abs(fu - vu).max() < 1e-12 and np.abs(fd - vd).max() < 1e-12


def test_complex_step_matches_central_differences():
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = np.array([rng.uniform(0.01, 0.4), rng.uniform(0.01, 0.4), rng.uniform(0, 0.05),
                      rng.uniform(-0.01, 0.01), rng.uniform(0, 0.05)])
        d = xc.pbe_point_derivatives(*[np.array([v]) for v in x])
        for k in range(5):
            h = 1e-6 * max(abs(x[k]), 1e-3)
            xp, xm = x.copy(), x.copy()
            xp[k] += h
            xm[k] -= h
            fd = (xc.pbe_energy_density(*xp) - xc.pbe_energy_density(*xm)) / (2 * h)
            assert abs(d[1 + k][0] - fd) < 1e-6 * max(1.0, abs(fd)), k


def test_large_gradient_limits():
    """At a huge gradient F_x -> 1 + kappa and H -> -eps_c (e_c -> 0), so
    e_xc -> (1 + kappa) e_x^LDA."""
    r = np.array([0.05])
    big = np.array([1e9])
    e_big = xc.pbe_point_derivatives(r, r, big, big, big)[0]
    ex_lda = xc.exchange(r, r)[0]
    assert abs(e_big[0] / ex_lda[0] - (1 + xc.PBE_KAPPA)) < 1e-3


def test_grid_potential_is_the_energy_derivative():
    s = dict(inputs.tiny_cell(), xc="pbe")
    m = orc.Model(s)
    psi = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"]))
    pot = orc.potentials(m, psi)
    ru, rd = pot.rho[0, 0].copy(), pot.rho[0, 1].copy()
    e, vu, vd = orc.gga_xc(m, ru, rd)
    dV = m.omega / m.ntot
    rng = np.random.default_rng(2)
    flat = np.argsort(ru.ravel())[::-1]
    for j in list(flat[:3]) + list(rng.choice(flat[: len(flat) // 2], 3)):
        idx = np.unravel_index(j, ru.shape)
        for spin, v in ((0, vu), (1, vd)):
            eps = 1e-6 * max(ru[idx], 1e-6)
            Es = []
            for sgn in (1, -1):
                a, b = ru.copy(), rd.copy()
                (a if spin == 0 else b)[idx] += sgn * eps
                Es.append(orc.gga_xc(m, a, b)[0].sum() * dV)
            fd = (Es[0] - Es[1]) / (2 * eps)
            assert abs(fd - v[idx] * dV) < 1e-6 * abs(v[idx] * dV) + 1e-12, (j, spin)
