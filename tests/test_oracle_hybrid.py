"""Pins of the oracle's hybrid exact exchange (reading R26 of
oracle/roks.py) on the CPU, on the tiny cell with PBE and a fraction 0.25 of
exact exchange:

* K^{sigma L} is symmetric and negative semi-definite (a Coulomb kernel
  with a minus sign);
* the exchange energy, built from pair Hartree energies, is half the
  occupation-weighted expectation of the operator, built by applying it
  (two routes: this pins the factor 1/2 and the weights);
* the functional's directional derivatives by central differences equal the
  gradient formed with the operator, for out-of-subspace variations and for
  rotations (K enters H^{sigma L} as the derivative of a E_x^HF)."""
import numpy as np
import scipy.linalg

from oracle import roks as orc
from paper_2605_28637_amd import inputs


def _model():
    s = dict(inputs.tiny_cell(), xc="pbe", exx=0.25)
    m = orc.Model(s)
    psi = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"]))
    return m, psi


def test_exchange_operator_is_symmetric_and_negative():
    m, psi = _model()
    pot = orc.potentials(m, psi)
    a = inputs.random_coefficients(m.miller, m.cell, 2, 41)
    Ka = orc.exx_apply(m, pot.u, 0, 0, a)
    ab = orc.dot(a[0], Ka[1])
    ba = orc.dot(a[1], Ka[0])
    assert abs(ab - ba) < 1e-12 * max(1.0, abs(ab))
    assert orc.dot(a[0], Ka[0]) < 0 and orc.dot(a[1], Ka[1]) < 0


def test_exchange_energy_is_half_the_operator_expectation():
    m, psi = _model()
    pot = orc.potentials(m, psi)
    for L in range(m.nconf):
        E = orc.exx_energy(m, pot.u, L)
        ev = 0.0
        for s in range(2):
            K = orc.exx_apply(m, pot.u, L, s, psi)
            ev += sum(float(m.occ[L, s, n]) * orc.dot(psi[n], K[n]) for n in range(m.nb))
        assert abs(E - 0.5 * ev) < 1e-12 * max(1.0, abs(E)), L


def test_directional_derivatives_with_exact_exchange():
    m, psi = _model()
    gr = orc.gradient(m, psi)
    d = inputs.random_coefficients(m.miller, m.cell, m.nb, 21)
    d = d - orc.overlap(psi, d).T @ psi
    d /= np.sqrt(np.sum(np.abs(d) ** 2))
    h = 1e-4
    fd = (orc.energy(m, orc.orthonormalize(psi + h * d))
          - orc.energy(m, orc.orthonormalize(psi - h * d))) / (2 * h)
    an = 2 * float(np.sum(np.real(np.conj(d) * gr.gI)))
    assert abs(fd - an) < 1e-7 * max(1, abs(an))
    rng = np.random.default_rng(3)
    A = rng.normal(size=(m.nb, m.nb))
    A = A - A.T
    fd = (orc.energy(m, scipy.linalg.expm(h * A).T @ psi)
          - orc.energy(m, scipy.linalg.expm(-h * A).T @ psi)) / (2 * h)
    an = float(np.sum(A * (gr.theta - gr.theta.T)))
    assert abs(fd - an) < 1e-7 * max(1, abs(an))
