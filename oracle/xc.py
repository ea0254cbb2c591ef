"""Spin-polarised LDA exchange-correlation for the oracle (FP64, NumPy).

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

The paper names only "LDA" (Sec. III / IV A); the form used here is the
spin-polarised Slater-Dirac exchange plus the Perdew-Wang 1992 correlation
(Phys. Rev. B 45, 13244), written from the published parametrisation.  The
PW92 constants below are not reproduced anywhere in the paper, so their
absolute values are "parity unpinned": the tests pin the exchange part by its
closed form and both parts' potentials by finite differences of the energy,
plus the spin-symmetry and full-polarisation limits.

Every function returns, per grid point, the energy density e = rho * eps_xc
and the two spin potentials v_up = d e / d rho_up, v_dn = d e / d rho_dn.
Densities below RHO_FLOOR give e = v = 0 and |zeta| is clamped to 1.
"""
from __future__ import annotations

import numpy as np

RHO_FLOOR = 1e-12

# PW92 G(rs; A, alpha1, beta1..beta4), p = 1, for eps_c(rs, 0), eps_c(rs, 1), -alpha_c(rs)
PW92_PARAMS = {
    "ec0": (0.031091, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294),
    "ec1": (0.015545, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517),
    "mac": (0.016887, 0.11125, 10.357, 3.6231, 0.88026, 0.49671),
}
FZ20 = 1.709921  # f''(0) as printed by PW92
TWO43M2 = 2.0 ** (4.0 / 3.0) - 2.0


def exchange(rho_up: np.ndarray, rho_dn: np.ndarray):
    """Slater-Dirac exchange: e_x = -(3/4)(6/pi)^(1/3) (rho_up^(4/3) + rho_dn^(4/3))."""
    ru = np.maximum(rho_up, 0.0)
    rd = np.maximum(rho_dn, 0.0)
    cx = (6.0 / np.pi) ** (1.0 / 3.0)
    e = -0.75 * cx * (ru ** (4.0 / 3.0) + rd ** (4.0 / 3.0))
    vu = -cx * ru ** (1.0 / 3.0)
    vd = -cx * rd ** (1.0 / 3.0)
    dead = (ru + rd) < RHO_FLOOR
    return np.where(dead, 0.0, e), np.where(dead, 0.0, vu), np.where(dead, 0.0, vd)


def _pw92_g(rs: np.ndarray, prm):
    """G(rs) = -2A(1 + a1 rs) ln(1 + 1/Q), Q = 2A(b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2);
    returns (G, dG/drs)."""
    A, a1, b1, b2, b3, b4 = prm
    srs = np.sqrt(rs)
    Q = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs)
    dQ = 2.0 * A * (0.5 * b1 / srs + b2 + 1.5 * b3 * srs + 2.0 * b4 * rs)
    lg = np.log1p(1.0 / Q)
    G = -2.0 * A * (1.0 + a1 * rs) * lg
    dG = -2.0 * A * a1 * lg + 2.0 * A * (1.0 + a1 * rs) * dQ / (Q * Q + Q)
    return G, dG


def correlation(rho_up: np.ndarray, rho_dn: np.ndarray):
    """PW92 correlation with the spin interpolation
    eps_c = ec0 + ac f(z)/f''(0) (1 - z^4) + (ec1 - ec0) f(z) z^4."""
    ru = np.maximum(rho_up, 0.0)
    rd = np.maximum(rho_dn, 0.0)
    rho = ru + rd
    dead = rho < RHO_FLOOR
    rho_s = np.where(dead, 1.0, rho)
    z = np.clip((ru - rd) / rho_s, -1.0, 1.0)
    rs = (3.0 / (4.0 * np.pi * rho_s)) ** (1.0 / 3.0)
    ec0, dec0 = _pw92_g(rs, PW92_PARAMS["ec0"])
    ec1, dec1 = _pw92_g(rs, PW92_PARAMS["ec1"])
    mac, dmac = _pw92_g(rs, PW92_PARAMS["mac"])
    ac, dac = -mac, -dmac
    opz, omz = 1.0 + z, 1.0 - z
    f = (opz ** (4.0 / 3.0) + omz ** (4.0 / 3.0) - 2.0) / TWO43M2
    fp = (4.0 / 3.0) * (opz ** (1.0 / 3.0) - omz ** (1.0 / 3.0)) / TWO43M2
    z3 = z ** 3
    z4 = z3 * z
    eps = ec0 + ac * f / FZ20 * (1.0 - z4) + (ec1 - ec0) * f * z4
    deps_drs = dec0 + dac * f / FZ20 * (1.0 - z4) + (dec1 - dec0) * f * z4
    deps_dz = (4.0 * z3 * f * (ec1 - ec0 - ac / FZ20)
               + fp * (z4 * (ec1 - ec0) + (1.0 - z4) * ac / FZ20))
    common = eps - rs / 3.0 * deps_drs
    vu = common + (1.0 - z) * deps_dz
    vd = common - (1.0 + z) * deps_dz
    e = rho * eps
    return np.where(dead, 0.0, e), np.where(dead, 0.0, vu), np.where(dead, 0.0, vd)


def lda(rho_up: np.ndarray, rho_dn: np.ndarray, kind: str = "pw92"):
    """Spin-polarised LDA: kind "pw92" (Slater + PW92) or "x" (exchange only)."""
    ex, vxu, vxd = exchange(rho_up, rho_dn)
    if kind == "x":
        return ex, vxu, vxd
    if kind != "pw92":
        raise ValueError(kind)
    ec, vcu, vcd = correlation(rho_up, rho_dn)
    return ex + ec, vxu + vcu, vxd + vcd
