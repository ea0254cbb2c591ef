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


# ---------------------------------------------------------------------------
# PBE (generalised gradient approximation), spin-polarised
# ---------------------------------------------------------------------------
# Perdew, Burke and Ernzerhof, Phys. Rev. Lett. 77, 3865 (1996), written from
# the published form: exchange by spin scaling, E_x[n_up, n_dn] =
# (E_x[2 n_up] + E_x[2 n_dn]) / 2 with e_x[n] = n eps_x^unif(n) F_x(s),
# F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa), s = |grad n| / (2 k_F n);
# correlation e_c = n (eps_c^PW92(r_s, zeta) + H), H = gamma phi^3
# ln(1 + beta/gamma t^2 (1 + A t^2) / (1 + A t^2 + A^2 t^4)),
# A = beta/gamma / (exp(-eps_c / (gamma phi^3)) - 1), t = |grad n| / (2 phi k_s n),
# phi = ((1 + zeta)^(2/3) + (1 - zeta)^(2/3)) / 2, k_s = (4 k_F / pi)^(1/2).
# The paper uses PBE (Sec. III) without restating it.  The energy density is
# written once, in operations that stay analytic for complex arguments, and
# its partial derivatives come from the complex step f'(x) = Im f(x + i h) / h
# (no subtraction, so exact to rounding): "parity unpinned" for the printed
# constants, pinned by the LDA limit and by finite differences of the energy.
PBE_KAPPA = 0.804
PBE_BETA = 0.06672455060314922
PBE_MU = PBE_BETA * np.pi ** 2 / 3.0
PBE_GAMMA = (1.0 - np.log(2.0)) / np.pi ** 2


def _pw92_eps(rho, z):
    """eps_c^PW92(r_s(rho), zeta), complex-safe (no clamps)."""
    rs = (3.0 / (4.0 * np.pi * rho)) ** (1.0 / 3.0)

    def G(prm):
        A, a1, b1, b2, b3, b4 = prm
        srs = np.sqrt(rs)
        Q = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs)
        return -2.0 * A * (1.0 + a1 * rs) * np.log(1.0 + 1.0 / Q)

    ec0, ec1, ac = G(PW92_PARAMS["ec0"]), G(PW92_PARAMS["ec1"]), -G(PW92_PARAMS["mac"])
    f = ((1.0 + z) ** (4.0 / 3.0) + (1.0 - z) ** (4.0 / 3.0) - 2.0) / TWO43M2
    z4 = z ** 4
    return ec0 + ac * f / FZ20 * (1.0 - z4) + (ec1 - ec0) * f * z4


def pbe_energy_density(ru, rd, suu, sud, sdd, xscale=1.0):
    """e_xc(rho_up, rho_dn, sigma_uu, sigma_ud, sigma_dd), sigma_ab =
    grad rho_a . grad rho_b, with the exchange part scaled by xscale (1 - a
    for a hybrid with a fraction a of exact exchange); all densities above
    the floor."""
    def ex_spin(r, s):
        n = 2.0 * r
        kf = (3.0 * np.pi ** 2 * n) ** (1.0 / 3.0)
        s2 = 4.0 * s / (4.0 * kf * kf * n * n)          # |grad n|^2 = 4 sigma
        Fx = 1.0 + PBE_KAPPA - PBE_KAPPA / (1.0 + PBE_MU * s2 / PBE_KAPPA)
        ex_unif = -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * n ** (1.0 / 3.0)
        return 0.5 * n * ex_unif * Fx

    rho = ru + rd
    z = (ru - rd) / rho
    eps_c = _pw92_eps(rho, z)
    phi = 0.5 * ((1.0 + z) ** (2.0 / 3.0) + (1.0 - z) ** (2.0 / 3.0))
    kf = (3.0 * np.pi ** 2 * rho) ** (1.0 / 3.0)
    ks2 = 4.0 * kf / np.pi
    g2 = suu + 2.0 * sud + sdd
    t2 = g2 / (4.0 * phi * phi * ks2 * rho * rho)
    phi3 = phi ** 3
    A = (PBE_BETA / PBE_GAMMA) / (np.exp(-eps_c / (PBE_GAMMA * phi3)) - 1.0)
    At2 = A * t2
    H = PBE_GAMMA * phi3 * np.log(1.0 + PBE_BETA / PBE_GAMMA * t2 * (1.0 + At2)
                                  / (1.0 + At2 + At2 * At2))
    return xscale * (ex_spin(ru, suu) + ex_spin(rd, sdd)) + rho * (eps_c + H)


def pbe_point_derivatives(ru, rd, suu, sud, sdd, xscale=1.0):
    """e and its partial derivatives (d/d rho_up, d/d rho_dn, d/d sigma_uu,
    d/d sigma_ud, d/d sigma_dd) by the complex step, per point; points whose
    total density is below the floor give zeros."""
    args = [np.asarray(a, dtype=np.float64) for a in (ru, rd, suu, sud, sdd)]
    live = (args[0] + args[1]) >= RHO_FLOOR
    floor = 1e-30
    a = [np.where(live, np.maximum(args[0], floor), 1.0), np.where(live, np.maximum(args[1], floor), 1.0),
         np.where(live, args[2], 0.0), np.where(live, args[3], 0.0), np.where(live, args[4], 0.0)]
    e = np.real(pbe_energy_density(*a, xscale=xscale))
    d = []
    for k in range(5):
        h = 1e-20 * np.maximum(np.abs(a[k]), 1e-20)
        b = [x.astype(complex) for x in a]
        b[k] = b[k] + 1j * h
        d.append(np.imag(pbe_energy_density(*b, xscale=xscale)) / h)
    return (np.where(live, e, 0.0),) + tuple(np.where(live, x, 0.0) for x in d)
