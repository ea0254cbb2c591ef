"""DIIS on the ROKS residual: the CPU oracle of roks_diis_step.

Test infrastructure only, like the rest of oracle/: only tests/,
__graft_entry__.smoke() and bench.py's CPU baseline may call it.

Sec. II A rewrites the stationarity condition of the singlet functional
(Eq. gradient at g = 0) as Eq. residual_frank, F^n|n> = sum_m |m> Lambda_mn,
and names the DIIS method of Hutter, Luthi and Parrinello (1994) for driving
that residual to zero, with the couplings lambda_ab = 1/2, lambda_ba = -1/2 of
the two open shells as the variant that steers away from the triplet-like
collapse; its implementation details are left to a later report.  The steps
below are this build's reading, in this order (D1-D5):

D1  residual r_n = F^n|n> - sum_m |m> Lambda_mn with
    Lambda_mn = theta_mn - lambda_mn (theta_mn - theta_nm) (real Gamma-point
    orbitals: theta*_nm = theta_nm; with the overlap S of reading R27 the
    sum runs over S|m>, as in Eq. gradient).  The printed equation carries the
    antisymmetric term with a plus sign and a second sum over m; the reading
    takes the sign that makes it Eq. gradient's zero: with every
    lambda_mn = 1/2, r_n is the full gradient g_I + g_II.  With the
    asymmetric coupling, lambda_ab = 1/2 and lambda_ba = -1/2 for the open
    bands a < b (lambda_mn multiplies the coefficient of |m> in the residual
    of band n); both residual components of the pair are then
    (theta_ab - theta_ba) / 2, so the fixed points are the same stationary
    states, while the step along the a-b rotation changes sign.
D2  error vector e_n = K_n r_n with the Teter preconditioner of Eq. prec_k
    and reading R1 (E_ref from r_n itself; the descent sign carried by K),
    and no projection: the paper notes that DIIS uses K alone.
D3  B_ij = sum_n <e^i_n|e^j_n> over the kept iterates (at most `history`,
    the oldest dropped first); the coefficients c minimise c^T B c subject to
    sum_i c_i = 1 (the bordered linear system of DIIS).  If that system is
    singular, the oldest iterates are dropped until it is not.
D4  psi' = sum_i c_i (psi^i + step e^i).
D5  psi'' = psi' orthonormalised by the Cholesky factor of its Gram matrix
    (of <m|S|n> under R27), band order kept (the CG's reading R9).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Tuple

import numpy as np

from . import roks as orc

LAMBDA = 0.5


def open_bands(model: orc.Model) -> List[int]:
    """Bands of the open shells (neither closed nor virtual), in band order."""
    return [n for n in range(model.nb)
            if not model.shell_closed[model.band_shell[n]]
            and not model.shell_virtual[model.band_shell[n]]]


def couplings(model: orc.Model, asymmetric: bool) -> np.ndarray:
    """lambda_mn of D1."""
    lam = np.full((model.nb, model.nb), LAMBDA)
    if asymmetric:
        ob = open_bands(model)
        if len(ob) == 2:
            a, b = ob
            lam[a, b] = LAMBDA
            lam[b, a] = -LAMBDA
    return lam


def residual(model: orc.Model, gr: orc.Gradient, asymmetric: bool = False) -> np.ndarray:
    """D1: r_n = F^n|n> - sum_m S|m> Lambda_mn."""
    th = gr.theta
    Lam = th - couplings(model, asymmetric) * (th - th.T)
    return gr.Y - Lam.T @ orc.apply_S(model, gr.psi)


def error_vectors(model: orc.Model, r: np.ndarray) -> np.ndarray:
    """D2: e_n = K_n r_n, Teter K with E_ref from r_n."""
    e = np.zeros_like(r)
    for n in range(model.nb):
        Er = orc.teter_reference_energy(model, r[n])
        if Er <= 0.0:
            continue
        x = 0.5 * model.g2 / Er
        e[n] = -(2.0 / Er) * orc.teter_polynomial_ratio(x) * r[n]
    return e


def diis_coefficients(B: np.ndarray) -> Optional[np.ndarray]:
    """D3: argmin c^T B c with sum c = 1 from the bordered system; None when
    it is singular."""
    k = len(B)
    A = np.zeros((k + 1, k + 1))
    A[:k, :k] = B
    A[:k, k] = 1.0
    A[k, :k] = 1.0
    rhs = np.zeros(k + 1)
    rhs[k] = 1.0
    try:
        sol = np.linalg.solve(A, rhs)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(sol)):
        return None
    return sol[:k]


@dataclasses.dataclass
class DiisState:
    psi: np.ndarray
    kept: List[Tuple[np.ndarray, np.ndarray]] = dataclasses.field(default_factory=list)


@dataclasses.dataclass
class DiisInfo:
    E: float            # energy of the step's input orbitals
    rnorm2: float       # sum_n <r_n|r_n>
    used: int           # iterates combined
    coeffs: np.ndarray
    open_coupling: float  # theta_ab - theta_ba of the open pair (0 without one)


def diis_step(model: orc.Model, state: DiisState, history: int = 6, step: float = 0.3,
              asymmetric: bool = False) -> DiisInfo:
    gr = orc.gradient(model, state.psi)
    r = residual(model, gr, asymmetric)
    e = error_vectors(model, r)
    state.kept.append((state.psi, e))
    state.kept = state.kept[-history:]
    while True:
        k = len(state.kept)
        B = np.array([[sum(orc.dot(state.kept[i][1][n], state.kept[j][1][n])
                           for n in range(model.nb)) for j in range(k)] for i in range(k)])
        c = diis_coefficients(B)
        if c is not None or k == 1:
            break
        state.kept = state.kept[1:]
    if c is None:
        c = np.ones(1)
    new = sum(c[i] * (state.kept[i][0] + step * state.kept[i][1]) for i in range(len(c)))
    state.psi = orc.orthonormalize(new, model)
    ob = open_bands(model)
    oc = float(gr.theta[ob[0], ob[1]] - gr.theta[ob[1], ob[0]]) if len(ob) == 2 else 0.0
    return DiisInfo(gr.pot.E, float(sum(orc.dot(r[n], r[n]) for n in range(model.nb))),
                    len(c), c, oc)


def diis_solve(model: orc.Model, psi0: np.ndarray, tol: float = 1e-10, maxiter: int = 500,
               history: int = 6, step: float = 0.3, asymmetric: bool = False):
    """DIIS steps until the energy changes by less than tol on two consecutive
    steps (the CG's rule); returns the state and the step records."""
    st = DiisState(orc.orthonormalize(psi0, model))
    hist: List[DiisInfo] = []
    hits = 0
    for _ in range(maxiter):
        info = diis_step(model, st, history, step, asymmetric)
        if hist and abs(info.E - hist[-1].E) < tol:
            hits += 1
        else:
            hits = 0
        hist.append(info)
        if hits >= 2:
            break
    return st, hist
