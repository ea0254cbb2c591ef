"""Geometry relaxation and the Franck-Condon cycle: the CPU oracle of
roks_relax / roks_franck_condon.

Test infrastructure only, like the rest of oracle/: only tests/,
__graft_entry__.smoke() and bench.py's CPU baseline may call it.

Sec. IV B relaxes the atomic positions in the ground and the excited state
(fixed cell, forces below a threshold) and reports the vertical absorption
energy, the two Franck-Condon shifts, the emission energy and the
mass-weighted displacement Delta Q between the two equilibrium geometries.
The optimiser is not specified; this build's reading (G0-G4):

G0  the energy of a geometry is the electronic E (the constrained functional
    of Sec. II A at its minimum) plus an ion-ion pair repulsion
    sum_{I<J, images} B exp(-|R_I - R_J - t| / rho) over the 27 nearest cell
    translations t: the paper's total energies carry the ions' Coulomb
    repulsion, which the synthetic Gaussian-well atoms lack (without it the
    wells fuse).  The forces are Eq. force_hf's plus this term's.

G1  BFGS in Cartesian positions: inverse Hessian H_0 = h0 I; step s = H F
    with F the Hellmann-Feynman forces (Eq. force_hf) of the electronic
    minimum, scaled down so that no atom moves more than max_step; after the
    new forces, with y = F_old - F_new, the BFGS update of H when s.y > 0,
    else H = h0 I.
G2  the orbitals of each geometry: CG from those of the previous geometry,
    restarted every scf_restart iterations (without restarts the excited
    state's solve from ground-state orbitals can stall far above its
    minimum), to |dE| < scf_tol on two consecutive iterations.
G3  a step that raises the energy is halved, at most four times, and H is
    reset to h0 I; a fifth rise takes the step anyway.
G4  stop when max_I |F_I| < fmax (or after maxsteps steps).

Franck-Condon cycle (the paper's definitions): R_gs from the ground-state
relaxation; E_abs = E^ex(R_gs) - E^gs(R_gs), the excited state solved from
the ground-state orbitals; R_ex from the excited-state relaxation started at
R_gs; E_FC,ex = E^ex(R_gs) - E^ex(R_ex); E_FC,gs = E^gs(R_ex) - E^gs(R_gs);
E_emi = E_abs - E_FC,ex - E_FC,gs; Delta Q = [sum_a M_a |R^ex_a - R^gs_a|^2]^1/2
(masses in amu, lengths in bohr).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List

import numpy as np

from . import roks as orc


@dataclasses.dataclass
class RelaxParams:
    fmax: float = 1e-4       # Ha/bohr
    maxsteps: int = 60
    scf_tol: float = 1e-11   # Ha
    scf_maxiter: int = 800
    scf_restart: int = 20
    max_step: float = 0.2    # bohr
    h0: float = 1.0          # bohr^2 / Ha
    pair_B: float = 1.0      # Ha
    pair_rho: float = 0.4    # bohr


def pair_repulsion(pos: np.ndarray, cell: np.ndarray, B: float, rho: float):
    """G0: E = sum_{I<J} sum_t B exp(-r / rho), r = |R_I - R_J - t| over the
    27 translations t = (i, j, k) . cell, i, j, k in {-1, 0, 1}; F = -dE/dR."""
    nat = len(pos)
    E = 0.0
    F = np.zeros((nat, 3))
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)],
                      dtype=float) @ np.asarray(cell)
    for I in range(nat):
        for J in range(I + 1, nat):
            for t in shifts:
                d = pos[I] - pos[J] - t
                r = float(np.sqrt(d @ d))
                e = B * np.exp(-r / rho)
                E += e
                f = (e / rho) * d / r
                F[I] += f
                F[J] -= f
    return E, F


@dataclasses.dataclass
class RelaxResult:
    pos: np.ndarray
    psi: np.ndarray
    E: float
    forces: np.ndarray
    steps: int
    scf_iterations: int
    converged: bool
    history: List[Dict]


def _electrons(model: orc.Model, psi: np.ndarray, p: RelaxParams):
    """G2 and G0: the orbitals, the total energy and the CG iterations."""
    # with overlap coefficients (R27) S moves with the atoms: the start
    # orbitals are S-orthonormalised for this geometry first
    st, h = orc.solve(model, psi, tol=p.scf_tol, maxiter=p.scf_maxiter,
                      orthonormalize_start=model.has_q, restart_period=p.scf_restart)
    Ep, _ = pair_repulsion(model.pos, model.cell, p.pair_B, p.pair_rho)
    return st.psi, h[-1].E1 + Ep, len(h)


def total_forces(model: orc.Model, psi: np.ndarray, p: RelaxParams) -> np.ndarray:
    _, Fp = pair_repulsion(model.pos, model.cell, p.pair_B, p.pair_rho)
    return orc.forces(model, psi) + Fp


def bfgs(evaluate, x0: np.ndarray, state0, p: RelaxParams):
    """G1, G3, G4 on a function given by evaluate(x, state) -> (E, F, state,
    work): the energy and forces at x, the electronic state reached from
    `state`, the work done.  Every trial of a step starts from the state of
    the accepted geometry.  Returns x, E, F, state, steps, work, history."""
    n = len(x0)
    nat = n // 3
    x = np.asarray(x0, dtype=float).copy()
    E, F, state, work = evaluate(x, state0)
    H = p.h0 * np.eye(n)
    fm = lambda v: float(np.linalg.norm(v.reshape(nat, 3), axis=1).max())
    hist = [{"E": E, "fmax": fm(F)}]
    steps = 0
    while steps < p.maxsteps and fm(F) >= p.fmax:
        s = H @ F
        big = fm(s)
        if big > p.max_step:
            s *= p.max_step / big
        for halving in range(5):
            E_n, F_n, st_n, w = evaluate(x + s, state)
            work += w
            if E_n <= E or halving == 4:
                break
            s *= 0.5
            H = p.h0 * np.eye(n)
        y = F - F_n
        sy = float(s @ y)
        if sy > 0.0:
            rho = 1.0 / sy
            V = np.eye(n) - rho * np.outer(s, y)
            H = V @ H @ V.T + rho * np.outer(s, s)
        else:
            H = p.h0 * np.eye(n)
        x, E, F, state = x + s, E_n, F_n, st_n
        steps += 1
        hist.append({"E": E, "fmax": fm(F)})
    return x, E, F, state, steps, work, hist


def relax(model: orc.Model, psi: np.ndarray, p: RelaxParams = RelaxParams()) -> RelaxResult:
    nat = len(model.pos)

    def evaluate(x, psi_start):
        model.set_positions(x.reshape(nat, 3))
        psi_n, E, n = _electrons(model, psi_start, p)
        return E, total_forces(model, psi_n, p).reshape(-1), psi_n, n

    x, E, F, psi, steps, nscf, hist = bfgs(evaluate, model.pos.reshape(-1), psi, p)
    model.set_positions(x.reshape(nat, 3))
    fmax = float(np.linalg.norm(F.reshape(nat, 3), axis=1).max())
    return RelaxResult(x.reshape(nat, 3), psi, E, F.reshape(nat, 3), steps, nscf, fmax < p.fmax, hist)


def franck_condon(gs_system: Dict, ex_system: Dict, psi0: np.ndarray, masses: np.ndarray,
                  p: RelaxParams = RelaxParams()) -> Dict:
    """The cycle of Sec. IV B from the start positions of gs_system and the
    (orthonormal) start orbitals psi0 of the ground state."""
    mg = orc.Model(gs_system)
    me = orc.Model(ex_system)
    rg = relax(mg, psi0, p)
    R_gs = rg.pos.copy()
    me.set_positions(R_gs)
    psi_ex, E_ex_gs, _ = _electrons(me, rg.psi, p)
    re = relax(me, psi_ex, p)
    R_ex = re.pos.copy()
    mg.set_positions(R_ex)
    _, E_gs_ex, _ = _electrons(mg, rg.psi, p)
    E_abs = E_ex_gs - rg.E
    fc_ex = E_ex_gs - re.E
    fc_gs = E_gs_ex - rg.E
    dQ = float(np.sqrt(np.sum(np.asarray(masses)[:, None] * (R_ex - R_gs) ** 2)))
    return {"E_gs_at_gs": rg.E, "E_ex_at_gs": E_ex_gs, "E_ex_at_ex": re.E, "E_gs_at_ex": E_gs_ex,
            "E_abs": E_abs, "E_FC_ex": fc_ex, "E_FC_gs": fc_gs, "E_emi": E_abs - fc_ex - fc_gs,
            "dQ": dQ, "R_gs": R_gs, "R_ex": R_ex, "gs_steps": rg.steps, "ex_steps": re.steps,
            "gs_converged": rg.converged, "ex_converged": re.converged}
