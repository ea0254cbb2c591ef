"""Dense brute-force paths for tiny cells (oracle; FP64).

TEST INFRASTRUCTURE ONLY.  These build explicit plane-wave Hamiltonian
matrices, so they are a second, independent route to what oracle.roks
computes with FFTs:

* H_{GG'} = |G|^2/2 delta_GG' + V~(G - G') + sum_ij beta_i(G) D_ij beta_j(G')*
  with V~(m) = N^-3 sum_j V(r_j) e^{-i G_m . r_j} taken modulo the grid, the
  exact matrix of the grid-based local operator.
* A closed-shell self-consistent-field loop by dense diagonalisation with
  Pulay mixing of the density: a different algorithm from the CG of the
  paper's Sec. II A that must reach the same ground-state energy.  With
  overlap coefficients it solves the generalised problem H c = eps S c with
  the explicit S_{GG'} = delta_GG' + sum_kl beta_k(G) q_kl beta_l(G')*.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import roks, xc as xcmod


def local_matrix(model: "roks.Model", vloc: np.ndarray) -> np.ndarray:
    vt = np.fft.fftn(vloc) / model.ntot
    d = model.miller[:, None, :] - model.miller[None, :, :]
    return vt[d[..., 0] % model.grid[0], d[..., 1] % model.grid[1], d[..., 2] % model.grid[2]]


def nonlocal_matrix(model: "roks.Model") -> np.ndarray:
    return model.beta.T @ model.D @ np.conj(model.beta)


def overlap_matrix(model: "roks.Model") -> np.ndarray:
    """The explicit S on the full sphere (the identity without q)."""
    S = np.eye(model.npw, dtype=complex)
    if model.nproj:
        S += model.beta.T @ model.Q @ np.conj(model.beta)
    return S


def hamiltonian_matrix(model: "roks.Model", vloc: np.ndarray) -> np.ndarray:
    return np.diag(0.5 * model.g2).astype(complex) + local_matrix(model, vloc) + nonlocal_matrix(model)


def scf_closed_shell(model: "roks.Model", n_occ: int, tol: float = 1e-12, maxiter: int = 200,
                     history: int = 8, mix: float = 0.5):
    """Restricted closed-shell SCF: rho = 2 sum_{n<n_occ} |psi_n|^2 from the
    lowest eigenvectors of the dense H[rho]; Pulay (DIIS) density mixing.
    Returns (E, eigenvectors [n_occ][npw], eigenvalues)."""
    def density_of(C):
        # eigenvectors carry an arbitrary phase, so use |u|^2 of the complex field
        u = np.array([np.fft.ifftn(model.to_grid(c)) * model.ntot for c in C])
        return 2.0 * (np.abs(u) ** 2).sum(axis=0) / model.omega

    def energy_of(C, rho):
        kin = roks.band_kinetic(model, C)
        P = np.conj(model.beta) @ C.T  # complex: eigenvectors carry a phase
        enl = np.real(np.einsum("in,ij,jn->n", np.conj(P), model.D, P))
        vh, eh = roks.hartree(model, rho)
        e, _, _ = xcmod.lda(0.5 * rho, 0.5 * rho, model.xc)
        return (2.0 * (kin.sum() + enl.sum()) + model.integrate(model.vext_r * rho) + eh
                + model.integrate(e))

    def potential_of(rho):
        vh, _ = roks.hartree(model, rho)
        _, vu, _ = xcmod.lda(0.5 * rho, 0.5 * rho, model.xc)
        return model.vext_r + vh + vu

    Smat = overlap_matrix(model)

    def eig(H):
        # S-orthonormal eigenvectors of H c = eps S c
        return scipy.linalg.eigh(H, Smat)

    H = hamiltonian_matrix(model, model.vext_r)
    w, V = eig(H)
    C = V[:, :n_occ].T
    rho = density_of(C)
    rhos, resid = [], []
    E_old = None
    for it in range(maxiter):
        H = hamiltonian_matrix(model, potential_of(rho))
        w, V = eig(H)
        C = V[:, :n_occ].T
        rho_out = density_of(C)
        E = energy_of(C, rho_out)
        r = rho_out - rho
        rhos.append(rho.copy())
        resid.append(r)
        rhos, resid = rhos[-history:], resid[-history:]
        k = len(resid)
        B = np.empty((k + 1, k + 1))
        for i in range(k):
            for j in range(k):
                B[i, j] = np.sum(resid[i] * resid[j])
        B[k, :], B[:, k], B[k, k] = -1.0, -1.0, 0.0
        rhs = np.zeros(k + 1)
        rhs[k] = -1.0
        try:
            coef = np.linalg.solve(B, rhs)[:k]
        except np.linalg.LinAlgError:
            coef = np.zeros(k)
            coef[-1] = 1.0
        rho = sum(c * (x + mix * y) for c, x, y in zip(coef, rhos, resid))
        if E_old is not None and abs(E - E_old) < tol and np.abs(r).max() < 1e-9:
            break
        E_old = E
    return E, C, w[:n_occ]
