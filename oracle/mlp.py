"""Oracle of the learned rescaling of the Teter preconditioner (FP64, NumPy).

TEST INFRASTRUCTURE ONLY.

This part is not in the paper: it modifies the preconditioner K of Eq.
(prec_k) by a per-coefficient factor s_theta > 0 predicted by a small
multilayer perceptron, p_I = (1 - P) (s_theta K g_I).  Definitions (the GPU
library implements the same ones independently):

* network: x (3) -> Linear(3, 64) -> GELU -> Linear(64, 64) -> GELU ->
  Linear(64, 1) = o;  s = exp(2 tanh(o)) in [e^-2, e^2], so K stays negative
  definite.  GELU(z) = z Phi(z) with the normal CDF Phi (erf form).
  Parameters, flat (4 481): W1[64][3], b1[64], W2[64][64], b2[64], w3[64], b3.
* features of band n and coefficient G depend on |G|^2 only through the
  band's Teter variable: x1 = log(1 + (|G|^2/2) / E_ref,n), x2 = log <n|T|n>,
  x3 = log ||g_I,n||  (E_ref,n as in reading R1).  Coefficients with equal
  |G|^2 (a "G shell") share one network evaluation.
* target: the converged orbitals psi_inf, aligned to the current ones psi_i
  within each occupation shell by the orthogonal polar factor of
  O_mn = <psi_inf_m|psi_i_n> (orthogonal Procrustes), give the correction
  delta_n = (1 - P_i) psi_inf'_n.
* loss of one recorded iterate (a segment; scale free as a whole, the line
  search fixes the step length): L = 1 - <a|delta>^2 / (<a|a> <delta|delta>)
  with a_n = s K g_I,n and the inner products summed over all occupied bands
  with a gradient, so the shape within a band and the relative weights of
  the bands are both trained.  The inner products are taken in an energy
  norm, <x|y>_h = sum_G h_n(G) x*(G) y(G) with the diagonal Hessian model
  h_n(G) = |G|^2/2 + <n|T|n>: a stiff component that the correction does
  not need then costs what it costs the line search.  With moments per
  (band n, G shell k): alpha = <Kg_n|delta_n>_h,k, beta = <Kg_n|Kg_n>_h,k,
  gamma = <delta_n|delta_n>_h,k,
  A = sum s alpha, B = sum s^2 beta, C = sum gamma over the segment and
  L = 1 - A^2/(B C); the training loss is the mean over segments with
  B, C > 0.  band_loss takes one segment per row.
* inference: one constant for all bands makes sum_n <s K g_n|g_n> equal to
  the plain preconditioner's; the loss leaves this overall length free.
* optimiser: Adam (Kingma & Ba 2015) with bias correction.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np
import scipy.linalg
from scipy.special import erf

WIDTH = 64
NFEAT = 3
NPARAM = WIDTH * NFEAT + WIDTH + WIDTH * WIDTH + WIDTH + WIDTH + 1  # 4481


def unpack(theta: np.ndarray) -> Dict[str, np.ndarray]:
    t = np.asarray(theta, dtype=np.float64)
    assert t.size == NPARAM
    o = 0
    out = {}
    for name, shape in (("W1", (WIDTH, NFEAT)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)),
                        ("b2", (WIDTH,)), ("w3", (WIDTH,)), ("b3", (1,))):
        n = int(np.prod(shape))
        out[name] = t[o:o + n].reshape(shape)
        o += n
    return out


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def forward(theta: np.ndarray, X: np.ndarray):
    """o and the activations of every layer for samples X [S][3]."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    o = h2 @ p["w3"] + p["b3"][0]
    return o, (X, z1, h1, z2, h2)


def scale_of(o: np.ndarray) -> np.ndarray:
    return np.exp(2.0 * np.tanh(o))


def backward(theta: np.ndarray, cache, do: np.ndarray) -> np.ndarray:
    """Gradient of sum_s do_s o_s with respect to the flat parameters."""
    p = unpack(theta)
    X, z1, h1, z2, h2 = cache
    g = {}
    g["w3"] = h2.T @ do
    g["b3"] = np.array([do.sum()])
    dz2 = np.outer(do, p["w3"]) * gelu_prime(z2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"]) * gelu_prime(z1)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return np.concatenate([g[k].ravel() for k in ("W1", "b1", "W2", "b2", "w3", "b3")])


def init_params(seed: int) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every weight and bias,
    last layer scaled by 1e-2 so the untrained network is close to s = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for shape, fan in (((WIDTH, NFEAT), NFEAT), ((WIDTH,), NFEAT), ((WIDTH, WIDTH), WIDTH),
                       ((WIDTH,), WIDTH), ((WIDTH,), WIDTH), ((1,), WIDTH)):
        b = 1.0 / math.sqrt(fan)
        parts.append(rng.uniform(-b, b, size=shape).ravel())
    t = np.concatenate(parts)
    u = unpack(t)
    u["w3"][:] *= 1e-2
    u["b3"][:] = 0.0
    return t.astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# features, G shells, targets and moments
# ---------------------------------------------------------------------------
def g_shells(g2half: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Distinct |G|^2/2 values (keyed at 1e-9 Ha) and the shell index of each G."""
    keys = np.rint(np.asarray(g2half) * 1e9).astype(np.int64)
    uniq, inv = np.unique(keys, return_inverse=True)
    first = np.zeros(len(uniq))
    first[inv] = np.asarray(g2half)
    return first, inv


def band_features(model, psi: np.ndarray, gI: np.ndarray, g2sh: np.ndarray):
    """Features [n][k][3] of every band n and G shell k; bands with g_I = 0 get
    NaN rows (no samples)."""
    from . import roks
    nb = len(psi)
    X = np.full((nb, len(g2sh), NFEAT), np.nan)
    ekin = roks.band_kinetic(model, psi)
    for n in range(nb):
        Er = roks.teter_reference_energy(model, gI[n])
        gn = math.sqrt(max(roks.dot(gI[n], gI[n]), 0.0))
        if Er <= 0 or gn <= 0:
            continue
        X[n, :, 0] = np.log1p(g2sh / Er)
        X[n, :, 1] = math.log(ekin[n])
        X[n, :, 2] = math.log(gn)
    return X


def plain_teter_Kg(model, gI: np.ndarray) -> np.ndarray:
    from . import roks
    out = np.zeros_like(gI)
    for n in range(len(gI)):
        Er = roks.teter_reference_energy(model, gI[n])
        if Er <= 0:
            continue
        x = 0.5 * model.g2 / Er
        out[n] = -(2.0 / Er) * roks.teter_polynomial_ratio(x) * gI[n]
    return out


def normalized_scale(model, gI: np.ndarray, s_shell: np.ndarray, shell_of_G: np.ndarray):
    """Full-sphere factor [nb][npw] applied to K: the network's s of (band,
    G shell), times one constant for all bands chosen so that
    sum_n <s K g_n|g_n> equals the plain sum_n <K g_n|g_n> (the first-order
    energy change along the out-of-subspace direction is kept).  Rows of
    s_shell that hold NaN (bands without features) give s = 1 and take part
    in neither sum."""
    from . import roks
    out = np.ones((model.nb, model.npw))
    a = b = 0.0
    rows = []
    for n in range(model.nb):
        if np.isnan(s_shell[n]).any():
            continue
        Er = roks.teter_reference_energy(model, gI[n])
        if Er <= 0:
            continue
        w = (2.0 / Er) * roks.teter_polynomial_ratio(0.5 * model.g2 / Er) * np.abs(gI[n]) ** 2
        s = s_shell[n][shell_of_G]
        a += float(w.sum())
        b += float((s * w).sum())
        rows.append((n, s))
    r = a / b if a > 0 and b > 0 else 1.0
    for n, s in rows:
        out[n] = s * r
    return out


def aligned_correction(model, psi_i: np.ndarray, psi_inf: np.ndarray) -> np.ndarray:
    """delta_n = (1 - P_i) psi_inf'_n with psi_inf aligned to psi_i per shell."""
    from . import roks
    aligned = np.zeros_like(psi_inf)
    for X in range(model.nshell):
        sel = np.where(model.band_shell == X)[0]
        O = roks.overlap(psi_inf[sel], psi_i[sel])  # O_mn = <inf_m|i_n>
        Q, _ = scipy.linalg.polar(O)                # O = Q H, Q orthogonal
        aligned[sel] = Q.T @ psi_inf[sel]           # inf'_n = sum_m Q_mn inf_m
    return aligned - roks.overlap(psi_i, aligned).T @ psi_i


def moments(model, Kg: np.ndarray, delta: np.ndarray, shell_of_G: np.ndarray, nsh: int,
            ekin: np.ndarray):
    """alpha, beta, gamma [n][k]: <Kg|delta>_h, <Kg|Kg>_h, <delta|delta>_h
    restricted to G shell k (full-sphere sums), in the energy norm of band n:
    every G weighted by h_n(G) = |G|^2/2 + ekin[n]."""
    nb = len(Kg)
    a = np.zeros((nb, nsh))
    b = np.zeros((nb, nsh))
    c = np.zeros((nb, nsh))
    for n in range(nb):
        h = 0.5 * model.g2 + ekin[n]
        np.add.at(a[n], shell_of_G, h * np.real(np.conj(Kg[n]) * delta[n]))
        np.add.at(b[n], shell_of_G, h * np.abs(Kg[n]) ** 2)
        np.add.at(c[n], shell_of_G, h * np.abs(delta[n]) ** 2)
    return a, b, c


def band_loss(s: np.ndarray, alpha: np.ndarray, beta: np.ndarray, gamma: np.ndarray):
    """Mean over segments (rows, with B, C > 0) of 1 - A^2/(B C); also dL/ds."""
    A = (s * alpha).sum(axis=1)
    B = (s * s * beta).sum(axis=1)
    Cc = gamma.sum(axis=1)
    ok = (Cc > 0) & (B > 0)
    nb = max(int(ok.sum()), 1)
    L = np.where(ok, 1.0 - A * A / np.where(ok, B * Cc, 1.0), 0.0)
    dLds = np.zeros_like(s)
    r = np.where(ok, -2.0 * A / np.where(ok, B * B * Cc, 1.0), 0.0) / nb
    dLds = r[:, None] * (alpha * B[:, None] - A[:, None] * s * beta)
    return float(L[ok].mean()) if ok.any() else 0.0, dLds


def loss_and_grad(theta: np.ndarray, X: np.ndarray, alpha, beta, gamma):
    """Loss over segments: X [nseg][len][3] and moments [nseg][len]."""
    nb, nsh, _ = X.shape
    o, cache = forward(theta, X.reshape(-1, NFEAT))
    t = np.tanh(o)
    s = np.exp(2.0 * t).reshape(nb, nsh)
    L, dLds = band_loss(s, alpha, beta, gamma)
    do = (dLds.ravel() * s.ravel() * 2.0 * (1.0 - t * t))
    return L, backward(theta, cache, do)


def adam_step(theta, m, v, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
