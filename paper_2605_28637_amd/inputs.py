"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *describes* problems: cells, atoms, species parameters,
occupation tables and seeded random numbers.  It holds none of the method's
arithmetic (no sphere construction, no FFT, no potentials, no energies), so
both the CPU oracle and the GPU library can consume its output without
sharing any computational code.

Conventions (Hartree atomic units, lengths in bohr, energies in Ha):

* ``cell`` rows are the lattice vectors a1, a2, a3.
* A species is a dict ``{"A", "sigma", "proj": [(l, rp), ...], "D": [[...]]}``
  describing a Gaussian local well v(r) = -A exp(-r^2 / (2 sigma^2)) and
  separable Gaussian projectors of angular momentum l in {0, 1} and radius rp
  with the symmetric coupling matrix D over the radial channels; an optional
  symmetric ``"q"`` of the same shape gives the overlap coefficients of
  S = 1 + sum q |beta><beta| (absent: S = 1).
* ``occ[L][s][n]`` in {0, 1} is the occupation f_n^{sigma L} of band n in
  configuration L and spin s (0 = up, 1 = down); ``cL[L]`` the configuration
  weights.  For the singlet the configurations are the mixed-spin
  determinant (weight 2) and the triplet determinant (weight -1), the Ziegler
  sum rule of the paper's introduction (Eq. ziegler_sum).
* Random band coefficients are drawn per Miller triple from a counter-based
  generator (splitmix64 + Box-Muller), so any ordering of the plane-wave list
  receives the same value for the same G, and c(-G) = conj(c(G)).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177
HA_PER_EV = 1.0 / 27.211386

# ---------------------------------------------------------------------------
# counter-based random numbers keyed on (seed, band, Miller triple)
# ---------------------------------------------------------------------------
_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def _uniform(bits: np.ndarray) -> np.ndarray:
    """Map 64 random bits to a double in (0, 1)."""
    return ((bits >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def _canonical(miller: np.ndarray):
    """Representative of {G, -G}: l > 0, or l = 0 and k > 0, or l = k = 0, h >= 0."""
    h, k, l = miller[:, 0], miller[:, 1], miller[:, 2]
    canon = (l > 0) | ((l == 0) & (k > 0)) | ((l == 0) & (k == 0) & (h >= 0))
    rep = np.where(canon[:, None], miller, -miller)
    return rep, canon


def gaussian_pairs(seed: int, band: int, miller: np.ndarray) -> np.ndarray:
    """Complex standard normal xi1 + i xi2 keyed on (seed, band, canonical G).

    Returns values for the canonical representative, conjugated where the
    given triple is the non-canonical member of its +-G pair.
    """
    miller = np.asarray(miller, dtype=np.int64).reshape(-1, 3)
    rep, canon = _canonical(miller)
    key = (rep[:, 0] & 0xFFFF) | ((rep[:, 1] & 0xFFFF) << 16) | ((rep[:, 2] & 0xFFFF) << 32)
    base = _splitmix64(np.full(1, np.uint64(seed & 0xFFFFFFFFFFFFFFFF)))[0]
    base = _splitmix64(np.full(1, base ^ np.uint64(band)))[0]
    x = _splitmix64(key.astype(np.uint64) ^ base)
    u1 = _uniform(_splitmix64(x ^ np.uint64(0x1234567)))
    u2 = _uniform(_splitmix64(x ^ np.uint64(0x89ABCDEF)))
    r = np.sqrt(-2.0 * np.log(u1))
    xi = r * np.cos(2 * np.pi * u2) + 1j * r * np.sin(2 * np.pi * u2)
    xi = np.where(canon, xi, np.conj(xi))
    zero = (miller == 0).all(axis=1)
    xi[zero] = xi[zero].real
    return xi


def reciprocal(cell: np.ndarray) -> np.ndarray:
    """Rows b1, b2, b3 with a_i . b_j = 2 pi delta_ij."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(cell, dtype=np.float64)).T


def random_coefficients(miller: Sequence, cell: np.ndarray, nbands: int, seed: int) -> np.ndarray:
    """Seeded start vectors c_n(G) = (xi1 + i xi2) / (1 + |G|^2), c_n(0) real.

    ``miller`` may be any list of triples (a half-space list or the full
    sphere); the value for a triple does not depend on its position.
    Returns a complex array [nbands][len(miller)] (not orthonormalised).
    """
    miller = np.asarray(miller, dtype=np.int64).reshape(-1, 3)
    g = miller.astype(np.float64) @ reciprocal(cell)
    damp = 1.0 / (1.0 + (g * g).sum(axis=1))
    out = np.empty((nbands, len(miller)), dtype=np.complex128)
    for n in range(nbands):
        out[n] = gaussian_pairs(seed, n, miller) * damp
    return out


# ---------------------------------------------------------------------------
# occupation tables (the configurations of the paper's Fig. 1A / Sec. II A)
# ---------------------------------------------------------------------------
def roks_occupations(n_closed: int, n_virtual: int):
    """Mixed-spin (a up, b down; weight 2) and triplet (a up, b up; weight -1).

    Band order: closed, a, b, virtual.  Returns (occ[2][2][nb], cL[2]).
    """
    nb = n_closed + 2 + n_virtual
    occ = np.zeros((2, 2, nb), dtype=np.uint8)
    occ[:, :, :n_closed] = 1
    a, b = n_closed, n_closed + 1
    occ[0, 0, a] = 1  # M: a up
    occ[0, 1, b] = 1  # M: b down
    occ[1, 0, a] = 1  # T: a up
    occ[1, 0, b] = 1  # T: b up
    return occ, np.array([2.0, -1.0])


def ground_state_occupations(n_doubly: int, nb: int):
    """Closed-shell ground state: one configuration, weight 1."""
    occ = np.zeros((1, 2, nb), dtype=np.uint8)
    occ[0, :, :n_doubly] = 1
    return occ, np.array([1.0])


def triplet_occupations(n_closed: int, n_virtual: int):
    """High-spin triplet (a up, b up) as a single configuration, weight 1."""
    nb = n_closed + 2 + n_virtual
    occ = np.zeros((1, 2, nb), dtype=np.uint8)
    occ[0, :, :n_closed] = 1
    occ[0, 0, n_closed] = 1
    occ[0, 0, n_closed + 1] = 1
    return occ, np.array([1.0])


# ---------------------------------------------------------------------------
# species and geometries
# ---------------------------------------------------------------------------
def _species(A: float, sigma: float, proj: List[tuple], Ddiag: List[float]) -> Dict:
    D = np.diag(np.asarray(Ddiag, dtype=np.float64))
    return {"A": float(A), "sigma": float(sigma), "proj": [(int(l), float(rp)) for l, rp in proj],
            "D": D}


def _min_image_ok(pos: np.ndarray, p: np.ndarray, L: float, dmin: float) -> bool:
    if len(pos) == 0:
        return True
    d = pos - p
    d -= L * np.round(d / L)
    return bool((np.sqrt((d * d).sum(axis=1)) >= dmin).all())


def _random_positions(rng: np.random.Generator, natoms: int, lo: float, hi: float, L: float,
                      dmin: float) -> np.ndarray:
    pos = np.zeros((0, 3))
    tries = 0
    while len(pos) < natoms:
        p = rng.uniform(lo, hi, size=3)
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place atoms")
        if _min_image_ok(pos, p, L, dmin):
            pos = np.vstack([pos, p])
    return pos


def _system(name, cell, ecut, grid, species, species_of_atom, pos, occ, cL, xc="pw92", seed=0,
            n_closed=0):
    nb = occ.shape[2]
    return {
        "n_closed": int(n_closed),
        "name": name,
        "cell": np.asarray(cell, dtype=np.float64),
        "ecut": float(ecut),
        "grid": tuple(int(g) for g in grid),
        "species": species,
        "species_of_atom": np.asarray(species_of_atom, dtype=np.int32),
        "pos": np.asarray(pos, dtype=np.float64).reshape(-1, 3),
        "nbands": int(nb),
        "occ": np.asarray(occ, dtype=np.uint8),
        "cL": np.asarray(cL, dtype=np.float64),
        "xc": xc,
        "seed": int(seed),
    }


def grid_rule_ecut(L: float, N: int) -> float:
    """Cutoff whose sphere radius is a quarter of the grid: G_cut = pi N / (2 L)."""
    g = math.pi * N / (2.0 * L)
    return 0.5 * g * g


def tiny_cell(seed: int = 1000, ecut: float = 7.5, xc: str = "pw92", n_closed: int = 4,
              configuration: str = "roks") -> Dict:
    """Cubic 8 bohr box, 16^3 grid, 2 atoms (Gaussian well depth 2 Ha, width
    0.8 bohr, one s projector each, D = +1 Ha), 4 closed + 2 open bands.

    ``ecut`` = 7.5 Ha gives about 500 plane waves (485 in the full sphere).
    """
    L = 8.0
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = _random_positions(rng, 2, 0.0, L, L, 2.2)
    sp = [_species(2.0, 0.8, [(0, 0.8)], [1.0])]
    occ, cL = _occupations(configuration, n_closed, 0)
    return _system("tiny", np.eye(3) * L, ecut, (16, 16, 16), sp, [0, 0], pos, occ, cL, xc, seed,
                   n_closed)


def dimer(seed: int = 1100, d: float = 1.8, configuration: str = "roks", xc: str = "pw92") -> Dict:
    """Two unlike Gaussian-well atoms (depths 2.5 / 1.6 Ha, widths 0.8 /
    0.7 bohr, one s projector each) d bohr apart, slightly off axis, in the
    8 bohr box of the tiny cell (16^3 grid, 7.5 Ha): 2 closed + 2 open + 1
    virtual bands.  The geometry-relaxation workload: with the pair
    repulsion 1.0 exp(-r / 0.4) Ha its ground-state bond is about 1.4 bohr."""
    L = 8.0
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = np.array([[4.0 - d / 2, 4.0, 4.0], [4.0 + d / 2, 4.1, 3.9]]) + rng.normal(0, 0.02, (2, 3))
    sp = [_species(2.5, 0.8, [(0, 0.8)], [1.0]), _species(1.6, 0.7, [(0, 0.7)], [0.8])]
    occ, cL = _occupations(configuration, 2, 1)
    return _system("dimer", np.eye(3) * L, 7.5, (16, 16, 16), sp, [0, 1], pos, occ, cL, xc, seed, 2)


def _occupations(configuration: str, n_closed: int, n_virtual: int):
    if configuration == "roks":
        return roks_occupations(n_closed, n_virtual)
    if configuration == "gs":
        nb = n_closed + 2 + n_virtual
        return ground_state_occupations(n_closed + 1, nb)
    if configuration == "triplet":
        return triplet_occupations(n_closed, n_virtual)
    raise ValueError(configuration)


MOLECULE_SPECIES = [
    # species X: s (rp 0.6, D +1.0) and p (rp 0.7, D -0.3)
    _species(3.0, 0.9, [(0, 0.6), (1, 0.7)], [1.0, -0.3]),
    # species Y: s (rp 1.0, D +0.5) and p (rp 1.1, D -0.2)
    _species(2.5, 0.8, [(0, 1.0), (1, 1.1)], [0.5, -0.2]),
]


def molecule_box(seed: int = 2000, natoms: int = 20, nb: int = 40, N: int = 64, L: float = 24.0,
                 xc: str = "pw92", configuration: str = "roks") -> Dict:
    """Molecule-in-box: cubic box L, N^3 grid at the grid-rule cutoff, atoms in
    the central half-width cube (min separation 2.2 bohr), s + p projectors
    (4 per atom), nb bands = (nb - 4) closed + 2 open + 2 virtual."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = 0.25 * L, 0.75 * L
    pos = _random_positions(rng, natoms, lo, hi, L, 2.2)
    spa = np.arange(natoms) % 2
    occ, cL = _occupations(configuration, nb - 4, 2)
    return _system("molecule", np.eye(3) * L, grid_rule_ecut(L, N), (N, N, N), MOLECULE_SPECIES,
                   spa, pos, occ, cL, xc, seed, nb - 4)


OXIDE_SPECIES = [
    # cation: A 1 Ha, sigma 0.6; 2 s + 2 p channels (8 projectors)
    _species(1.0, 0.6, [(0, 0.6), (0, 1.0), (1, 0.7), (1, 1.1)], [1.0, 0.5, -0.3, -0.2]),
    # anion: A 2 Ha, sigma 0.8
    _species(2.0, 0.8, [(0, 0.6), (0, 1.0), (1, 0.7), (1, 1.1)], [1.0, 0.5, -0.3, -0.2]),
]


def oxide_vacancy(seed: int = 3000, a: float = 8.0, reps: int = 3, N: int = 96, nb: int = 432,
                  xc: str = "pw92", configuration: str = "roks", displacement: float = 0.02) -> Dict:
    """Rocksalt reps^3 conventional supercell (lattice constant a) with the anion
    nearest the centre removed, seeded Gaussian displacements, 8 projectors
    per atom, nb bands = (nb - 4) closed + 2 open + 2 virtual."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = a * reps
    cat = np.array([[0, 0, 0], [.5, .5, 0], [.5, 0, .5], [0, .5, .5]])
    ani = np.array([[.5, 0, 0], [0, .5, 0], [0, 0, .5], [.5, .5, .5]])
    cp, ap = [], []
    for i in range(reps):
        for j in range(reps):
            for k in range(reps):
                o = np.array([i, j, k], dtype=float)
                cp.extend((o + cat) * a)
                ap.extend((o + ani) * a)
    cp, ap = np.array(cp), np.array(ap)
    c = np.full(3, L / 2)
    far = np.argmin(((ap - c) ** 2).sum(axis=1))
    ap = np.delete(ap, far, axis=0)
    pos = np.vstack([cp, ap]) + rng.normal(0.0, displacement, size=(len(cp) + len(ap), 3))
    spa = np.array([0] * len(cp) + [1] * len(ap))
    occ, cL = _occupations(configuration, nb - 4, 2)
    return _system("oxide", np.eye(3) * L, grid_rule_ecut(L, N), (N, N, N), OXIDE_SPECIES, spa,
                   pos, occ, cL, xc, seed, nb - 4)


BATCH_GRIDS = (40, 48, 50, 54, 60, 64, 72, 80)


def batch_systems(seed: int = 4000, count: int = 32, xc: str = "pw92") -> List[Dict]:
    """Uneven molecule-in-box systems: natoms ~ U{10..60}, nb = 2 natoms, grid
    the allowed size nearest 40 + 0.8 (natoms - 10), box L = 24 N / 64 (so the
    grid-rule cutoff stays 8.77 Ha), atoms in the central 0.6 L cube."""
    out = []
    for s in range(count):
        rng = np.random.Generator(np.random.PCG64(seed + s))
        natoms = int(rng.integers(10, 61))
        nb = 2 * natoms
        target = 40 + 0.8 * (natoms - 10)
        N = min(BATCH_GRIDS, key=lambda n: (abs(n - target), n))
        L = 24.0 * N / 64.0
        pos = _random_positions(rng, natoms, 0.2 * L, 0.8 * L, L, 2.2)
        occ, cL = roks_occupations(nb - 4, 2)
        out.append(_system("batch%02d" % s, np.eye(3) * L, grid_rule_ecut(L, N), (N, N, N),
                           MOLECULE_SPECIES, np.arange(natoms) % 2, pos, occ, cL, xc, seed + s,
                           nb - 4))
    return out


def with_overlap(system: Dict, scale: float = 0.5) -> Dict:
    """Copy of ``system`` whose species carry overlap coefficients q (the
    PAW-like S = 1 + sum q |beta><beta|): q = scale * diag(1, 0.6, 0.4, 0.3)
    over the radial channels, plus scale / 5 between the first two channels
    when both have l = 0."""
    out = dict(system)
    spec = []
    for sp in system["species"]:
        n = len(sp["proj"])
        q = np.diag(scale * np.array([1.0, 0.6, 0.4, 0.3][:n]))
        if n >= 2 and sp["proj"][0][0] == 0 and sp["proj"][1][0] == 0:
            q[0, 1] = q[1, 0] = 0.2 * scale
        t = dict(sp)
        t["q"] = q
        spec.append(t)
    out["species"] = spec
    return out


def with_configuration(system: Dict, configuration: str) -> Dict:
    """Copy of ``system`` with the occupation table replaced (same bands).

    ``configuration`` is "roks" (mixed + triplet, weights 2, -1), "gs" (closed
    shell with n_closed + 1 doubly occupied bands) or "triplet"."""
    nb = system["nbands"]
    n_closed = system["n_closed"]
    occ, cL = _occupations(configuration, n_closed, nb - n_closed - 2)
    out = dict(system)
    out["occ"], out["cL"] = occ, cL
    return out
