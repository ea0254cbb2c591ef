"""ctypes binding of libroks.so (include/roks.h): argument marshalling only.

Every numerical step runs in the gfx950 library; this module converts the
seeded problem descriptions of ``inputs`` to the C structs, copies NumPy
arrays in and out, and raises on error statuses.  If the shared library is
missing the import of ``lib()`` raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libroks.so")

FP64, FP32, FP32_BF16X3 = 0, 1, 2
XC = {"pw92": 0, "x": 1, "pbe": 2}
FLAG_SUPPRESS_OPEN_COUPLING = 1
FLAG_CANONICALIZE = 2
FLAG_WEIGHT_PRECOND = 4
FLAG_AUTOTUNE = 8
FLAG_GRAPH = 16

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_SHAPE", 3: "ERR_HIP", 4: "ERR_OOM", 5: "ERR_NOT_PD",
          6: "ERR_LINESEARCH", 7: "ERR_NAN", 8: "ERR_STATE"}


class RoksError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


class Proj(C.Structure):
    _fields_ = [("l", C.c_int32), ("rp", C.c_double)]


class Species(C.Structure):
    _fields_ = [("A", C.c_double), ("sigma", C.c_double), ("nproj", C.c_int32),
                ("proj", C.POINTER(Proj)), ("D", C.POINTER(C.c_double)),
                ("q", C.POINTER(C.c_double))]


class System(C.Structure):
    _fields_ = [("cell", C.c_double * 9), ("ecut", C.c_double), ("grid", C.c_int32 * 3),
                ("natoms", C.c_int32), ("species", C.POINTER(C.c_int32)),
                ("pos", C.POINTER(C.c_double)), ("nspecies", C.c_int32),
                ("spec", C.POINTER(Species)), ("nbands", C.c_int32), ("nconfig", C.c_int32),
                ("occ", C.POINTER(C.c_uint8)), ("cL", C.POINTER(C.c_double)), ("xc", C.c_int32),
                ("precision", C.c_int32), ("flags", C.c_uint32), ("exx", C.c_double)]


class Energies(C.Structure):
    _fields_ = [("E", C.c_double), ("E_L", C.c_double * 2), ("kinetic", C.c_double * 2),
                ("nonlocal", C.c_double * 2), ("external", C.c_double * 2),
                ("hartree", C.c_double * 2), ("xc", C.c_double * 2)]

    def as_dict(self, nconf: int) -> Dict:
        d = {"E": self.E}
        for k in ("E_L", "kinetic", "nonlocal", "external", "hartree", "xc"):
            d[k] = np.array(list(getattr(self, k))[:nconf])
        return d


class StepInfo(C.Structure):
    _fields_ = [("E0", C.c_double), ("E1", C.c_double), ("delta", C.c_double),
                ("beta", C.c_double), ("dE0", C.c_double), ("norm_gI", C.c_double),
                ("max_Rab", C.c_double), ("restarted", C.c_int32), ("stalled", C.c_int32),
                ("evaluations", C.c_int32), ("iteration", C.c_int32), ("learned", C.c_int32),
                ("fallback", C.c_int32)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


DIIS_MAX_HISTORY = 8


class DiisParams(C.Structure):
    _fields_ = [("history", C.c_int32), ("step", C.c_double), ("asymmetric", C.c_int32)]


class DiisInfo(C.Structure):
    _fields_ = [("E", C.c_double), ("rnorm2", C.c_double), ("open_coupling", C.c_double),
                ("used", C.c_int32), ("coeffs", C.c_double * DIIS_MAX_HISTORY)]

    def as_dict(self) -> Dict:
        return {"E": self.E, "rnorm2": self.rnorm2, "open_coupling": self.open_coupling,
                "used": self.used, "coeffs": list(self.coeffs[: self.used])}


class RelaxParams(C.Structure):
    _fields_ = [("fmax", C.c_double), ("maxsteps", C.c_int32), ("scf_tol", C.c_double),
                ("scf_maxiter", C.c_int32), ("scf_restart", C.c_int32), ("max_step", C.c_double),
                ("h0", C.c_double), ("pair_B", C.c_double), ("pair_rho", C.c_double)]


RELAX_DEFAULTS = {"fmax": 1e-4, "maxsteps": 60, "scf_tol": 1e-11, "scf_maxiter": 800,
                  "scf_restart": 20, "max_step": 0.2, "h0": 1.0, "pair_B": 1.0, "pair_rho": 0.4}


def relax_params(**kw) -> RelaxParams:
    v = dict(RELAX_DEFAULTS)
    for k in kw:
        if k not in v:
            raise KeyError(k)
    v.update(kw)
    return RelaxParams(**v)


class RelaxInfo(C.Structure):
    _fields_ = [("E", C.c_double), ("fmax", C.c_double), ("steps", C.c_int32),
                ("scf_iterations", C.c_int32), ("converged", C.c_int32)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class FcResult(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("E_gs_at_gs", "E_ex_at_gs", "E_ex_at_ex", "E_gs_at_ex",
                                          "E_abs", "E_FC_ex", "E_FC_gs", "E_emi", "dQ")] + \
               [("gs_steps", C.c_int32), ("ex_steps", C.c_int32), ("converged", C.c_int32)]

    def as_dict(self) -> Dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None

# name -> (restype, argtypes)
_P = C.c_void_p
_SIGS = {
    "roks_create": (C.c_int, [C.POINTER(System), _P, C.POINTER(_P)]),
    "roks_destroy": (C.c_int, [_P]),
    "roks_last_error": (C.c_char_p, [_P]),
    "roks_version": (C.c_char_p, []),
    "roks_grid_rule": (C.c_int, [C.POINTER(C.c_double), C.c_double, C.POINTER(C.c_int32)]),
    "roks_sizes": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32)]),
    "roks_gvectors": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "roks_set_coeffs": (C.c_int, [_P, C.POINTER(C.c_double), C.c_int32]),
    "roks_get_coeffs": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "roks_set_coeffs_d": (C.c_int, [_P, _P, C.c_int32]),
    "roks_get_coeffs_d": (C.c_int, [_P, _P]),
    "roks_set_positions": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "roks_apply_h": (C.c_int, [_P, C.POINTER(C.c_double), C.c_uint32, C.POINTER(C.c_double)]),
    "roks_apply_h_d": (C.c_int, [_P, _P, C.c_uint32, _P]),
    "roks_apply_h_noalloc_d": (C.c_int, [_P, _P, C.c_uint32, _P]),
    "roks_energy_gradient": (C.c_int, [_P, C.POINTER(Energies), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]),
    "roks_subspace": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_double)]),
    "roks_pcg_step": (C.c_int, [_P, C.POINTER(StepInfo)]),
    "roks_graph_steps": (C.c_int, [_P, C.c_int32, C.POINTER(StepInfo), C.POINTER(C.c_int32)]),
    "roks_reset_cg": (C.c_int, [_P]),
    "roks_diis_step": (C.c_int, [_P, C.POINTER(DiisParams), C.POINTER(DiisInfo)]),
    "roks_diis_solve": (C.c_int, [_P, C.POINTER(DiisParams), C.c_double, C.c_int32,
                                  C.POINTER(DiisInfo), C.POINTER(C.c_int32)]),
    "roks_diis_reset": (C.c_int, [_P]),
    "roks_relax": (C.c_int, [_P, C.POINTER(RelaxParams), C.POINTER(RelaxInfo)]),
    "roks_get_positions": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "roks_franck_condon": (C.c_int, [_P, _P, C.POINTER(RelaxParams), C.POINTER(C.c_double),
                                     C.POINTER(FcResult)]),
    "roks_set_restart": (C.c_int, [_P, C.c_int32]),
    "roks_set_precision": (C.c_int, [_P, C.c_int32]),
    "roks_solve": (C.c_int, [_P, C.c_double, C.c_int32, C.POINTER(StepInfo), C.POINTER(C.c_int32)]),
    "roks_forces": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "roks_synchronize": (C.c_int, [_P]),
    "roks_timing_enable": (C.c_int, [_P, C.c_int32]),
    "roks_timing_only": (C.c_int, [_P, C.c_char_p]),
    "roks_timing_read": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "roks_mlp_create": (C.c_int, [C.POINTER(C.c_float), C.c_uint64, _P, C.POINTER(_P)]),
    "roks_mlp_destroy": (C.c_int, [_P]),
    "roks_mlp_last_error": (C.c_char_p, [_P]),
    "roks_mlp_set_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "roks_mlp_get_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "roks_mlp_forward": (C.c_int, [_P, C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_float)]),
    "roks_mlp_num_samples": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "roks_mlp_get_samples": (C.c_int, [_P, C.POINTER(C.c_float), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32)]),
    "roks_mlp_clear_samples": (C.c_int, [_P]),
    "roks_mlp_loss_grad": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_float)]),
    "roks_mlp_train": (C.c_int, [_P, C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "roks_record": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "roks_mlp_collect": (C.c_int, [_P, _P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "roks_set_mlp": (C.c_int, [_P, _P]),
    "roks_batch_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, C.POINTER(_P)]),
    "roks_batch_destroy": (C.c_int, [_P]),
    "roks_batch_solve": (C.c_int, [_P, C.c_double, C.c_int32, C.c_double, C.POINTER(C.c_int),
                                   C.POINTER(C.c_int32), C.POINTER(StepInfo)]),
    "roks_batch_steps": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int)]),
    "roks_batch_graph_steps": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int), C.POINTER(C.c_int32)]),
}

MLP_PARAMS = 4481


def lib() -> C.CDLL:
    """Load libroks.so (built in-tree); raises if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libroks.so is not built: run python -m paper_2605_28637_amd.build")
        L = C.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def grid_rule(cell: np.ndarray, ecut: float) -> tuple:
    """The grid roks_create takes for grid = (0, 0, 0) (host only)."""
    c = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(3, 3))
    g = (C.c_int32 * 3)()
    st = lib().roks_grid_rule(_dptr(c), float(ecut), g)
    if st != 0:
        raise RoksError(st, "roks_grid_rule failed")
    return tuple(int(v) for v in g)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _packed(c: np.ndarray) -> np.ndarray:
    """complex [..., npw] -> contiguous float64 [..., npw, 2]"""
    c = np.asarray(c)
    out = np.empty(c.shape + (2,), dtype=np.float64)
    out[..., 0] = c.real
    out[..., 1] = c.imag
    return out


def _unpacked(a: np.ndarray) -> np.ndarray:
    return a[..., 0] + 1j * a[..., 1]


class _SystemBuffers:
    """Keeps the arrays a System struct points to alive."""

    def __init__(self, system: Dict, precision: int, flags: int):
        s = system
        self.cell = np.ascontiguousarray(s["cell"], dtype=np.float64).reshape(9)
        self.pos = np.ascontiguousarray(s["pos"], dtype=np.float64).reshape(-1)
        self.spa = np.ascontiguousarray(s["species_of_atom"], dtype=np.int32)
        self.occ = np.ascontiguousarray(s["occ"], dtype=np.uint8)
        self.cL = np.ascontiguousarray(s["cL"], dtype=np.float64)
        nspec = len(s["species"])
        self.specs = (Species * max(1, nspec))()
        self.keep = []
        for i, sp in enumerate(s["species"]):
            npj = len(sp["proj"])
            pj = (Proj * max(1, npj))()
            for j, (l, rp) in enumerate(sp["proj"]):
                pj[j].l, pj[j].rp = int(l), float(rp)
            D = np.ascontiguousarray(np.asarray(sp["D"], dtype=np.float64).reshape(-1))
            if D.size == 0:
                D = np.zeros(1)
            self.keep += [pj, D]
            self.specs[i].A = float(sp["A"])
            self.specs[i].sigma = float(sp["sigma"])
            self.specs[i].nproj = npj
            self.specs[i].proj = C.cast(pj, C.POINTER(Proj))
            self.specs[i].D = _dptr(D)
            # overlap coefficients (absent: NULL, S = 1)
            if sp.get("q") is not None and npj > 0:
                q = np.ascontiguousarray(np.asarray(sp["q"], dtype=np.float64).reshape(-1))
                self.keep.append(q)
                self.specs[i].q = _dptr(q)
            else:
                self.specs[i].q = None
        st = System()
        for i in range(9):
            st.cell[i] = self.cell[i]
        st.ecut = float(s["ecut"])
        for d in range(3):
            st.grid[d] = int(s["grid"][d])
        st.natoms = len(self.spa)
        st.species = self.spa.ctypes.data_as(C.POINTER(C.c_int32))
        st.pos = _dptr(self.pos)
        st.nspecies = nspec
        st.spec = C.cast(self.specs, C.POINTER(Species))
        st.nbands = int(s["nbands"])
        st.nconfig = int(self.occ.shape[0])
        st.occ = self.occ.ctypes.data_as(C.POINTER(C.c_uint8))
        st.cL = _dptr(self.cL)
        st.xc = XC[s.get("xc", "pw92")]
        st.exx = float(s.get("exx", 0.0))
        st.precision = precision
        st.flags = flags
        self.struct = st


class Roks:
    """One ROKS problem on the GPU (a roks_ctx)."""

    def __init__(self, system: Dict, precision: int = FP64, flags: int = 0, stream: Optional[int] = None):
        self._L = lib()
        self.system = system
        self._buf = _SystemBuffers(system, precision, flags)
        h = _P()
        st = self._L.roks_create(C.byref(self._buf.struct), _P(stream or 0), C.byref(h))
        if st != 0:
            raise RoksError(st, self._L.roks_last_error(None).decode())
        self._h = h
        npw, nproj, nb = C.c_int32(), C.c_int32(), C.c_int32()
        grid = (C.c_int32 * 3)()
        self._check(self._L.roks_sizes(self._h, C.byref(npw), grid, C.byref(nproj), C.byref(nb)))
        self.npw, self.nproj, self.nb = npw.value, nproj.value, nb.value
        self.grid = tuple(grid)
        self.nconf = int(np.asarray(system["occ"]).shape[0])
        self.natoms = len(system["species_of_atom"])

    # -- plumbing -----------------------------------------------------------
    def _check(self, status: int):
        if status != 0:
            raise RoksError(status, self._L.roks_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.roks_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- ABI ------------------------------------------------------------------
    def miller(self) -> np.ndarray:
        m = np.empty((self.npw, 3), dtype=np.int32)
        self._check(self._L.roks_gvectors(self._h, m.ctypes.data_as(C.POINTER(C.c_int32))))
        return m

    def set_coeffs(self, c: np.ndarray, orthonormalize: bool = True):
        a = _packed(np.asarray(c).reshape(self.nb, self.npw))
        self._check(self._L.roks_set_coeffs(self._h, _dptr(a), 1 if orthonormalize else 0))

    def get_coeffs(self) -> np.ndarray:
        a = np.empty((self.nb, self.npw, 2))
        self._check(self._L.roks_get_coeffs(self._h, _dptr(a)))
        return _unpacked(a)

    def set_coeffs_d(self, ptr: int, orthonormalize: bool = True):
        """Orbitals from device memory [nb][npw][2] FP64 (e.g. a torch data_ptr)."""
        self._check(self._L.roks_set_coeffs_d(self._h, _P(ptr), 1 if orthonormalize else 0))

    def get_coeffs_d(self, ptr: int):
        self._check(self._L.roks_get_coeffs_d(self._h, _P(ptr)))

    def set_positions(self, pos: np.ndarray):
        p = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1)
        self._check(self._L.roks_set_positions(self._h, _dptr(p)))

    def apply_h(self, c: Optional[np.ndarray] = None, mask: int = 0) -> np.ndarray:
        nch = bin(mask).count("1") if mask else 1
        out = np.empty((nch, self.nb, self.npw, 2))
        cin = None
        if c is not None:
            cin = _packed(np.asarray(c).reshape(self.nb, self.npw))
        self._check(self._L.roks_apply_h(self._h, _dptr(cin) if cin is not None else None, mask,
                                         _dptr(out)))
        r = _unpacked(out)
        return r[0] if mask == 0 else r

    def energy_gradient(self):
        e = Energies()
        g = np.empty((self.nb, self.npw, 2))
        th = np.empty((self.nb, self.nb))
        self._check(self._L.roks_energy_gradient(self._h, C.byref(e), _dptr(g), _dptr(th)))
        return e.as_dict(self.nconf), _unpacked(g), th

    def subspace(self):
        R, k, A = (np.empty((self.nb, self.nb)) for _ in range(3))
        self._check(self._L.roks_subspace(self._h, _dptr(R), _dptr(k), _dptr(A)))
        return R, k, A

    def pcg_step(self) -> Dict:
        info = StepInfo()
        self._check(self._L.roks_pcg_step(self._h, C.byref(info)))
        return info.as_dict()

    def graph_steps(self, k: int):
        """k device-decided CG iterations replayed from one captured graph:
        (the leading accepted count, the k step records)."""
        info = (StepInfo * k)()
        acc = C.c_int32()
        self._check(self._L.roks_graph_steps(self._h, k, info, C.byref(acc)))
        return acc.value, [info[i].as_dict() for i in range(k)]

    def reset_cg(self):
        self._check(self._L.roks_reset_cg(self._h))

    def set_restart(self, period: int):
        self._check(self._L.roks_set_restart(self._h, period))

    def set_precision(self, precision: int):
        self._check(self._L.roks_set_precision(self._h, precision))

    def solve(self, tol: float = 1e-6, maxiter: int = 500):
        info = StepInfo()
        it = C.c_int32()
        self._check(self._L.roks_solve(self._h, tol, maxiter, C.byref(info), C.byref(it)))
        return info.as_dict(), it.value

    def diis_step(self, history: int = 6, step: float = 0.3, asymmetric: bool = False) -> Dict:
        p = DiisParams(history, step, 1 if asymmetric else 0)
        info = DiisInfo()
        self._check(self._L.roks_diis_step(self._h, C.byref(p), C.byref(info)))
        return info.as_dict()

    def diis_solve(self, tol: float = 1e-6, maxiter: int = 500, history: int = 6, step: float = 0.3,
                   asymmetric: bool = False):
        p = DiisParams(history, step, 1 if asymmetric else 0)
        info = DiisInfo()
        it = C.c_int32()
        self._check(self._L.roks_diis_solve(self._h, C.byref(p), tol, maxiter, C.byref(info),
                                            C.byref(it)))
        return info.as_dict(), it.value

    def diis_reset(self):
        self._check(self._L.roks_diis_reset(self._h))

    def relax(self, **params) -> Dict:
        p = relax_params(**params)
        info = RelaxInfo()
        self._check(self._L.roks_relax(self._h, C.byref(p), C.byref(info)))
        return info.as_dict()

    def get_positions(self) -> np.ndarray:
        pos = np.empty((max(1, self.natoms), 3))
        self._check(self._L.roks_get_positions(self._h, _dptr(pos)))
        return pos[: self.natoms]

    def forces(self) -> np.ndarray:
        f = np.empty((max(1, self.natoms), 3))
        self._check(self._L.roks_forces(self._h, _dptr(f)))
        return f[: self.natoms]

    def synchronize(self):
        self._check(self._L.roks_synchronize(self._h))

    def record(self, max_records: int, stride: int = 1):
        self._check(self._L.roks_record(self._h, max_records, stride))

    def set_mlp(self, mlp: Optional["Mlp"]):
        self._mlp = mlp  # keep the network alive while attached
        self._check(self._L.roks_set_mlp(self._h, mlp.handle if mlp is not None else None))

    def timing_enable(self, on: bool = True):
        self._check(self._L.roks_timing_enable(self._h, 1 if on else 0))

    def timing_only(self, kernel: Optional[str]):
        self._check(self._L.roks_timing_only(self._h, kernel.encode() if kernel else None))

    def timing_read(self, kernel: str) -> Dict:
        ms, n, by, fl = C.c_double(), C.c_int32(), C.c_double(), C.c_double()
        self._check(self._L.roks_timing_read(self._h, kernel.encode(), C.byref(ms), C.byref(n),
                                             C.byref(by), C.byref(fl)))
        return {"ms_total": ms.value, "launches": n.value, "bytes": by.value, "flops": fl.value}

    # device-pointer variants (torch tensors or raw ints)
    def apply_h_d(self, c_in_ptr: Optional[int], mask: int, out_ptr: int):
        self._check(self._L.roks_apply_h_d(self._h, _P(c_in_ptr or 0), mask, _P(out_ptr)))

    def apply_h_noalloc_d(self, c_in_ptr: Optional[int], mask: int, out_ptr: int):
        self._check(self._L.roks_apply_h_noalloc_d(self._h, _P(c_in_ptr or 0), mask, _P(out_ptr)))


def franck_condon(gs: "Roks", ex: "Roks", masses, **params) -> Dict:
    """The Franck-Condon cycle of Sec. IV B on two contexts (roks_franck_condon)."""
    p = relax_params(**params)
    out = FcResult()
    m = np.ascontiguousarray(masses, dtype=np.float64)
    gs._check(gs._L.roks_franck_condon(gs._h, ex._h, C.byref(p), _dptr(m), C.byref(out)))
    return out.as_dict()


class Mlp:
    """The learned rescaling network (a roks_mlp)."""

    def __init__(self, theta: Optional[np.ndarray] = None, seed: int = 0, stream: Optional[int] = None):
        self._L = lib()
        h = _P()
        t = None
        if theta is not None:
            t = np.ascontiguousarray(theta, dtype=np.float32)
            assert t.size == MLP_PARAMS
        st = self._L.roks_mlp_create(_fptr(t) if t is not None else None, seed, _P(stream or 0),
                                     C.byref(h))
        if st != 0:
            raise RoksError(st, self._L.roks_mlp_last_error(None).decode())
        self._h = h

    @property
    def handle(self):
        return self._h

    def _check(self, status: int):
        if status != 0:
            raise RoksError(status, self._L.roks_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.roks_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta: np.ndarray):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        assert t.size == MLP_PARAMS
        self._check(self._L.roks_mlp_set_params(self._h, _fptr(t)))

    def get_params(self) -> np.ndarray:
        t = np.empty(MLP_PARAMS, dtype=np.float32)
        self._check(self._L.roks_mlp_get_params(self._h, _fptr(t)))
        return t

    def forward(self, x: np.ndarray) -> np.ndarray:
        xx = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)
        o = np.empty(len(xx), dtype=np.float32)
        self._check(self._L.roks_mlp_forward(self._h, _fptr(xx), len(xx), _fptr(o)))
        return o

    def num_samples(self):
        S, nb = C.c_int64(), C.c_int32()
        self._check(self._L.roks_mlp_num_samples(self._h, C.byref(S), C.byref(nb)))
        return S.value, nb.value

    def get_samples(self):
        """(x [S][3] float32, moments [3][S] (alpha, beta, gamma), band offsets)"""
        S, nb = self.num_samples()
        x = np.empty((max(S, 1), 3), dtype=np.float32)
        mom = np.empty((3, max(S, 1)))
        off = np.empty(nb + 1, dtype=np.int32)
        self._check(self._L.roks_mlp_get_samples(self._h, _fptr(x), _dptr(mom),
                                                 off.ctypes.data_as(C.POINTER(C.c_int32))))
        return x[:S], mom[:, :S], off

    def clear_samples(self):
        self._check(self._L.roks_mlp_clear_samples(self._h))

    def loss_grad(self):
        loss = C.c_double()
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        self._check(self._L.roks_mlp_loss_grad(self._h, C.byref(loss), _fptr(g)))
        return loss.value, g

    def train(self, steps: int, lr: float) -> np.ndarray:
        hist = np.empty(max(steps, 1))
        self._check(self._L.roks_mlp_train(self._h, steps, lr, _dptr(hist)))
        return hist[:steps]

    def collect(self, roks: Roks):
        used, skipped = C.c_int32(), C.c_int32()
        self._check(self._L.roks_mlp_collect(self._h, roks.handle, C.byref(used), C.byref(skipped)))
        return used.value, skipped.value


class Batch:
    """Independent contexts solved side by side (a roks_batch): a work queue,
    longest system first, drained by `workers` host threads (four by
    default, one per hardware queue of the device)."""

    def __init__(self, systems, workers: int = 4):
        self._L = lib()
        self.systems = list(systems)
        n = len(self.systems)
        arr = (_P * n)(*[r.handle for r in self.systems])
        h = _P()
        st = self._L.roks_batch_create(arr, n, workers, C.byref(h))
        if st != 0:
            raise RoksError(st, "roks_batch_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.roks_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, tol: float = 1e-6, maxiter: int = 500, switch_tol: float = 0.0):
        """Per system: (status, iterations, final step info)."""
        n = len(self.systems)
        st = (C.c_int * n)()
        its = (C.c_int32 * n)()
        info = (StepInfo * n)()
        rc = self._L.roks_batch_solve(self._h, tol, maxiter, switch_tol, st, its, info)
        if rc != 0:
            raise RoksError(rc, "roks_batch_solve failed")
        return [(st[i], its[i], info[i].as_dict()) for i in range(n)]

    def steps(self, k: int):
        n = len(self.systems)
        st = (C.c_int * n)()
        rc = self._L.roks_batch_steps(self._h, k, st)
        if rc != 0:
            raise RoksError(rc, "roks_batch_steps failed")
        return list(st)

    def graph_steps(self, k: int):
        """roks_graph_steps(k) on every context: (statuses, accepted counts)."""
        n = len(self.systems)
        st = (C.c_int * n)()
        acc = (C.c_int32 * n)()
        rc = self._L.roks_batch_graph_steps(self._h, k, st, acc)
        if rc != 0:
            raise RoksError(rc, "roks_batch_graph_steps failed")
        return list(st), list(acc)
