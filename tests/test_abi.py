"""CPU-side checks of the C ABI library: it loads, exports every declared
symbol, and rejects invalid problems before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from helpers import ROOT, ensure_built
from paper_2605_28637_amd import inputs


def _declared():
    src = open(os.path.join(ROOT, "include", "roks.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(roks_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    rb = ensure_built()
    L = C.CDLL(rb.LIBPATH)
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert b"gfx950" in rb.lib().roks_version()


def test_binding_covers_the_abi():
    rb = ensure_built()
    assert set(_declared()) == set(rb._SIGS)


def _create_status(system, **kw):
    rb = ensure_built()
    try:
        r = rb.Roks(system, **kw)
    except rb.RoksError as e:
        return e.status, str(e)
    r.close()
    return 0, ""


def test_invalid_grid_for_cutoff_is_a_shape_error():
    s = dict(inputs.tiny_cell())
    s["ecut"] = 40.0  # sphere no longer fits the 16^3 grid
    st, msg = _create_status(s)
    assert st == 2, msg


def test_unsupported_grid_factor_is_a_shape_error():
    s = dict(inputs.tiny_cell())
    s["grid"] = (16, 16, 14)  # 7 is not a supported radix
    st, msg = _create_status(s)
    assert st == 2, msg


def test_band_order_is_validated():
    s = dict(inputs.tiny_cell())
    occ = s["occ"].copy()
    occ[:, :, [0, 4]] = occ[:, :, [4, 0]]  # an open-shell band before closed ones
    s["occ"] = occ
    st, msg = _create_status(s)
    assert st == 1, msg


def test_bad_occupation_values_rejected():
    s = dict(inputs.tiny_cell())
    occ = s["occ"].copy()
    occ[0, 0, 0] = 2
    s["occ"] = occ
    st, msg = _create_status(s)
    assert st == 1, msg


def test_asymmetric_D_rejected():
    s = inputs.molecule_box(natoms=2, nb=8, N=16, L=8.0)
    sp = [dict(x) for x in s["species"]]
    D = np.array(sp[0]["D"], dtype=float)
    D[0, 1] = 0.3
    sp[0]["D"] = D
    s = dict(s)
    s["species"] = sp
    st, msg = _create_status(s)
    assert st == 1, msg


def test_nonfinite_position_rejected():
    s = dict(inputs.tiny_cell())
    pos = s["pos"].copy()
    pos[0, 0] = np.nan
    s["pos"] = pos
    st, msg = _create_status(s)
    assert st == 1, msg


def test_precision_tier_validated():
    st, msg = _create_status(inputs.tiny_cell(), precision=7)
    assert st == 1, msg


def test_grid_rule_gives_the_workload_grids():
    """grid = (0, 0, 0) at create: G_cut = pi N / (2 L) with N the next
    2^a 3^b 5^c size; the molecule, oxide and batch cells were set up with
    exactly that rule, the tiny cell (7.5 Ha on 16^3) with a larger cutoff."""
    rb = ensure_built()
    for s in (inputs.molecule_box(), inputs.oxide_vacancy(), *inputs.batch_systems()[:6]):
        assert rb.grid_rule(s["cell"], s["ecut"]) == tuple(s["grid"]), s["name"]
    # a cutoff just above the rule's value for 64 needs the next size (72)
    assert rb.grid_rule(np.eye(3) * 24.0, inputs.grid_rule_ecut(24.0, 64) * 1.001) == (72, 72, 72)
    # non-cubic: each axis on its own
    g = rb.grid_rule(np.diag([10.0, 12.0, 15.0]), inputs.grid_rule_ecut(15.0, 30))
    assert g == (20, 24, 30)
    assert rb.lib().roks_grid_rule(None, 1.0, None) == 1
