"""Batches of uneven systems: the batch runs every context's CG iterations
from its own host thread on its own stream, so its results must equal, bit
for bit, the same contexts run one after the other (every reduction in the
library has a fixed order), in FP64 and in the FP32 tier."""
import numpy as np
import pytest

from helpers import ensure_built
from paper_2605_28637_amd import inputs

pytestmark = pytest.mark.gpu


def _contexts(rb, systems, precision=0, flags=0):
    out = []
    for s in systems:
        r = rb.Roks(s, precision=precision, flags=flags)
        r.set_coeffs(inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"]), True)
        out.append(r)
    return out


def _uneven(count=5):
    """The first systems of the 32-system uneven batch (10-60 atoms, 40^3-80^3
    grids), smallest band counts first so the test stays short."""
    systems = inputs.batch_systems(count=12)
    systems.sort(key=lambda s: s["nbands"])
    return systems[:count]


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_steps_equal_sequential(precision):
    rb = ensure_built()
    systems = _uneven()
    print("batch", [(s["grid"][0], s["nbands"]) for s in systems], "precision", precision, flush=True)
    seq = _contexts(rb, systems, precision)
    for r in seq:
        for _ in range(6):
            r.pcg_step()
    par = _contexts(rb, systems, precision)
    b = rb.Batch(par, workers=4)
    assert b.steps(6) == [0] * len(systems)
    for r1, r2 in zip(seq, par):
        np.testing.assert_array_equal(r1.get_coeffs(), r2.get_coeffs())
        e1, _, _ = r1.energy_gradient()
        e2, _, _ = r2.energy_gradient()
        assert e1["E"] == e2["E"]
    b.close()
    for r in seq + par:
        r.close()


def test_batch_solve_ladder_equals_sequential():
    rb = ensure_built()
    systems = _uneven(3)
    seq = _contexts(rb, systems, 1)
    res_seq = []
    for r in seq:
        i1, n1 = r.solve(tol=1e-5, maxiter=300)
        r.set_precision(0)
        i2, n2 = r.solve(tol=1e-7, maxiter=300)
        res_seq.append((n1 + n2, i2["E1"]))
    par = _contexts(rb, systems, 1)
    b = rb.Batch(par, workers=3)
    res = b.solve(tol=1e-7, maxiter=300, switch_tol=1e-5)
    for (st, its, info), (n, E) in zip(res, res_seq):
        assert st == 0
        assert its == n and info["E1"] == E
    b.close()
    for r in seq + par:
        r.close()


def test_autotuned_splits_are_shared_within_the_process():
    """With the autotuner on, the first context that meets a GEMM shape times
    the split counts; later contexts of the same shape reuse the choice, so a
    batch after a sequential run still reproduces it bit for bit, and the
    result agrees with the untuned heuristic to rounding."""
    rb = ensure_built()
    systems = _uneven(2)
    seq = _contexts(rb, systems, 0, rb.FLAG_AUTOTUNE)
    for r in seq:
        for _ in range(3):
            r.pcg_step()
    par = _contexts(rb, systems, 0, rb.FLAG_AUTOTUNE)
    b = rb.Batch(par, workers=2)
    b.steps(3)
    plain = _contexts(rb, systems, 0, 0)
    for r in plain:
        for _ in range(3):
            r.pcg_step()
    for r1, r2, r3 in zip(seq, par, plain):
        c1, c2, c3 = r1.get_coeffs(), r2.get_coeffs(), r3.get_coeffs()
        np.testing.assert_array_equal(c1, c2)
        assert np.abs(c1 - c3).max() < 1e-8 * np.abs(c3).max()
    b.close()
    for r in seq + par + plain:
        r.close()


def test_batch_rejects_repeated_contexts():
    rb = ensure_built()
    s = _uneven(1)[0]
    r = rb.Roks(s)
    with pytest.raises(rb.RoksError):
        rb.Batch([r, r])
    r.close()


_TUNE_CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_2605_28637_amd import inputs, roks as rb
s = sorted(inputs.batch_systems(count=12), key=lambda s: s["nbands"])[0]
r = rb.Roks(s, flags=rb.FLAG_AUTOTUNE)
r.set_coeffs(inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"]), True)
for _ in range(3):
    r.pcg_step()
np.save(sys.argv[2], r.get_coeffs())
r.close()
"""


def test_tuning_cache_file_is_written_and_read(tmp_path):
    """ROKS_TUNE_CACHE: a first process times the shapes and writes the file
    (JSON for this device); a second process sharing it makes the same
    choices and reproduces the first bit for bit; a third, given the file with
    every choice changed to another valid one, differs at the rounding level
    only, which shows the choices come from the file."""
    import json
    import os
    import subprocess
    import sys

    from helpers import ROOT
    cache = tmp_path / "tune.json"
    env = dict(os.environ, ROKS_TUNE_CACHE=str(cache))

    def child(out):
        print("child process", out, flush=True)
        subprocess.run([sys.executable, "-c", _TUNE_CHILD, ROOT, str(out)], env=env, check=True,
                       timeout=300)
        return np.load(out)

    c1 = child(tmp_path / "a.npy")
    with open(cache) as f:
        doc = json.load(f)
    assert doc["arch"].startswith("gfx") and doc["cus"] > 0 and len(doc["wdot"]) > 0
    assert all(len(e) == 4 and e[3] != 0 for e in doc["wdot"])
    c2 = child(tmp_path / "b.npy")
    np.testing.assert_array_equal(c1, c2)
    for e in doc["wdot"]:
        v = e[3]
        e[3] = (1 if v != 1 else 2) if v > 0 else (-1 if v != -1 else -2)
    with open(cache, "w") as f:
        f.write('{"arch": "%s", "cus": %d, "wdot": [\n' % (doc["arch"], doc["cus"]))
        f.write(",\n".join("[%d, %d, %d, %d]" % tuple(e) for e in doc["wdot"]))
        f.write("]}\n")
    c3 = child(tmp_path / "c.npy")
    assert not np.array_equal(c1, c3)
    assert np.abs(c1 - c3).max() < 1e-8 * np.abs(c1).max()
