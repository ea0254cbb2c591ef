"""roks_apply_h_noalloc_d (the allocation-free variant of roks_apply_h_d, its
scratch in a static device array) against roks_apply_h_d on the same
context, through the C ABI: two calls in a row, the second on a smaller
system (fewer bands, smaller grid), in shell mode and channel mode, on the
orbitals and on caller vectors; the oxide cell (its column buffer in several
chunks of band pairs) last.  FP64 bar: 1e-10 per band."""
import numpy as np
import pytest

from helpers import band_rel, ensure_built, small_molecule
from paper_2605_28637_amd import inputs

pytestmark = pytest.mark.gpu


def _torch_bands(c):
    import torch
    return torch.from_numpy(np.stack([c.real, c.imag], -1)).cuda().contiguous()


def _compare(system, mask, precision=0, tol=1e-10):
    import torch
    rb = ensure_built()
    print("noalloc case", system["name"], system["grid"], system["nbands"], mask, precision, flush=True)
    g = rb.Roks(system, precision=precision)
    g.set_coeffs(inputs.random_coefficients(g.miller(), system["cell"], g.nb, system["seed"]), True)
    nch = bin(mask).count("1") if mask else 1
    out_ref = torch.empty((nch, g.nb, g.npw, 2), dtype=torch.float64, device="cuda")
    out = torch.full_like(out_ref, float("nan"))
    v = _torch_bands(inputs.random_coefficients(g.miller(), system["cell"], g.nb, 99))
    torch.cuda.synchronize()
    with pytest.raises(rb.RoksError) as e:  # no potentials formed yet
        g.apply_h_noalloc_d(None, mask, out.data_ptr())
    assert e.value.status == 8
    g.energy_gradient()
    for src in (None, v):
        ptr = None if src is None else src.data_ptr()
        g.apply_h_d(ptr, mask, out_ref.data_ptr())
        g.apply_h_noalloc_d(ptr, mask, out.data_ptr())
        g.synchronize()
        a, b = out.cpu().numpy(), out_ref.cpu().numpy()
        assert np.isfinite(a).all()
        for k in range(nch):
            ac = a[k, ..., 0] + 1j * a[k, ..., 1]
            bc = b[k, ..., 0] + 1j * b[k, ..., 1]
            assert band_rel(ac, bc) < tol, (k, src is None)
    g.close()


def test_two_calls_second_smaller():
    _compare(inputs.molecule_box(), 0)
    _compare(small_molecule(), 0)


def test_channel_mode_and_fp32_tier():
    _compare(small_molecule(), 0b1011)
    _compare(small_molecule(), 0, precision=1, tol=1e-12)


def test_oxide_in_chunks_of_band_pairs():
    _compare(inputs.oxide_vacancy(), 0)
