"""The H-application of many uneven systems captured into one hipGraph.

roks_apply_h_noalloc_d allocates nothing and never synchronises, so a caller
can capture it: here the applies of several batch members (uneven grids and
band counts, shell mode and all four channels of both configurations), each
context created on the capturing stream, go into one graph.  The graph is
replayed several times with the program's own eager work and synchronisations
between replays, and every replay is compared with the eager result bit for
bit (the same kernels in the same order on the same data)."""
import numpy as np
import pytest

from helpers import ensure_built
from paper_2605_28637_amd import inputs

pytestmark = pytest.mark.gpu


def _members(count):
    systems = inputs.batch_systems(count=12)
    systems.sort(key=lambda s: s["nbands"])
    return systems[:count]


def test_batch_apply_graph_replays_match_eager():
    import torch
    rb = ensure_built()
    stream = torch.cuda.Stream()
    systems = _members(4)
    print("graph members", [(s["grid"][0], s["nbands"]) for s in systems], flush=True)
    ctxs, outs, refs, masks = [], [], [], []
    for i, s in enumerate(systems):
        r = rb.Roks(s, stream=stream.cuda_stream)
        r.set_coeffs(inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"]), True)
        r.energy_gradient()  # the potentials the applies use
        mask = 0 if i % 2 == 0 else 0b1111
        nch = 1 if mask == 0 else 4
        outs.append(torch.empty((nch, r.nb, r.npw, 2), dtype=torch.float64, device="cuda"))
        refs.append(torch.empty_like(outs[-1]))
        ctxs.append(r)
        masks.append(mask)
    torch.cuda.synchronize()
    # eager: first use sets every kernel's LDS limit, so the capture makes no
    # runtime call beyond the launches
    for r, ref, m in zip(ctxs, refs, masks):
        r.apply_h_noalloc_d(None, m, ref.data_ptr())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for r, o, m in zip(ctxs, outs, masks):
            r.apply_h_noalloc_d(None, m, o.data_ptr())
    torch.cuda.synchronize()
    scratch = [torch.empty_like(o) for o in outs]
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (o, ref) in enumerate(zip(outs, refs)):
            assert torch.equal(o, ref), (rep, k)
        # eager work of the program between replays, on the same contexts
        for r, sc, m in zip(ctxs, scratch, masks):
            r.apply_h_noalloc_d(None, m, sc.data_ptr())
        torch.cuda.synchronize()
        for sc, ref in zip(scratch, refs):
            assert torch.equal(sc, ref)
    del g
    for r in ctxs:
        r.close()
