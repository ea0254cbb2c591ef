#!/usr/bin/env python
"""Benchmark of the ROKS hot path on one MI355X.

Headline workload: the rocksalt oxide-vacancy supercell (3 x 3 x 3
conventional cells, a = 8 bohr, one anion removed: 215 atoms, 96^3 grid at
the grid-rule cutoff of 19.74 Ha, 28 889 stored plane waves, 8 Gaussian
projectors per atom = 1 720, 432 bands = 428 closed + 2 open + 2 virtual,
mixed-spin and triplet configurations of the singlet), FP64.

One step = one pass of the whole hot path: densities, potentials and
energies of both configurations, F^n|n> for every band (the band
H-applications), theta / g_I / R / A, the projected Teter preconditioner,
Fletcher-Reeves directions, the line search (Cholesky orthonormalisation,
rotation, trial energies), the commit, and the forces.  value = band
H-applications per second over the timed steps (nbands per step).

Kernel times come from HIP events the library records on its own stream
(roks_timing_*), with the algorithmic bytes and flops of every launch: one
pass with every kernel family recorded (the per-family table), then the
timed region with events only around the dominant family (the roofline
entry), so the other launches run undisturbed.

Extras on the same line: the FP32 and BF16x3 tiers on the same workload, the 64^3 /
40-band molecule-in-box (configuration of the earlier headline), ROKS
time-to-converge (plain FP64 against the FP32 ladder and the learned
preconditioner, each judged by plain FP64 iterations), the uneven batch, and
the oracle's rate on the host cores.

Prints ONE JSON line.  Inputs are resident on the GPU when timing starts.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2605_28637_amd import inputs  # noqa: E402
from paper_2605_28637_amd import roks as rb  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
RESTART = 20

# HBM traffic per launch of a kernel family on a workload, from the rocprofv3
# FETCH_SIZE / WRITE_SIZE passes summarised in profiles/ (scaled by the
# copy-kernel calibration); reported only while the sources of the family's
# kernels are the ones measured.
TRAFFIC = {
    ("gemm_expand", "oxide", 0): {
        "bytes_per_launch": 1.18339e+09,
        "profile": "profiles/gemm_expand_oxide_fp64_traffic.md",
        "sources": ["paper_2605_28637_amd/csrc/tile_gemm.hip"],
        "sha256": "98ca437b0ae4f7ecccfd42604e55306926e694890d15466f079b6e1cbf8c430a"},
}
KERNELS = ("zpass_bwd", "plane_apply", "plane_density", "zpass_fwd", "fft3d", "gemm_wdot",
           "gemm_expand", "xc", "proj_bf3")


def roofline(name, k, fp32=False):
    """Roofline entry of one kernel family from its summed time and work: the
    band products and expansions (gemm_*) against the FP64 matrix cores, the
    BF16x3 projector products (proj_bf3, flops of the three BF16 products)
    against the dense BF16 matrix cores (2.5 PFLOP/s), the transforms and
    pointwise passes against the vector units of their tier (FP64 78.6, FP32
    157.3 TFLOP/s), each against HBM when its algorithmic flop/byte lies
    below that peak's ridge."""
    if not k["launches"] or k["ms_total"] <= 0:
        return None
    avg_s = k["ms_total"] * 1e-3 / k["launches"]
    by, fl = k["bytes"] / k["launches"], k["flops"] / k["launches"]
    mfma = name.startswith("gemm") or name == "proj_bf3"
    if name == "proj_bf3":
        peak = BF16_PEAK_TFLOPS
    else:
        peak = FP64_PEAK_TFLOPS if (mfma or not fp32) else FP32_VECTOR_PEAK_TFLOPS
    ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    if fl > 0 and fl / by > ridge:
        ach = fl / avg_s / 1e12
        return {"bound": "mfma" if mfma else "alu", "kernel": name, "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                "flops_per_launch": fl, "bytes_per_launch": by, "avg_launch_ms": avg_s * 1e3}
    ach = by / avg_s / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": by,
            "flops_per_launch": fl, "avg_launch_ms": avg_s * 1e3}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, nsample=12):
    """The oracle, as it stands, on a bounded sample of the headline
    workload: the band H-applications F^{X(n)}|n> (shell mode, what a CG step
    applies per band) of `nsample` bands spread over every shell, timed with
    the BLAS threads on all host cores and then on one; the potentials of the
    same orbitals (one energy evaluation, part of every step) timed apart."""
    from threadpoolctl import threadpool_limits

    from oracle import roks as orc
    cores = len(os.sched_getaffinity(0))
    m = orc.Model(system)
    psi = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, system["seed"]))
    t0 = time.perf_counter()
    pot = orc.potentials(m, psi)
    t_pot = time.perf_counter() - t0
    pot.u = None
    idx = np.unique(np.linspace(0, m.nb - 1, nsample).astype(int))

    def rate(limit):
        with threadpool_limits(limits=limit):
            t0 = time.perf_counter()
            for n in idx:
                X = m.band_shell[n]
                if not m.shell_virtual[X]:
                    orc.apply_shell_operator(m, pot, X, psi[n:n + 1])
            return len(idx) / (time.perf_counter() - t0)

    r_all, r_one = rate(cores), rate(1)
    return {"value": r_all, "unit": "band H-applies/s", "cores": cores, "kind": "oracle",
            "one_core_value": r_one, "cpu_model": _cpu_model(),
            "energy_evaluation_s": t_pot,
            "sample": "oracle F^{X(n)}|n> of %d of the %d oxide bands (every shell; 96^3, 1 720 "
                      "projectors), BLAS threads on all %d host cores (one_core_value: one "
                      "thread); the potentials of those orbitals formed beforehand, %.1f s, "
                      "not in the rate" % (len(idx), m.nb, cores, t_pot)}


def _converge(rb_system, c0, tol, precision, net, restart, switch_tol=1e-5, maxiter=3000, flags=0):
    """One solve: FP32 iterations to |dE| < switch_tol, then FP64 to tol (a pure
    FP64 solve when precision is FP64)."""
    r = rb.Roks(rb_system, precision=precision, flags=flags)
    r.set_coeffs(c0, True)
    r.set_restart(restart)
    if net is not None:
        r.set_mlp(net)
    it = 0
    if precision == rb.FP32:
        try:
            _, n = r.solve(tol=switch_tol, maxiter=maxiter)
            it += n
        except rb.RoksError as e:
            if e.status != 6:  # a stall above the FP32 resolution: move on to FP64
                raise
        r.set_precision(rb.FP64)
    info, n = r.solve(tol=tol, maxiter=maxiter)
    return r, info, it + n


def _judged(r, info, tol, net, restart, max_rounds=6, maxiter=3000):
    """The plain FP64 method judges the result: three plain iterations (no
    network, no restarts, fresh directions) from it must each stay within tol
    of its energy; otherwise the variant solves on and is judged again.
    Returns the judged energy, the iterations the judging took (its plain
    iterations and any further solves) and the rounds."""
    extra, rounds = 0, 0
    E = info["E1"]
    while True:
        rounds += 1
        r.set_mlp(None)
        r.set_precision(rb.FP64)
        r.set_restart(0)
        r.reset_cg()
        Es = [r.pcg_step()["E1"] for _ in range(3)]
        extra += 3
        drift = max(abs(e - E) for e in Es)
        E = Es[-1]
        if drift < tol or rounds >= max_rounds:
            return E, extra, rounds, drift
        r.set_restart(restart)
        if net is not None:
            r.set_mlp(net)
        i2, n = r.solve(tol=tol, maxiter=maxiter)
        extra += n
        E = i2["E1"]


def time_to_converge(system, tol, precision, net, restart, flags=0):
    """Ground state from the seeded start, then the singlet from the
    ground-state orbitals, each judged by plain FP64 iterations, then the
    singlet forces; wall time of all of it."""
    gs = inputs.with_configuration(system, "gs")
    rg = rb.Roks(gs)
    c0 = inputs.random_coefficients(rg.miller(), gs["cell"], rg.nb, gs["seed"])
    rg.close()
    t0 = time.perf_counter()
    rg, ig, itg = _converge(gs, c0, tol, precision, net, restart, flags=flags)
    E_gs, jg, rounds_g, drift_g = _judged(rg, ig, tol, net, restart)
    c = rg.get_coeffs()
    rg.close()
    r, ie, ite = _converge(system, c, tol, precision, net, restart, flags=flags)
    E_s, js, rounds_s, drift_s = _judged(r, ie, tol, net, restart)
    F = r.forces()
    r.synchronize()
    dt = time.perf_counter() - t0
    r.close()
    return {"seconds": dt, "gs_iterations": itg + jg, "singlet_iterations": ite + js,
            "E_gs": E_gs, "E_singlet": E_s, "excitation_Ha": E_s - E_gs, "forces": F,
            "judge": {"plain_fp64_iterations": 3, "rounds_gs": rounds_g, "rounds_singlet": rounds_s,
                      "drift_gs_Ha": drift_g, "drift_singlet_Ha": drift_s,
                      "passed": bool(drift_g < tol and drift_s < tol)},
            "tol_Ha": tol,
            "arithmetic": "fp32 tier to |dE| < 1e-5 Ha, then fp64" if precision == rb.FP32 else "fp64",
            "preconditioner": "learned rescaling of Teter" if net is not None else "Teter",
            "cg_restart_period": restart,
            "iterations_driven": "graph mode (device decisions, replays of 8)"
            if flags & rb.FLAG_GRAPH else "host"}


def train_network(seeds, steps=600, lr=3e-3):
    """Training pairs from recorded FP64 runs (ground state, then singlet) of
    the training seeds, then Adam on the GPU."""
    t0 = time.perf_counter()
    net = rb.Mlp(seed=1)
    for sd in seeds:
        s = inputs.molecule_box(seed=sd)
        gs = inputs.with_configuration(s, "gs")
        rg = rb.Roks(gs)
        rg.set_coeffs(inputs.random_coefficients(rg.miller(), gs["cell"], rg.nb, gs["seed"]), True)
        rg.set_restart(RESTART)
        rg.record(300, 1)
        rg.solve(tol=1e-9, maxiter=3000)
        net.collect(rg)
        c = rg.get_coeffs()
        rg.close()
        r = rb.Roks(s)
        r.set_coeffs(c, True)
        r.set_restart(RESTART)
        r.record(300, 1)
        r.solve(tol=1e-9, maxiter=3000)
        net.collect(r)
        r.close()
    t1 = time.perf_counter()
    hist = net.train(steps, lr)
    t2 = time.perf_counter()
    S, nseg = net.num_samples()
    return net, {"seeds": seeds, "samples": S, "recorded_iterates": nseg,
                 "collect_seconds": t1 - t0, "train_seconds": t2 - t1, "adam_steps": steps,
                 "loss_first": float(hist[0]), "loss_last": float(hist[-1])}


def _start(system):
    gs = inputs.with_configuration(system, "gs")
    r = rb.Roks(gs)
    c0 = inputs.random_coefficients(r.miller(), gs["cell"], r.nb, gs["seed"])
    r.close()
    return gs, c0


def _steps_to(r, Eref, precision, switch_tol=1e-5, maxiter=3000):
    """CG steps until E <= Eref + 1e-6 Ha (FP32 first when precision is FP32,
    FP64 from the first two consecutive |dE| < switch_tol on)."""
    hits, k = 0, 0
    fp32 = precision == rb.FP32
    while k < maxiter:
        i = r.pcg_step()
        k += 1
        if i["E1"] - Eref < 1e-6:
            return k
        if fp32:
            hits = hits + 1 if abs(i["E1"] - i["E0"]) < switch_tol else 0
            if hits >= 2:
                r.set_precision(rb.FP64)
                fp32 = False
    return -1


def time_to_reference(system, ref, precision, net, restart):
    """Wall time until the ground state and then the singlet (from the
    ground-state orbitals of the same run) are within 1e-6 Ha of the
    tightly converged reference energies; singlet forces at the end."""
    gs, c0 = _start(system)
    t0 = time.perf_counter()
    out = {}
    c = c0
    for name, s, Eref in (("gs", gs, ref["E_gs"]), ("singlet", system, ref["E_singlet"])):
        r = rb.Roks(s, precision=precision)
        r.set_coeffs(c, True)
        r.set_restart(restart)
        if net is not None:
            r.set_mlp(net)
        out[name + "_iterations"] = _steps_to(r, Eref, precision)
        if name == "gs":
            c = r.get_coeffs()
            r.close()
    F = r.forces()
    r.synchronize()
    out["seconds"] = time.perf_counter() - t0
    out["max_force_diff_vs_reference"] = float(np.abs(F - ref["forces"]).max())
    r.close()
    return out


def converge_report(system, tol=1e-6):
    """ROKS time-to-converge, two ways for every variant: the stopping rule
    |dE| < 1e-6 Ha on two consecutive iterations, and the time to come
    within 1e-6 Ha of a tightly converged (1e-10 Ha) plain FP64 reference.
    Variants: the plain FP64 method (Fletcher-Reeves without restarts), then
    with restarts every 20 steps, the FP32 tier, the learned rescaling
    (network trained on three other seeds; training time reported, not
    counted), and both."""
    gs, c0 = _start(system)
    rg, ig, _ = _converge(gs, c0, 1e-10, rb.FP64, None, RESTART)
    c = rg.get_coeffs()
    rg.close()
    rr, ie, _ = _converge(system, c, 1e-10, rb.FP64, None, RESTART)
    ref = {"E_gs": ig["E1"], "E_singlet": ie["E1"], "forces": rr.forces()}
    rr.close()
    out = {"reference": {"E_gs": ref["E_gs"], "E_singlet": ref["E_singlet"],
                         "excitation_Ha": ref["E_singlet"] - ref["E_gs"], "tol_Ha": 1e-10}}
    net, tr = train_network([2001, 2002, 2003])
    for k, prec, nn, rs in (("plain_fp64", rb.FP64, None, 0),
                            ("plain_fp64_restart", rb.FP64, None, RESTART),
                            ("mixed_plain_restart", rb.FP32, None, RESTART),
                            ("fp64_learned", rb.FP64, net, RESTART),
                            ("mixed_learned", rb.FP32, net, RESTART)):
        v = time_to_converge(system, tol, prec, nn, rs)
        F = v.pop("forces")
        v["dE_singlet_vs_reference_Ha"] = v["E_singlet"] - ref["E_singlet"]
        v["d_excitation_vs_reference_Ha"] = v["excitation_Ha"] - (ref["E_singlet"] - ref["E_gs"])
        v["max_force_diff_vs_reference"] = float(np.abs(F - ref["forces"]).max())
        v["to_reference"] = time_to_reference(system, ref, prec, nn, rs)
        out[k] = v
    # the variants with restarts again with their iterations in graph mode
    for k, prec, nn in (("plain_fp64_restart_graph", rb.FP64, None),
                        ("mixed_plain_restart_graph", rb.FP32, None),
                        ("mixed_learned_graph", rb.FP32, net)):
        v = time_to_converge(system, tol, prec, nn, RESTART, flags=rb.FLAG_GRAPH)
        F = v.pop("forces")
        v["dE_singlet_vs_reference_Ha"] = v["E_singlet"] - ref["E_singlet"]
        v["max_force_diff_vs_reference"] = float(np.abs(F - ref["forces"]).max())
        out[k] = v
    net.close()
    out["training"] = tr
    sec = {k: out[k]["seconds"] for k in ("plain_fp64", "plain_fp64_restart", "mixed_plain_restart",
                                          "fp64_learned", "mixed_learned")}
    out["speedups_judged"] = {
        "mixed_learned_vs_plain_fp64": sec["plain_fp64"] / sec["mixed_learned"],
        "mixed_learned_vs_plain_fp64_restart": sec["plain_fp64_restart"] / sec["mixed_learned"],
        "learned_vs_plain_restart_fp64": sec["plain_fp64_restart"] / sec["fp64_learned"],
        "fp32_tier_vs_fp64_restart": sec["plain_fp64_restart"] / sec["mixed_plain_restart"],
        "fp32_tier_with_learned_vs_fp64_learned": sec["fp64_learned"] / sec["mixed_learned"],
        "graph_vs_host_fp64_restart": sec["plain_fp64_restart"] / out["plain_fp64_restart_graph"]["seconds"],
        "graph_vs_host_fp32_tier_restart":
            sec["mixed_plain_restart"] / out["mixed_plain_restart_graph"]["seconds"],
        "graph_vs_host_mixed_learned": sec["mixed_learned"] / out["mixed_learned_graph"]["seconds"]}
    out["speedup_mixed_learned_vs_plain_fp64_to_reference"] = (
        out["plain_fp64"]["to_reference"]["seconds"] / out["mixed_learned"]["to_reference"]["seconds"])
    return out


def batch_report(steps=8, workers=4):
    """The uneven batch: 32 molecule-in-box systems (10-60 atoms, 20-120
    bands, 40^3-80^3 grids), ROKS (mixed-spin and triplet), FP32 tier; a fixed
    number of CG steps on every system, one after the other and then as a
    batch (work queue, longest first, one stream per worker; four workers,
    one per hardware queue of the device: with eight the host-driven batch
    is 14 % slower)."""
    systems = inputs.batch_systems()
    def make():
        out = []
        for s in systems:
            r = rb.Roks(s, precision=rb.FP32)
            r.set_coeffs(inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"]), True)
            out.append(r)
        return out
    total_bands = sum(s["nbands"] for s in systems)
    seq = make()
    for r in seq:
        r.pcg_step()  # warm-up (first-use allocations)
    t0 = time.perf_counter()
    for r in seq:
        for _ in range(steps):
            r.pcg_step()
        r.synchronize()  # one context after another: its last step's tail included
    t_seq = time.perf_counter() - t0
    par = make()
    b = rb.Batch(par, workers=workers)
    b.steps(1)
    t0 = time.perf_counter()
    st = b.steps(steps)
    t_par = time.perf_counter() - t0
    same = all(np.array_equal(r1.get_coeffs(), r2.get_coeffs()) for r1, r2 in zip(seq, par))
    b.close()
    for r in seq + par:
        r.close()
    return {"systems": len(systems), "bands_total": total_bands,
            "grids": sorted({s["grid"][0] for s in systems}), "steps_each": steps,
            "workers": workers, "arithmetic": "fp32 tier", "sequential_seconds": t_seq,
            "batched_seconds": t_par,
            "sequential_band_applies_per_s": total_bands * steps / t_seq,
            "batched_band_applies_per_s": total_bands * steps / t_par,
            "speedup": t_seq / t_par, "all_ok": all(x == 0 for x in st),
            "batched_equals_sequential": bool(same)}


def cg_graph_report(steps=8, workers=4):
    """CG iterations in graph mode (every decision on the device, k
    iterations captured once per context and replayed) against the same
    iterations driven from the host, FP32 tier: the 32 uneven batch members
    (one graph per member, replayed on the workers' streams), and the
    smallest alone on its own stream."""
    systems = sorted(inputs.batch_systems(), key=lambda s: s["nbands"])

    def make():
        out = []
        for s in systems:
            r = rb.Roks(s, precision=rb.FP32)
            r.set_coeffs(inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"]), True)
            out.append(r)
        return out
    total_bands = sum(s["nbands"] for s in systems)
    res = {"systems": len(systems), "bands_total": total_bands,
           "grids": sorted({s["grid"][0] for s in systems}), "steps_each": steps,
           "workers": workers, "arithmetic": "fp32 tier"}
    host = make()
    b = rb.Batch(host, workers=workers)
    b.steps(steps)  # warm-up
    t0 = time.perf_counter()
    st = b.steps(steps)
    t_host = time.perf_counter() - t0
    b.close()
    graph = make()
    b = rb.Batch(graph, workers=workers)
    b.graph_steps(steps)  # capture (and one replay)
    t0 = time.perf_counter()
    st2, acc = b.graph_steps(steps)
    t_graph = time.perf_counter() - t0
    b.close()
    res.update({"host_seconds": t_host, "graph_seconds": t_graph,
                "host_band_applies_per_s": total_bands * steps / t_host,
                "graph_band_applies_per_s": total_bands * steps / t_graph,
                "speedup": t_host / t_graph,
                "all_ok": all(x == 0 for x in st + st2),
                "graph_steps_accepted": int(sum(acc)), "graph_steps_run": steps * len(systems),
                # members that reach the tier's resolution stop accepting
                # steps (a graph halts at its first rejection): the rate of
                # accepted band-steps only
                "graph_accepted_band_steps_per_s":
                    sum(a * s["nbands"] for a, s in zip(acc, systems)) / t_graph})
    # one member alone: host steps against graph replays on its own stream
    one_h, one_g = host[0], graph[0]
    for _ in range(2):
        one_h.pcg_step()
    one_h.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_h.pcg_step()
    one_h.synchronize()
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    a1, _ = one_g.graph_steps(steps)
    t2 = time.perf_counter() - t0
    res["single"] = {"grid": systems[0]["grid"][0], "nbands": systems[0]["nbands"],
                     "host_ms_per_step": 1e3 * t1 / steps, "graph_ms_per_step": 1e3 * t2 / steps,
                     "accepted": a1}
    for r in host + graph:
        r.close()
    return res


def batch_solve_report(tol=1e-6, switch_tol=1e-5, workers=4):
    """The 32-system batch solved to |dE| < tol (FP32 tier to switch_tol,
    then FP64: the precision ladder), iterations driven from the host and
    then in graph mode (ROKS_FLAG_GRAPH), from the same starts."""
    systems = inputs.batch_systems()
    res = {"systems": len(systems), "tol_Ha": tol, "switch_tol_Ha": switch_tol, "workers": workers}
    energies = {}
    for name, flags in (("host", 0), ("graph", rb.FLAG_GRAPH)):
        ctxs = []
        for s in systems:
            r = rb.Roks(s, precision=rb.FP32, flags=flags)
            r.set_coeffs(inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"]), True)
            ctxs.append(r)
        b = rb.Batch(ctxs, workers=workers)
        t0 = time.perf_counter()
        out = b.solve(tol=tol, maxiter=3000, switch_tol=switch_tol)
        res[name + "_seconds"] = time.perf_counter() - t0
        res[name + "_iterations"] = int(sum(o[1] for o in out))
        res[name + "_all_ok"] = all(o[0] == 0 for o in out)
        energies[name] = [o[2]["E1"] for o in out]
        b.close()
        for r in ctxs:
            r.close()
    res["speedup"] = res["host_seconds"] / res["graph_seconds"]
    res["max_abs_dE_graph_vs_host_Ha"] = float(max(abs(a - b) for a, b in
                                                   zip(energies["host"], energies["graph"])))
    return res


def batch_cg_only(mode, steps=8, workers=4):
    """The 32-system batch (FP32 tier): a warm-up call, then `steps` CG
    iterations of every system driven from the host (roks_batch_steps) or in
    graph mode (roks_batch_graph_steps); one JSON line with the timed call's
    wall time."""
    systems = inputs.batch_systems()
    ctxs = []
    for s in systems:
        r = rb.Roks(s, precision=rb.FP32)
        r.set_coeffs(inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"]), True)
        ctxs.append(r)
    b = rb.Batch(ctxs, workers=workers)
    run = (lambda: b.steps(steps)) if mode == "host" else (lambda: b.graph_steps(steps))
    run()
    t0 = time.perf_counter()
    run()
    dt = time.perf_counter() - t0
    b.close()
    for r in ctxs:
        r.close()
    print(json.dumps({"batch_cg": mode, "systems": len(systems), "steps_each": steps,
                      "workers": workers, "seconds": dt,
                      "band_applies_per_s": sum(s["nbands"] for s in systems) * steps / dt}))


def oxide_graph_report(system, steps=4):
    """Graph mode on the oxide supercell (FP64): `steps` CG iterations
    replayed from one graph against the same iterations driven from the
    host, from the same start (forces not included)."""
    res = {}
    for mode in ("host", "graph"):
        r = rb.Roks(system)
        r.set_coeffs(inputs.random_coefficients(r.miller(), system["cell"], r.nb, system["seed"]), True)
        if mode == "host":
            r.pcg_step()
            r.synchronize()
            t0 = time.perf_counter()
            infos = [r.pcg_step() for _ in range(steps)]
            r.synchronize()
        else:
            r.pcg_step()
            r.graph_steps(steps)  # capture (and one replay)
            r.reset_cg()
            r.set_coeffs(inputs.random_coefficients(r.miller(), system["cell"], r.nb,
                                                    system["seed"]), True)
            r.pcg_step()
            r.synchronize()
            t0 = time.perf_counter()
            acc, infos = r.graph_steps(steps)
            res["graph_accepted"] = acc
        res[mode + "_ms_per_iteration"] = 1e3 * (time.perf_counter() - t0) / steps
        res[mode + "_E1"] = infos[-1]["E1"]
        r.close()
    res["speedup"] = res["host_ms_per_iteration"] / res["graph_ms_per_iteration"]
    res["nbands"] = system["nbands"]
    return res


def graph_report(reps=20):
    """The H-application (shell mode, both configurations' operators) of all
    32 uneven batch systems, FP32 tier, through the allocation-free entry
    point on one stream: eager calls one system after another, then the same
    calls captured once into a hipGraph and replayed."""
    import torch
    systems = inputs.batch_systems()
    stream = torch.cuda.Stream()
    ctxs, outs = [], []
    for s in systems:
        r = rb.Roks(s, precision=rb.FP32, stream=stream.cuda_stream)
        r.set_coeffs(inputs.random_coefficients(r.miller(), s["cell"], r.nb, s["seed"]), True)
        r.energy_gradient()
        outs.append(torch.empty((r.nb, r.npw, 2), dtype=torch.float64, device="cuda"))
        ctxs.append(r)
    total_bands = sum(r.nb for r in ctxs)

    def eager():
        for r, o in zip(ctxs, outs):
            r.apply_h_noalloc_d(None, 0, o.data_ptr())

    eager()
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    t0 = time.perf_counter()
    for _ in range(reps):
        eager()
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / reps
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        eager()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    same = all(torch.equal(o, r) for o, r in zip(outs, ref))
    del g
    for r in ctxs:
        r.close()
    return {"systems": len(systems), "bands_total": total_bands, "arithmetic": "fp32 tier",
            "launches": "roks_apply_h_noalloc_d per system, one stream",
            "eager_ms_per_round": 1e3 * t_eager, "graph_ms_per_round": 1e3 * t_graph,
            "eager_band_applies_per_s": total_bands / t_eager,
            "graph_band_applies_per_s": total_bands / t_graph, "speedup": t_eager / t_graph,
            "graph_equals_eager": bool(same)}


def graph_report_child(timeout=600):
    """graph_report in a child process whose PyTorch GPU context is created
    before the library's (this process has the library's runtime already)."""
    import subprocess
    code = ("import json, sys; sys.path.insert(0, %r); import bench; bench.init_torch_gpu(); "
            "print(json.dumps(bench.graph_report()))" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=timeout)
    if r.returncode != 0:
        return {"error": r.stderr.strip().splitlines()[-1] if r.stderr.strip() else "failed"}
    return json.loads(r.stdout.strip().splitlines()[-1])


def calibrate_copy(mib=512, reps=3):
    """A plain copy kernel of known size (y = 1.0 * x, FP32, contiguous) for
    scaling the FETCH_SIZE / WRITE_SIZE counters: it reads and writes
    exactly `mib` MiB per launch."""
    import torch
    n = mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_kernel": "elementwise y = 1.0 * x (torch.mul, FP32)", "launches": reps,
                      "read_bytes_per_launch": 4 * n, "write_bytes_per_launch": 4 * n}))


def measure(system, precision, steps, warmup, table_steps=None):
    """Steps of the whole hot path (one CG iteration + forces each) on one
    context: a pass with every kernel family event-timed (the table), then the
    timed region with events around the dominant family only."""
    r = rb.Roks(system, precision=precision)
    r.set_coeffs(inputs.random_coefficients(r.miller(), system["cell"], r.nb, system["seed"]), True)
    for _ in range(warmup):
        r.pcg_step()
        r.forces()
    r.synchronize()
    r.timing_enable(True)
    for _ in range(table_steps or steps):
        r.pcg_step()
        r.forces()
    r.synchronize()
    kernels = {k: r.timing_read(k) for k in KERNELS}
    r.timing_enable(False)
    fp32 = precision != rb.FP64
    roofs = {k: roofline(k, v, fp32) for k, v in kernels.items()}
    dom = max((k for k in kernels if roofs[k]), key=lambda k: kernels[k]["ms_total"])
    r.timing_only(dom)
    r.timing_enable(True)
    r.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.pcg_step()
        r.forces()
    r.synchronize()
    elapsed = time.perf_counter() - t0
    dom_live = r.timing_read(dom)
    r.timing_enable(False)
    r.timing_only(None)
    nb, npw = r.nb, r.npw
    r.close()
    roof_live = roofline(dom, dom_live, fp32)
    key = (dom, system["name"], precision)
    if roof_live and key in TRAFFIC:
        t = TRAFFIC[key]
        digest = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read()
                                         for f in t["sources"])).hexdigest()
        if digest == t["sha256"]:
            roof_live["traffic"] = t["bytes_per_launch"]
            roof_live["traffic_source"] = t["profile"]
    # the band H-apply pipeline (z pass G->r, plane multiply, z pass r->G);
    # the G->r z pass also serves every density evaluation, so its time and
    # bytes are prorated to the H-apply launches
    na = kernels["plane_apply"]["launches"]
    zb = kernels["zpass_bwd"]
    frac_zb = na / max(1, zb["launches"])
    happ_ms = (kernels["plane_apply"]["ms_total"] + kernels["zpass_fwd"]["ms_total"]
               + frac_zb * zb["ms_total"])
    happ_bytes = (kernels["plane_apply"]["bytes"] + kernels["zpass_fwd"]["bytes"]
                  + frac_zb * zb["bytes"])
    pipeline = {"achieved_GBs": happ_bytes / (happ_ms * 1e-3) / 1e9 if happ_ms else None,
                "frac_hbm": happ_bytes / (happ_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if happ_ms else None,
                "ms_per_all_band_apply": happ_ms / max(1, na),
                "band_applies_per_s": nb * na / (happ_ms * 1e-3) if happ_ms else None}
    return {"nb": nb, "npw": npw, "elapsed": elapsed, "steps": steps,
            "band_applies_per_s": nb * steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
            "roofline": roof_live,
            "kernels": {k: dict(v, roofline_frac=(roofs[k] or {}).get("frac"))
                        for k, v in kernels.items()},
            "h_apply_pipeline": pipeline}


def init_torch_gpu():
    """PyTorch carries its own HIP runtime: its GPU context must exist before
    the library's when a leg hands it torch streams or buffers."""
    import torch
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="the headline line only (no FP32 tier, molecule, converge, batch, CPU legs)")
    ap.add_argument("--tier", choices=("fp64", "fp32", "bf16x3"), default="fp64",
                    help="arithmetic tier of the headline measurement (profiling runs)")
    ap.add_argument("--batch-cg", choices=("host", "graph"), default=None,
                    help="only the 32-system batch's CG iterations (8 each, after a "
                         "warm-up call), driven from the host or in graph mode: the "
                         "workload of the graph-mode kernel trace")
    ap.add_argument("--molecule-only", action="store_true",
                    help="only the 64^3 molecule-in-box steps (FP64), one JSON line: the "
                         "second workload of the plane-pass counters")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the copy kernel that scales the HBM byte counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.batch_cg:
        batch_cg_only(args.batch_cg)
        return
    if args.molecule_only:
        m = measure(inputs.molecule_box(), rb.FP64, args.steps, args.warmup,
                    table_steps=min(args.steps, 4))
        print(json.dumps({"molecule_64": {k: m[k] for k in ("band_applies_per_s", "ms_per_step",
                                                              "nb", "npw")}}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    system = inputs.oxide_vacancy()
    tier = {"fp64": rb.FP64, "fp32": rb.FP32, "bf16x3": rb.FP32_BF16X3}[args.tier]
    head = measure(system, tier, args.steps, args.warmup, table_steps=min(args.steps, 4))
    out = {
        "metric": "band H-applies/s",
        "value": head["band_applies_per_s"],
        "unit": "band H-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[args.tier],
        "data": "synthetic",
        "config": {"workload": "rocksalt oxide-vacancy supercell: 3x3x3 conventional cells, "
                               "a = 8 bohr, one anion removed (215 atoms), 96^3 grid, ecut "
                               "19.74 Ha, %d stored plane waves, 8 Gaussian projectors per atom "
                               "(1 720), %d bands (428 closed + 2 open + 2 virtual), mixed-spin "
                               "+ triplet; step = one ROKS CG iteration + forces"
                               % (head["npw"], head["nb"]),
                   "precision": args.tier, "bands": head["nb"], "grid": [96, 96, 96]},
        "roofline": head["roofline"],
        "kernels": head["kernels"],
        "h_apply_pipeline": head["h_apply_pipeline"],
    }
    if not args.no_extras:
        t32 = measure(system, rb.FP32, args.steps, args.warmup, table_steps=2)
        out["oxide_fp32_tier"] = {k: t32[k] for k in ("band_applies_per_s", "ms_per_step",
                                                       "roofline", "h_apply_pipeline")}
        tb = measure(system, rb.FP32_BF16X3, args.steps, args.warmup, table_steps=2)
        out["oxide_bf16x3_tier"] = {
            "arithmetic": "fp32 FFTs and potentials; projector products BF16x3 on the BF16 "
                          "matrix cores; band overlaps, Gram, rotation, energies fp64",
            **{k: tb[k] for k in ("band_applies_per_s", "ms_per_step", "roofline",
                                  "h_apply_pipeline")},
            "proj_bf3": tb["kernels"]["proj_bf3"]}
        tq = measure(inputs.with_overlap(system, 0.3), rb.FP64, args.steps, args.warmup,
                     table_steps=2)
        out["oxide_overlap"] = {
            "workload": "the same supercell with overlap coefficients q (S = 1 + sum q "
                        "|beta><beta|, q = 0.3 diag(1, 0.6, 0.4, 0.3) + 0.06 between the s "
                        "channels), fp64",
            **{k: tq[k] for k in ("band_applies_per_s", "ms_per_step", "roofline")},
            "cost_vs_s_equal_1": tq["ms_per_step"] / head["ms_per_step"]
            if args.tier == "fp64" else None}
        out["oxide_graph_cg"] = oxide_graph_report(system)
        mol = inputs.molecule_box()
        m = measure(mol, rb.FP64, max(args.steps, 20), args.warmup, table_steps=10)
        out["molecule_64"] = {
            "workload": "molecule-in-box: cubic 24 bohr, 64^3 grid, ecut 8.77 Ha, %d stored plane "
                        "waves, 20 atoms x 4 projectors, %d bands; step = one ROKS CG iteration "
                        "+ forces, fp64" % (m["npw"], m["nb"]),
            **{k: m[k] for k in ("band_applies_per_s", "ms_per_step", "roofline", "kernels",
                                 "h_apply_pipeline")}}
        if not args.no_converge:
            out["time_to_converge"] = converge_report(mol)
        if not args.no_batch:
            out["batch"] = batch_report()
            out["batch_apply_graph"] = graph_report_child()
            out["batch_cg_graph"] = cg_graph_report()
            out["batch_solve_graph"] = batch_solve_report()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(system)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
