#!/usr/bin/env python
"""Benchmark of the ROKS hot path on one MI355X.

Workload: the molecule-in-box cell (cubic 24 bohr box, 64^3 grid at the
grid-rule cutoff of 8.77 Ha, 8 539 stored plane waves, 20 seeded atoms with
4 Gaussian projectors each, 40 bands = 36 closed + 2 open + 2 virtual,
mixed-spin and triplet configurations of the singlet), FP64.

One step = one pass of the whole hot path: densities, potentials and
energies of both configurations, F^n|n> for every band (the band
H-applications), theta / g_I / R / A, the projected Teter preconditioner,
Fletcher-Reeves directions, the line search (Cholesky orthonormalisation,
rotation, trial energies), the commit, and the forces.  value = band
H-applications per second over the timed steps (nbands per step).

Kernel times come from HIP events the library records on its own stream
(roks_timing_*), with the algorithmic bytes and flops of every launch.

Prints ONE JSON line.  Inputs are resident on the GPU when timing starts.
"""
import argparse
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
KERNELS = ("zpass_bwd", "plane_apply", "plane_density", "zpass_fwd", "fft3d", "gemm_wdot",
           "gemm_expand", "xc")


def roofline(name, k):
    """Roofline entry of one kernel family from its summed time and work."""
    if not k["launches"] or k["ms_total"] <= 0:
        return None
    avg_s = k["ms_total"] * 1e-3 / k["launches"]
    by, fl = k["bytes"] / k["launches"], k["flops"] / k["launches"]
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if fl > 0 and fl / by > ridge:
        ach = fl / avg_s / 1e12
        return {"bound": "mfma", "kernel": name, "achieved": ach, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS, "traffic": None,
                "flops_per_launch": fl, "avg_launch_ms": avg_s * 1e3}
    ach = by / avg_s / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "bytes_per_launch": by,
            "avg_launch_ms": avg_s * 1e3}


def cpu_baseline(system):
    """The oracle, as it stands, on a bounded sample: one CG iteration of the
    same workload from the same start, on one host thread."""
    from threadpoolctl import threadpool_limits

    from oracle import roks as orc
    with threadpool_limits(limits=1):
        m = orc.Model(system)
        psi = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, system["seed"]))
        st = orc.CGState(psi=psi)
        t0 = time.perf_counter()
        orc.pcg_step(m, st)
        dt = time.perf_counter() - t0
    return {"value": m.nb / dt, "unit": "band H-applies/s", "cores": 1, "kind": "oracle",
            "sample": "one oracle CG iteration (%d band applications of F^n plus line search) "
                      "on the same 64^3 / 40-band workload, single host thread, %.1f s"
                      % (m.nb, dt)}


def time_to_converge(system, tol=1e-6, maxiter=600):
    """Ground state first, then the singlet from the ground-state orbitals."""
    gs = inputs.with_configuration(system, "gs")
    t0 = time.perf_counter()
    rg = rb.Roks(gs)
    rg.set_coeffs(inputs.random_coefficients(rg.miller(), gs["cell"], rg.nb, gs["seed"]), True)
    ig, itg = rg.solve(tol=tol, maxiter=maxiter)
    c = rg.get_coeffs()
    rg.close()
    r = rb.Roks(system)
    r.set_coeffs(c, True)
    ie, ite = r.solve(tol=tol, maxiter=maxiter)
    F = r.forces()
    r.close()
    dt = time.perf_counter() - t0
    return {"seconds": dt, "gs_iterations": itg, "singlet_iterations": ite, "E_gs": ig["E1"],
            "E_singlet": ie["E1"], "excitation_Ha": ie["E1"] - ig["E1"],
            "max_force": float(np.abs(F).max()), "tol_Ha": tol, "dtype": "f64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-converge", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    system = inputs.molecule_box()
    r = rb.Roks(system)
    r.set_coeffs(inputs.random_coefficients(r.miller(), system["cell"], r.nb, system["seed"]), True)
    for _ in range(args.warmup):
        r.pcg_step()
        r.forces()
    r.synchronize()
    r.timing_enable(True)
    r.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r.pcg_step()
        r.forces()
    r.synchronize()
    elapsed = time.perf_counter() - t0
    kernels = {k: r.timing_read(k) for k in KERNELS}
    r.timing_enable(False)
    nb, npw = r.nb, r.npw
    r.close()

    roofs = {k: roofline(k, v) for k, v in kernels.items()}
    dom = max((k for k in kernels if roofs[k]), key=lambda k: kernels[k]["ms_total"])
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

    out = {
        "metric": "band H-applies/s",
        "value": nb * args.steps / elapsed,
        "unit": "band H-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "molecule-in-box: cubic 24 bohr, 64^3 grid, ecut 8.77 Ha, "
                               "%d stored plane waves, 20 atoms x 4 projectors, %d bands "
                               "(36 closed + 2 open + 2 virtual), mixed-spin + triplet; step = "
                               "one ROKS CG iteration + forces" % (npw, nb),
                   "precision": "fp64", "bands": nb, "grid": [64, 64, 64]},
        "roofline": roofs[dom],
        "kernels": {k: dict(v, roofline_frac=(roofs[k] or {}).get("frac"))
                    for k, v in kernels.items()},
        "h_apply_pipeline": {"achieved_GBs": happ_bytes / (happ_ms * 1e-3) / 1e9 if happ_ms else None,
                             "frac_hbm": (happ_bytes / (happ_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                          if happ_ms else None),
                             "ms_per_all_band_apply": happ_ms / max(1, na),
                             "band_applies_per_s": nb * na / (happ_ms * 1e-3) if happ_ms else None},
    }
    if not args.no_converge:
        out["time_to_converge"] = time_to_converge(system)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(system)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
