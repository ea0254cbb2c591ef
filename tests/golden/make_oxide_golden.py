"""Write tests/golden/oxide_cg3.json: the oracle's first three CG iterations on
the rocksalt oxide-vacancy supercell (3 x 3 x 3 conventional cells, a = 8
bohr, one anion removed: 215 atoms, 96^3 grid, 432 bands, 1 720 projectors),
from the seeded start orthonormalised by Cholesky.

Calls only the oracle (and the seeded input descriptions).  Stored, per
iteration: E0, E1, the step length, the Fletcher-Reeves ratio, dE/d delta at
0, ||g_I|| and the open-shell coupling (Sec. II A: Eqs. orbital_update,
cg_search, gradient, prec_grad_I, prec_k, r_matrix_singlet); for the start
orbitals the diagonal of theta, the per-band ||g_I,n||^2 and sampled rows of
theta, R and A; for the orbitals before and after the three steps the probe
sums s_n = <r|psi_n> of every band (r: seeded random vector, full sphere)
and sampled coefficients; the Hellmann-Feynman forces after the third step
(Eq. force_hf).

Runs in ~15-30 min on one CPU socket:  python tests/golden/make_oxide_golden.py

With --overlap SCALE the species carry the overlap coefficients of
inputs.with_overlap(system, SCALE) (S = 1 + sum q |beta><beta|, Sec. II A),
the start is S-orthonormalised, and --steps CG iterations are stored in
tests/golden/oxide_overlap_cg<steps>.json:
python tests/golden/make_oxide_golden.py --overlap 0.3 --steps 1
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import roks as orc  # noqa: E402
from paper_2605_28637_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
PROBE_SEED = 31337
SAMPLE_BANDS = [0, 1, 107, 213, 214, 320, 427, 428, 429, 430, 431]
ROW_BANDS = [0, 427, 428, 429, 430, 431]


def sample_millers(m):
    """G = 0, the 12 smallest |G| and 11 with |G| near the cutoff (fixed
    choice by Miller index, independent of any storage order)."""
    order = np.lexsort((m.miller[:, 2], m.miller[:, 1], m.miller[:, 0], np.round(m.g2, 9)))
    small = [tuple(m.miller[i]) for i in order[:13]]
    big = [tuple(m.miller[i]) for i in order[-11:]]
    return [list(map(int, t)) for t in small + big]


def state_record(m, psi, probe, millers):
    look = {tuple(t): i for i, t in enumerate(m.miller)}
    idx = [look[tuple(t)] for t in millers]
    probes = np.real(np.conj(probe) @ psi.T)
    coef = {str(n): [[float(psi[n, i].real), float(psi[n, i].imag)] for i in idx]
            for n in SAMPLE_BANDS}
    return {"probe": probes.tolist(), "coef": coef}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--overlap", type=float, default=0.0)
    ap.add_argument("--steps", type=int, default=3)
    args = ap.parse_args()
    t0 = time.time()
    s = inputs.oxide_vacancy()
    if args.overlap:
        s = inputs.with_overlap(s, args.overlap)
        out_path = os.path.join(HERE, "oxide_overlap_cg%d.json" % args.steps)
    else:
        out_path = os.path.join(HERE, "oxide_cg%d.json" % args.steps)
    m = orc.Model(s)
    print("model: npw %d nproj %d nb %d (%.0f s)" % (m.npw, m.nproj, m.nb, time.time() - t0),
          flush=True)
    probe = inputs.gaussian_pairs(PROBE_SEED, 0, m.miller)
    millers = sample_millers(m)
    psi = orc.orthonormalize(inputs.random_coefficients(m.miller, m.cell, m.nb, s["seed"]), m)
    out = {"system": "oxide_vacancy(seed=%d)" % s["seed"], "overlap_scale": args.overlap,
           "probe_seed": PROBE_SEED,
           "sample_bands": SAMPLE_BANDS, "row_bands": ROW_BANDS, "millers": millers,
           "start": state_record(m, psi, probe, millers)}
    gr = orc.gradient(m, psi)
    print("start gradient (%.0f s)" % (time.time() - t0), flush=True)
    out["start"].update({
        "E": gr.pot.E, "E_L": gr.pot.E_L.tolist(),
        "theta_diag": np.diag(gr.theta).tolist(),
        "gI_norm2": np.real(np.sum(np.conj(gr.gI) * gr.gI, axis=1)).tolist(),
        "theta_rows": {str(n): gr.theta[n].tolist() for n in ROW_BANDS},
        "R_rows": {str(n): gr.R[n].tolist() for n in ROW_BANDS},
        "A_rows": {str(n): gr.A[n].tolist() for n in ROW_BANDS},
    })
    del gr
    st = orc.CGState(psi=psi)
    steps = []
    for it in range(args.steps):
        info = orc.pcg_step(m, st)
        steps.append({"E0": info.E0, "E1": info.E1, "delta": info.delta, "beta": info.beta,
                      "dE0": info.dE0, "norm_gI": info.norm_gI, "max_Rab": info.max_Rab,
                      "restarted": bool(info.restarted), "stalled": bool(info.stalled),
                      "evaluations": info.evaluations})
        print("step %d: %s (%.0f s)" % (it + 1, steps[-1], time.time() - t0), flush=True)
    out["steps"] = steps
    out["final"] = state_record(m, st.psi, probe, millers)
    out["final"]["forces"] = orc.forces(m, st.psi).tolist()
    print("forces (%.0f s)" % (time.time() - t0), flush=True)
    with open(out_path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", out_path)


if __name__ == "__main__":
    main()
