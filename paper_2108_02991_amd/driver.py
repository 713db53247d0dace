"""Projected-gradient loop over `sparkling_step` (the inner loop of Algorithm 1 at
one resolution level) with per-iteration JSON records.

    python -m paper_2108_02991_amd.driver --workload c5_loop --precision fp32_comp \\
        --iters 100 --out run.jsonl

Every record holds F, F^a, F^r, the step size, whether the Barzilai-Borwein
step was used, the constraint violations after projection and the wall time
of the step (HIP-synchronised).  The initial trajectory is projected once
before the first iteration.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import api, configs


def run(workload: configs.Workload, precision: str, iters: int, device="cuda:0",
        out=None, log_every: int = 1):
    """Runs `iters` projected gradient steps; returns the list of records."""
    dev = torch.device(device)
    a, b = api.alpha_beta(configs.GMAX, configs.SMAX, configs.RASTER_DT, configs.DWELL_DT,
                          workload.fov, workload.kmax, configs.GAMMA_BAR, workload.half_width)
    prm = api.Params(workload.n_shots, workload.n_samples, workload.grid, precision=precision,
                     half_width=workload.half_width, a_max=a, b_max=b, te_index=0,
                     n_pit=workload.n_pit)
    K = torch.tensor(workload.trajectory(), dtype=prm.dtype, device=dev)
    rho = torch.tensor(workload.density(), dtype=prm.dtype, device=dev)
    viol0 = api.project_(K, prm)
    state = api.StepState(prm, dev)
    records = []
    for it in range(iters):
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        info = api.step_(K, rho, prm, state, it, workload.eta_fixed)
        torch.cuda.synchronize(dev)
        rec = {"iter": it, "precision": precision, "F": info["F"], "Fa": info["Fa"],
               "Fr": info["Fr"], "eta": info["eta"], "bb_used": info["bb_used"],
               "viol": [float(v) for v in info["viol"]], "s": time.perf_counter() - t0}
        if it == 0:
            rec["viol_initial_projection"] = [float(v) for v in viol0]
        records.append(rec)
        if out is not None:
            out.write(json.dumps(rec) + "\n")
            out.flush()
        if log_every and (it % log_every == 0 or it == iters - 1):
            print(f"[driver] {precision} iter {it}: F={info['F']:.12e} eta={info['eta']:.5g} "
                  f"viol={np.round(info['viol'], 4).tolist()} {rec['s']:.3f}s",
                  file=sys.stderr, flush=True)
    F, _, _, _ = api.energy(K, rho, prm)
    records.append({"final_F": F, "precision": precision})
    if out is not None:
        out.write(json.dumps(records[-1]) + "\n")
        out.flush()
    return records, K


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c5_loop")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--log-every", type=int, default=10)
    args = ap.parse_args()
    w = configs.WORKLOADS[args.workload]
    precision = args.precision or w.precision
    iters = args.iters if args.iters is not None else w.n_iters
    api.load_library()
    out = open(args.out, "a") if args.out else None
    try:
        run(w, precision, iters, out=out, log_every=args.log_every)
    finally:
        if out is not None:
            out.close()


if __name__ == "__main__":
    main()
