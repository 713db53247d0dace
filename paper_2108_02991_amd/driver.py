"""Drivers over the C ABI: the projected-gradient loop at one resolution level
(`run`) and the multi-resolution strategy of Algorithm 1 (`multiresolution`),
with per-iteration JSON records.

    python -m paper_2108_02991_amd.driver --workload c5_loop --precision fp32_comp \\
        --iters 100 --out run.jsonl

Every record holds F, F^a, F^r, the discrepancy D = F - (1/2) sum rho rho H
(the density's self-energy is computed once), ||grad F||_2 at the step's input,
the step size, whether the Barzilai-Borwein step was used and its quotient
s.s/s.y before the clamp, the constraint violations after projection, the wall
time of the step (HIP-synchronised) and the time of each kernel kind (HIP
events).  The initial trajectory is projected once before the first
iteration.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import sys
import time

import numpy as np
import torch

from . import api, configs


def fixed_step(prm: api.Params, rho_mass: float, rule: str, eta_fixed: float) -> float:
    """The fixed step of the first iterations: the workload's value ("fixed"), or
    1/L from the Lipschitz bound of the regularised kernel ("lipschitz")."""
    if rule == "lipschitz":
        return 1.0 / api.lipschitz_bound(prm.p, prm.eps, rho_mass, prm.kernel)
    return eta_fixed


def run(workload: configs.Workload, precision: str, iters: int, device="cuda:0",
        out=None, log_every: int = 1, rotation_variant: bool = False, kernel: str = "distance",
        eps: float = 0.0, eta_rule: str = "fixed", graph: bool = False,
        far_field: tuple = (0, 5, 0), warm_duals: bool = False):
    """Runs `iters` projected gradient steps; returns the list of records.

    With graph=True the step runs as two captured HIP graphs (fixed-step and
    Barzilai-Borwein phases) with no host synchronisation between steps; a
    record is then written only at the logged iterations and at the end.
    With warm_duals=True every projection starts from the previous one's dual
    variables (spk_params.proj_duals) instead of from zero."""
    dev = torch.device(device)
    a, b = api.alpha_beta(configs.GMAX, configs.SMAX, configs.RASTER_DT, configs.DWELL_DT,
                          workload.fov, workload.kmax, configs.GAMMA_BAR, workload.half_width)
    prm = api.Params(workload.n_shots, workload.n_samples, workload.grid, precision=precision,
                     half_width=workload.half_width, eps=eps, a_max=a, b_max=b, te_index=0,
                     n_pit=workload.n_pit, rotation_variant=rotation_variant, kernel=kernel,
                     far_field_depth=far_field[0], far_field_order=far_field[1],
                     far_field_adaptive=int(far_field[2]) if len(far_field) > 2 else 0)
    rho_host = workload.density()
    K = torch.tensor(workload.trajectory(), dtype=prm.dtype, device=dev)
    rho = torch.tensor(rho_host, dtype=prm.dtype, device=dev)
    eta = fixed_step(prm, float(rho_host.sum()), eta_rule, workload.eta_fixed)
    if warm_duals:
        prm.proj_duals = api.new_duals(prm, dev)
    viol0 = api.project_(K, prm)
    if warm_duals:
        # the duals of the jittered start's projection are far from what the
        # nearly feasible iterates need: the loop's first projection starts cold
        prm.proj_duals.zero_()
    state = api.StepState(prm, dev)
    records = []
    if graph:
        return _run_graph(K, rho, prm, state, eta, iters, precision, viol0, out, log_every)
    self_energy = density_self_energy(K, rho, prm)
    api.timing_enable(True)
    for it in range(iters):
        torch.cuda.synchronize(dev)
        api.timing_reset()
        t0 = time.perf_counter()
        info = api.step_(K, rho, prm, state, it, eta)
        torch.cuda.synchronize(dev)
        wall = time.perf_counter() - t0
        rec = {"iter": it, "precision": precision, "F": info["F"], "Fa": info["Fa"],
               "Fr": info["Fr"], "D": info["F"] - self_energy,
               "grad_norm": float(torch.linalg.vector_norm(state.g_prev.double())),
               "eta": info["eta"], "bb_used": info["bb_used"],
               "bb_quotient": info["bb_quotient"],
               "viol": [float(v) for v in info["viol"]], "s": wall,
               "kernel_ms": kernel_ms()}
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
    api.timing_enable(False)
    F, _, _, _ = api.energy(K, rho, prm)
    records.append({"final_F": F, "final_D": F - self_energy, "precision": precision})
    if out is not None:
        out.write(json.dumps(records[-1]) + "\n")
        out.flush()
    return records, K


KERNEL_KINDS = {"repulsion": api.KIND_REPULSION, "attraction": api.KIND_ATTRACTION,
                "interpolation": api.KIND_INTERPOLATION, "projection": api.KIND_PROJECTION,
                "other": api.KIND_OTHER}


def kernel_ms() -> dict:
    """Milliseconds per kernel kind since the last timing reset."""
    return {name: api.timing_query(kind)[0] for name, kind in KERNEL_KINDS.items()}


def density_self_energy(K, rho, prm) -> float:
    """(1/2) sum_{u,v} rho_u rho_v H(x_u - x_v), the constant that separates the
    objective F from the discrepancy D (one energy call with the discrepancy)."""
    F, _, _, D = api.energy(K, rho, dataclasses.replace(prm, discrepancy=True))
    return F - D


def _run_graph(K, rho, prm, state, eta, iters, precision, viol0, out, log_every):
    dev = K.device
    torch.cuda.synchronize(dev)
    t_cap = time.perf_counter()
    graphs = {False: api.StepGraph(K, rho, prm, state, eta, barzilai_borwein=False),
              True: api.StepGraph(K, rho, prm, state, eta, barzilai_borwein=True)}
    torch.cuda.synchronize(dev)
    capture_s = time.perf_counter() - t_cap
    records = []
    t0 = time.perf_counter()
    for it in range(iters):
        g = graphs[it >= 20]
        g.replay()
        if (log_every and it % log_every == 0) or it == iters - 1:
            torch.cuda.synchronize(dev)
            info = api.info_dict(g.info)
            rec = {"iter": it, "precision": precision, "graph": True, "F": info["F"],
                   "bb_quotient": info["bb_quotient"],
                   "Fa": info["Fa"], "Fr": info["Fr"], "eta": info["eta"],
                   "bb_used": info["bb_used"], "viol": [float(v) for v in info["viol"]],
                   "elapsed_s": time.perf_counter() - t0}
            if it == 0:
                rec["viol_initial_projection"] = [float(v) for v in viol0]
                rec["capture_s"] = capture_s
            records.append(rec)
            if out is not None:
                out.write(json.dumps(rec) + "\n")
                out.flush()
            print(f"[driver] graph {precision} iter {it}: F={info['F']:.12e} "
                  f"eta={info['eta']:.5g} {rec['elapsed_s']:.3f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize(dev)
    total = time.perf_counter() - t0
    F, _, _, _ = api.energy(K, rho, prm)
    records.append({"final_F": F, "precision": precision, "graph": True,
                    "s_per_iter": total / max(iters, 1)})
    if out is not None:
        out.write(json.dumps(records[-1]) + "\n")
        out.flush()
    return records, K


def parse_far_field(spec):
    """'DEPTH,ORDER', 'DEPTH,ORDER,adaptive' (one refinement level) or
    'DEPTH,ORDER,adaptive=R' -> (depth, order, R); None -> off."""
    if not spec:
        return 0, 5, 0
    f = spec.split(",")
    ok = len(f) == 2 or (len(f) == 3 and (f[2] == "adaptive" or f[2].startswith("adaptive=")))
    if not ok:
        raise ValueError(f"far field spec {spec!r}: expected DEPTH,ORDER[,adaptive[=R]]")
    R = 0 if len(f) == 2 else (1 if f[2] == "adaptive" else int(f[2].split("=")[1]))
    return int(f[0]), int(f[1]), R


# Largest level (samples in all shots) whose repulsion is summed exactly when
# the far field is on: the far field has a floor of about 10 ms per gradient
# (tree, tables and the M2L's dependent chain) while the exact sweep takes
# p^2 / 4.4e12 s, so the two cross near 2e5 samples.  On c3's shots a whole
# step at 131,072 samples takes 4.9 ms exact against 9.9 ms with the far
# field; at 262,144 the exact repulsion alone (15.6 ms) exceeds the far-field
# step (10.9 ms).
EXACT_MAX_P = 1 << 17


def _level_depth(depth: int, d: int, p: int, exact_max_p: int = EXACT_MAX_P) -> int:
    """Octree depth of the far field at decimation level d with p samples:
    8^depth leaves for p / 2^d samples keep about as many samples per leaf when
    the depth drops by one every three halvings; below depth 2, or at most
    exact_max_p samples, the sum is exact."""
    if depth == 0 or p <= exact_max_p:
        return 0
    dd = depth - (d + 1) // 3
    return dd if dd >= 2 else 0


def multiresolution(K0: torch.Tensor, rho: torch.Tensor, prm_full: api.Params, levels: int,
                    n_git: int, final_level: bool = True, eta_scale: float = 0.25, out=None,
                    log_every: int = 0, eta_rule: str = "fixed", warm_duals: bool = False,
                    exact_max_p: int = EXACT_MAX_P):
    """Algorithm 1 (multi-resolution SPARKLING) on the GPU.

    K0 holds the coarsest shots, prm_full.n_samples >> levels samples each.  At
    decimation level d the per-raster bounds are prm_full.a_max * 2^d and
    prm_full.b_max * 2^d (the scaling printed with Algorithm 1), n_git
    projected gradient steps run with a fixed step for the first 20 and
    Barzilai-Borwein after (state reset per level, eta_fixed from the level's
    p), and the result is up-sampled to twice the samples as the warm start of
    the next level.  With final_level=True the full resolution (d = 0) is
    optimised as well.  eta_rule="lipschitz" takes the fixed step 1/L of the
    regularised kernel at each level instead.  warm_duals=True carries the
    projection's dual variables from step to step within a level.  With the
    far field on, levels of at most exact_max_p samples are summed exactly.
    Returns the final K and the per-iteration records.
    """
    if prm_full.n_samples % (1 << levels):
        raise ValueError("n_samples must be divisible by 2^levels")
    Ns = prm_full.n_samples >> levels
    K = K0
    records = []
    for d in range(levels, -1 if final_level else 0, -1):
        depth = _level_depth(prm_full.far_field_depth, d, prm_full.n_shots * Ns, exact_max_p)
        prm = api.Params(prm_full.n_shots, Ns, prm_full.grid, precision=prm_full.precision,
                         half_width=prm_full.half_width, eps=prm_full.eps,
                         a_max=prm_full.a_max * 2.0 ** d, b_max=prm_full.b_max * 2.0 ** d,
                         te_index=prm_full.te_index, n_pit=prm_full.n_pit,
                         rotation_variant=prm_full.rotation_variant, kernel=prm_full.kernel,
                         attraction_field=prm_full.attraction_field,
                         far_field_depth=depth,
                         far_field_order=prm_full.far_field_order,
                         far_field_adaptive=prm_full.far_field_adaptive if depth > 0 else 0)
        if K.shape[1] != prm.p:
            raise ValueError(f"level {d}: K has {K.shape[1]} samples, expected {prm.p}")
        eta = fixed_step(prm, float(rho.sum().item()), eta_rule,
                         eta_scale * (2.0 * prm.half_width) * float(prm.p) ** (2.0 / 3.0))
        state = api.StepState(prm, K.device)
        if warm_duals:      # the dual state is per level (its shape follows N_s)
            prm.proj_duals = api.new_duals(prm, K.device)
        for it in range(n_git):
            torch.cuda.synchronize(K.device)
            t0 = time.perf_counter()
            info = api.step_(K, rho, prm, state, it, eta)
            torch.cuda.synchronize(K.device)
            rec = {"level": d, "iter": it, "n_samples": Ns, "F": info["F"], "Fa": info["Fa"],
                   "Fr": info["Fr"], "eta": info["eta"], "bb_used": info["bb_used"],
                   "bb_quotient": info["bb_quotient"],
                   "viol": [float(v) for v in info["viol"]], "s": time.perf_counter() - t0}
            records.append(rec)
            if out is not None:
                out.write(json.dumps(rec) + "\n")
                out.flush()
            if log_every and (it % log_every == 0 or it == n_git - 1):
                print(f"[driver] level {d} iter {it}: F={info['F']:.12e} eta={info['eta']:.5g}",
                      file=sys.stderr, flush=True)
        if d > 0:
            K = api.upsample(K, prm)
            Ns *= 2
    return K, records


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c5_loop")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--log-every", type=int, default=10)
    ap.add_argument("--levels", type=int, default=0,
                    help="run Algorithm 1 with this many decimation levels (0 = single level)")
    ap.add_argument("--field", action="store_true",
                    help="evaluate the attraction by the grid interpolant")
    ap.add_argument("--rotation-variant", action="store_true",
                    help="per-axis gradient and slew bounds instead of Euclidean ones")
    ap.add_argument("--kernel", choices=["distance", "log"], default="distance")
    ap.add_argument("--eps", type=float, default=0.0, help="kernel regulariser")
    ap.add_argument("--eta", choices=["fixed", "lipschitz"], default="fixed",
                    help="fixed step of the first iterations: the workload's, or 1/L")
    ap.add_argument("--graph", action="store_true",
                    help="run the single-level loop as captured HIP graphs")
    ap.add_argument("--warm-duals", action="store_true",
                    help="start every projection from the previous one's dual variables")
    ap.add_argument("--n-pit", type=int, default=None,
                    help="projection iterations (default: the workload's)")
    ap.add_argument("--far-field", default=None, metavar="DEPTH,ORDER[,adaptive[=R]]",
                    help="repulsion by the Chebyshev fast multipole method (e.g. 5,6 or "
                         "5,6,adaptive=2)")
    ap.add_argument("--exact-max-p", type=int, default=EXACT_MAX_P,
                    help="with --levels and --far-field: levels of at most this many samples "
                         "are summed exactly")
    args = ap.parse_args()
    w = configs.WORKLOADS[args.workload]
    if args.n_pit is not None:
        w = dataclasses.replace(w, n_pit=args.n_pit)
    precision = args.precision or w.precision
    iters = args.iters if args.iters is not None else w.n_iters
    api.load_library()
    ffd, ffo, ffa = parse_far_field(args.far_field)
    out = open(args.out, "a") if args.out else None
    try:
        if args.levels == 0 and not args.field:
            run(w, precision, iters, out=out, log_every=args.log_every,
                rotation_variant=args.rotation_variant, kernel=args.kernel, eps=args.eps,
                eta_rule=args.eta, graph=args.graph, far_field=(ffd, ffo, ffa),
                warm_duals=args.warm_duals)
        else:
            dev = torch.device("cuda:0")
            a, b = api.alpha_beta(configs.GMAX, configs.SMAX, configs.RASTER_DT,
                                  configs.DWELL_DT, w.fov, w.kmax, configs.GAMMA_BAR,
                                  w.half_width)
            prm = api.Params(w.n_shots, w.n_samples, w.grid, precision=precision,
                             half_width=w.half_width, a_max=a, b_max=b, te_index=0,
                             n_pit=w.n_pit, rotation_variant=args.rotation_variant,
                             kernel=args.kernel, eps=args.eps, far_field_depth=ffd,
                             far_field_order=ffo, far_field_adaptive=ffa)
            from . import inputs
            K0 = inputs.radial_spokes(w.n_shots, w.n_samples >> args.levels, w.half_width,
                                      w.seed, w.jitter)
            K0 = torch.tensor(K0, dtype=prm.dtype, device=dev)
            rho = torch.tensor(w.density(), dtype=prm.dtype, device=dev)
            t0 = time.perf_counter()
            if args.field:
                prm.attraction_field = api.attraction_field(rho, prm)
                torch.cuda.synchronize(dev)
                print(f"[driver] node field in {time.perf_counter() - t0:.2f} s",
                      file=sys.stderr, flush=True)
            K, recs = multiresolution(K0, rho, prm, args.levels, iters, out=out,
                                      log_every=args.log_every, eta_rule=args.eta,
                                      warm_duals=args.warm_duals, exact_max_p=args.exact_max_p)
            torch.cuda.synchronize(dev)
            total = time.perf_counter() - t0
            F, _, _, _ = api.energy(K, rho, prm)
            summary = {"workload": w.name, "levels": args.levels, "n_git": iters,
                       "n_pit": w.n_pit, "precision": precision,
                       "field": args.field, "far_field": args.far_field,
                       "exact_max_p": args.exact_max_p, "total_s": total, "final_F": F,
                       "s_per_level": {str(d): sum(r["s"] for r in recs if r["level"] == d)
                                       for d in range(args.levels, -1, -1)}}
            print(json.dumps(summary), flush=True)
            if out is not None:
                out.write(json.dumps(summary) + "\n")
    finally:
        if out is not None:
            out.close()


if __name__ == "__main__":
    main()
