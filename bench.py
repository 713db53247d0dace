"""Benchmark: projected-gradient SPARKLING steps at 8.4 M samples on one MI355X.

A step is one pass of the whole hot path through the C ABI (sparkling_step):
all-pairs repulsion sweep, attraction sweep against the 192^3 density,
slab combines, gradient and energies, the step-size policy, the descent
update, the per-shot projection and the constraint check.  Inputs are
synthetic (seeded jittered radial spokes, radial density) and resident in HBM
before the timed region.

The jittered spokes are projected once before the warm-up (--init-pit
iterations, untimed), as the optimisation loop starts from projected shots;
every timed step then runs the workload's n_pit projection iterations.

Warm-up and timed steps each stop at a wall budget (--warmup-budget,
--time-budget): after a step, no further step starts if one more of the mean
length would pass the budget.  An exact 8.4M-sample step takes about 26 s, so
the default 20 timed steps become about 4; the line reports the steps actually
timed (`steps`) beside the requested ones (`steps_requested`).

Prints one JSON line.  `value` is pair interactions per second over the whole
step (p^2 repulsion + p*G^3 attraction per step); the roofline object is for
the dominant kernel (the repulsion sweep), timed live with HIP events on the
stream it runs on, against the FP32 vector peak and, under `ceiling`, against
the measured issue rate of the pair's own instruction mix.  The CPU baseline is the FP64 oracle timed on a bounded
sample of targets of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X FP32 vector peak (packed FP32, 256 CU x 2.4 GHz).
FP32_VECTOR_PEAK_TFLOPS = 157.3
# Algorithmic flops per pair of the sweeps with energy: 3 subtractions, 5 for
# |d|^2, 1 reciprocal square root, 6 for the three force FMAs, 2 for the
# energy FMA (repulsion); the attraction adds 1 for the density weight.  The
# log kernel swaps the reciprocal square root for a reciprocal and the energy
# FMA for a log2 and an add: the same count.
FLOP_PER_PAIR_REPULSION = 17
# Without the per-pair energy term (--energy-from-force: F^r from the forces).
FLOP_PER_PAIR_REPULSION_NO_ENERGY = 15
FLOP_PER_PAIR_ATTRACTION = 18


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "repulsion_sweep_c3_traffic.md")
SWEEP_SOURCES = [os.path.join(ROOT, "paper_2108_02991_amd", "csrc", f)
                 for f in ("sweep.hip", "sweep.h")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class EngineClock:
    """The GPU's shader (GFX) clock, sampled through amd-smi's metrics every
    `period_s` while the timed steps run (the published peaks assume 2.4 GHz).
    All amd-smi calls run on a daemon thread, so the benchmark never waits on
    the library: `stop()` waits at most a few seconds for the thread.
    `result()` gives the median, mean, minimum and maximum in MHz over the
    samples (each the mean of the per-XCD clocks), or None when the library or
    the device's metrics are not reachable (`error` then says why) or the timed
    region ended before the first sample."""

    def __init__(self, period_s: float = 0.1):
        self.period = period_s
        self.samples: list[float] = []
        self.error = None
        self._stop = threading.Event()
        self._thread = None

    def start(self, device_index: int = 0) -> "EngineClock":
        try:
            import torch
            bus = getattr(torch.cuda.get_device_properties(device_index), "pci_bus_id", None)
        except Exception as e:   # noqa: BLE001  (reported, never fatal)
            self.error = f"{type(e).__name__}: {e}"
            return self
        self._thread = threading.Thread(target=self._run, args=(bus,), daemon=True)
        self._thread.start()
        return self

    @staticmethod
    def _read(smi, handle) -> float:
        m = smi.amdsmi_get_gpu_metrics_info(handle)
        clocks = m.get("current_gfxclks")
        valid = [float(c) for c in (clocks if isinstance(clocks, list) else [])
                 if isinstance(c, (int, float)) and 0 < c < 10000]
        if valid:
            return sum(valid) / len(valid)
        c = m.get("current_gfxclk")
        if isinstance(c, (int, float)) and 0 < c < 10000:
            return float(c)
        raise RuntimeError("no GFX clock in the device metrics")

    def _run(self, bus):
        try:
            import amdsmi
            amdsmi.amdsmi_init()
        except Exception as e:   # noqa: BLE001
            self.error = f"{type(e).__name__}: {e}"
            return
        try:
            handles = amdsmi.amdsmi_get_processor_handles()
            match = [h for h in handles if bus is not None
                     and int(amdsmi.amdsmi_get_gpu_device_bdf(h).split(":")[1], 16) == bus]
            if len(match) != 1:
                match = handles if len(handles) == 1 else []
            if not match:
                raise RuntimeError(f"no unique amd-smi device for PCI bus {bus}")
            self._read(amdsmi, match[0])    # reachable? (before the work starts: not a sample)
            while not self._stop.wait(self.period):
                try:
                    self.samples.append(self._read(amdsmi, match[0]))
                except Exception:   # noqa: BLE001  (a missed sample)
                    pass
        except Exception as e:   # noqa: BLE001
            self.error = f"{type(e).__name__}: {e}"
        finally:
            try:
                amdsmi.amdsmi_shut_down()
            except Exception:   # noqa: BLE001
                pass

    def stop(self, wait_s: float = 5.0):
        self._stop.set()
        if self._thread is not None:
            self._thread.join(wait_s)
            if self._thread.is_alive():
                self.error = self.error or "clock sampler still busy after the timed region"

    def result(self):
        samples = list(self.samples)
        if not samples:
            return None
        mean = sum(samples) / len(samples)
        return {"mhz_median": float(np.median(samples)), "mhz_mean": mean,
                "mhz_min": min(samples), "mhz_max": max(samples),
                "samples": len(samples), "period_s": self.period,
                "source": "amd-smi gpu metrics (mean of the per-XCD GFX clocks) during the "
                          "timed steps",
                "fp32_peak_at_median_clock_tflops":
                    FP32_VECTOR_PEAK_TFLOPS * float(np.median(samples)) / 2400.0}


def sweep_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload: str, precision: str, kernel: str = "distance",
                     energy: bool = True, pairs_per_launch: float | None = None):
    """HBM bytes per repulsion launch from the committed counter summary, or None
    when the summary is missing, is for another workload or another variant of
    the sweep (kernel, per-pair energy on or off), for launches of another size
    (pairs_per_launch, when given), or the sweep sources changed since the
    counters were taken."""
    try:
        with open(TRAFFIC_RECORD) as f:
            rec = dict(line[2:].split(": ", 1) for line in f.read().splitlines()
                       if line.startswith("- ") and ": " in line)
    except OSError:
        return None
    if (rec.get("source_sha256") != sweep_source_hash() or rec.get("workload") != workload
            or rec.get("precision") != precision or rec.get("kernel", "distance") != kernel
            or rec.get("energy") != ("true" if energy else "false")):
        return None
    if pairs_per_launch is not None and (
            "pairs_per_launch" not in rec
            or abs(float(rec["pairs_per_launch"]) - pairs_per_launch) > 1e-6 * pairs_per_launch):
        return None
    return float(rec["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3_fp32_comp_8p4M")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU time budget of the oracle baseline (0 = skip)")
    ap.add_argument("--fp64-fraction", type=float, default=1.0 / 16,
                    help="fraction of targets of the plain-FP64 comparison run (0 = skip)")
    ap.add_argument("--attraction", choices=["direct", "field"], default="direct",
                    help="attraction by the direct sum over the density cells (default) or by "
                         "trilinear interpolation of a precomputed node field")
    ap.add_argument("--kernel", choices=["distance", "log"], default="distance",
                    help="pair kernel H: the distance |d| (default) or log(|d|^2 + eps^2)/2")
    ap.add_argument("--eps", type=float, default=None,
                    help="kernel regulariser (default 0 for the distance kernel, a quarter "
                         "of the mean sample spacing for the log kernel)")
    ap.add_argument("--eta", choices=["fixed", "lipschitz"], default=None,
                    help="fixed step: the workload's (default, distance kernel) or 1/L from "
                         "the Lipschitz bound (default for the log kernel; needs eps > 0)")
    ap.add_argument("--far-field", default=None, metavar="DEPTH,ORDER[,adaptive[=R]]",
                    help="repulsion by the Chebyshev fast multipole method (e.g. 5,6 or "
                         "5,6,adaptive=2) instead of all p^2 pairs; value is then an "
                         "equivalent rate and roofline null")
    ap.add_argument("--time-budget", type=float, default=120.0,
                    help="wall seconds of the timed region: after each step, timing stops "
                         "early if one more step of the mean length would pass this budget "
                         "(at least one step is timed)")
    ap.add_argument("--warmup-budget", type=float, default=30.0,
                    help="wall seconds of warm-up steps, by the same rule (at least one step "
                         "when --warmup > 0)")
    ap.add_argument("--energy-from-force", action="store_true",
                    help="F^r from the repulsion forces (Euler's theorem for H = |d|): the "
                         "sweep skips its per-pair energy term (15 flop/pair)")
    ap.add_argument("--init-pit", type=int, default=3000,
                    help="projection iterations of the one untimed projection of the initial "
                         "trajectory before the warm-up, as the optimisation loop starts from "
                         "projected shots (0 = start from the raw jittered spokes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, run a plain 1 GiB device copy three times "
                         "(reference dispatches for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the path runs on one GPU only; multi-GPU runs are not supported "
              f"(asked for {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2108_02991_amd as spk
    from paper_2108_02991_amd import configs, driver

    w = configs.WORKLOADS[args.workload]
    precision = args.precision or w.precision
    dev = torch.device("cuda:0")
    spk.load_library()
    a, b = spk.alpha_beta(configs.GMAX, configs.SMAX, configs.RASTER_DT, configs.DWELL_DT,
                          w.fov, w.kmax, configs.GAMMA_BAR, w.half_width)
    p_total = w.n_shots * w.n_samples
    eps = args.eps if args.eps is not None else (
        0.25 * 2 * w.half_width / p_total ** (1.0 / 3.0) if args.kernel == "log" else 0.0)
    ff_depth, ff_order, ff_adaptive = driver.parse_far_field(args.far_field)
    prm = spk.Params(w.n_shots, w.n_samples, w.grid, precision=precision,
                     half_width=w.half_width, eps=eps, a_max=a, b_max=b, te_index=0,
                     n_pit=w.n_pit, kernel=args.kernel, far_field_depth=ff_depth,
                     far_field_order=ff_order, far_field_adaptive=ff_adaptive,
                     energy_from_force=args.energy_from_force)
    p, M = prm.p, w.n_voxels

    log(f"workload {w.name}: p={p} G={w.grid} precision={precision} kernel={args.kernel} "
        f"eps={eps:.4g}")
    K_host = w.trajectory()
    rho_host = w.density()
    eta_rule = args.eta or ("lipschitz" if args.kernel == "log" else "fixed")
    eta = (1.0 / spk.lipschitz_bound(p, eps, float(rho_host.sum()), args.kernel)
           if eta_rule == "lipschitz" else w.eta_fixed)
    K = torch.tensor(K_host, dtype=prm.dtype, device=dev)
    rho = torch.tensor(rho_host, dtype=prm.dtype, device=dev)
    state = spk.StepState(prm, dev)
    init_viol = None
    if args.init_pit > 0:
        # the loop's starting point: the jittered spokes projected once (untimed)
        init_viol = spk.project_(K, dataclasses.replace(prm, n_pit=args.init_pit))
        log(f"initial trajectory projected ({args.init_pit} iterations): violations "
            f"{np.round(init_viol, 4).tolist()}")
    spk.workspace(prm, dev)
    field_s = None
    if args.attraction == "field":
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prm.attraction_field = spk.attraction_field(rho, prm)
        torch.cuda.synchronize()
        field_s = time.perf_counter() - t0
        log(f"node field precomputed in {field_s:.2f} s")

    # code-object load and first-launch costs, on a tiny problem in another
    # precision form (not a step; keeps the timed kernels' launch counts clean)
    other = "fp32_naive" if precision != "fp32_naive" else "fp32_comp"
    tiny = spk.Params(2, 8, 2, precision=other, a_max=a, b_max=b, n_pit=2)
    Kt = torch.zeros((3, 16), dtype=torch.float32, device=dev)
    spk.step_(Kt, torch.full((8,), 0.125, dtype=torch.float32, device=dev), tiny,
              spk.StepState(tiny, dev), 0, 1.0)
    torch.cuda.synchronize()
    log("inputs resident, kernels loaded")

    # issue bound of the repulsion pair on this device from measured component
    # rates (register-only probes, untimed region): what the sweep's fraction
    # is also read against
    probe = None
    if (not ff_depth and args.kernel == "distance" and precision == "fp32_comp"
            and not args.energy_from_force):
        try:
            probe = spk.pair_issue_bound(device=dev)
            log(f"pair issue bound: {probe['pairs_per_s']:.4g} pairs/s = "
                f"{probe['tflops_at_17']:.2f} TFLOP/s at 17 flop/pair (reciprocal square root "
                f"{probe['rsqrt_in_fma_slots']:.2f} FMA slots)")
        except Exception as e:   # noqa: BLE001  (a calibration; the line is kept without it)
            log(f"pair issue bound not measured: {type(e).__name__}: {e}")

    # Warm-up and timed steps each stop at a wall budget: an exact c3 step
    # takes about 26 s, so the requested counts may not fit.  Each step ends
    # with a host read of its info (sparkling_step synchronises the stream).
    it = 0
    warm = 0
    tw = time.perf_counter()
    while warm < args.warmup:
        spk.step_(K, rho, prm, state, it, eta)
        it += 1
        warm += 1
        el = time.perf_counter() - tw
        log(f"warmup step {warm} done ({el:.1f} s)")
        if el + el / warm > args.warmup_budget:
            break
    torch.cuda.synchronize()

    spk.timing_reset()
    spk.timing_enable(True)
    infos = []
    clock = EngineClock().start(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while len(infos) < args.steps:
        infos.append(spk.step_(K, rho, prm, state, it, eta))
        it += 1
        el = time.perf_counter() - t0
        log(f"step {it} done ({el:.1f} s): F={infos[-1]['F']:.9e} eta={infos[-1]['eta']:.4g}")
        if el + el / len(infos) > args.time_budget:
            break
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    clock.stop()
    spk.timing_enable(False)
    if clock.error:
        log(f"engine clock not sampled: {clock.error}")
    steps = len(infos)
    if steps < args.steps:
        log(f"timed {steps} of {args.steps} requested steps within the {args.time_budget:.0f} s "
            "budget")

    kern = {}
    for name, kind in (("repulsion", spk.KIND_REPULSION), ("attraction", spk.KIND_ATTRACTION),
                       ("projection", spk.KIND_PROJECTION), ("other", spk.KIND_OTHER),
                       ("interpolation", spk.KIND_INTERPOLATION)):
        ms, n, pairs = spk.timing_query(kind)
        kern[name] = {"ms": ms, "launches": n, "pairs": pairs}

    pairs_per_step = float(p) * p + (float(p) * M if args.attraction == "direct" else 0.0)
    ms_per_step = 1e3 * elapsed / steps
    value = pairs_per_step * steps / elapsed

    rep = kern["repulsion"]
    rep_avg_ms = rep["ms"] / max(rep["launches"], 1)
    rep_pairs_per_launch = rep["pairs"] / max(rep["launches"], 1)
    flop_rep = (FLOP_PER_PAIR_REPULSION_NO_ENERGY if args.energy_from_force
                else FLOP_PER_PAIR_REPULSION)
    achieved = flop_rep * rep_pairs_per_launch / (rep_avg_ms * 1e-3) / 1e12
    att = kern["attraction"]
    att_tflops = (FLOP_PER_PAIR_ATTRACTION * att["pairs"] / (att["ms"] * 1e-3) / 1e12
                  if att["ms"] > 0 else None)
    grad_ms = (rep["ms"] + att["ms"] + kern["interpolation"]["ms"] + kern["other"]["ms"]) / steps

    result = {
        "metric": "pair-interactions/s & sec per gradient eval at 8.4M samples, FP32-comp vs FP64",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "time_budget_s": args.time_budget,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "plain_fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_shots": w.n_shots, "n_samples": w.n_samples, "p": p,
                   "grid": w.grid, "precision": precision, "n_pit": w.n_pit,
                   "kernel": args.kernel, "eps": eps, "eta": eta_rule,
                   "attraction": args.attraction, "pairs_per_step": pairs_per_step,
                   "far_field": ({"depth": ff_depth, "order": ff_order, "adaptive": ff_adaptive}
                                 if ff_depth else None)},
        "s_per_grad_eval": grad_ms / 1e3,
        "kernels": {
            "repulsion": {"ms_per_step": rep["ms"] / steps, "launches_per_step":
                          rep["launches"] / steps, "avg_launch_ms": rep_avg_ms,
                          "pairs_per_s": rep["pairs"] / (rep["ms"] * 1e-3), "tflops": achieved},
            "attraction": {"ms_per_step": att["ms"] / steps, "launches_per_step":
                           att["launches"] / steps,
                           "pairs_per_s": att["pairs"] / (att["ms"] * 1e-3) if att["ms"] else None,
                           "tflops": att_tflops},
            "interpolation_ms_per_step": kern["interpolation"]["ms"] / steps,
            "field_precompute_s": field_s,
            "projection_ms_per_step": kern["projection"]["ms"] / steps,
            "other_ms_per_step": kern["other"]["ms"] / steps,
        },
        "roofline": ({"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                      "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                      "traffic": recorded_traffic(w.name, precision, args.kernel,
                                                  not args.energy_from_force,
                                                  rep_pairs_per_launch),
                      "ceiling": ({"kind": "issue bound of the pair from measured component "
                                           "rates: its 10 FP32 instructions at their stream "
                                           "rate plus one reciprocal square root at its cost "
                                           "(spk_probe_pair_mix, registers only)",
                                   "achieved": probe["tflops_at_17"],
                                   "frac_of_peak": probe["tflops_at_17"] / FP32_VECTOR_PEAK_TFLOPS,
                                   "kernel_frac_of_ceiling": achieved / probe["tflops_at_17"],
                                   "rsqrt_in_fma_slots": probe["rsqrt_in_fma_slots"],
                                   "fixed_order_mix_pairs_per_s":
                                       probe["fixed_order_mix_pairs_per_s"]}
                                  if probe else None)}
                     if not ff_depth else None),
        "engine_clock": clock.result(),
        "last_step": {k: (v.tolist() if isinstance(v, np.ndarray) else v)
                      for k, v in infos[-1].items()},
        "initial_projection": ({"n_pit": args.init_pit, "viol": init_viol.tolist()}
                               if init_viol is not None else None),
    }

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst

    if ff_depth:
        result["value_kind"] = ("equivalent: the all-pairs interactions a step stands for, per "
                                "second; the far field approximates the repulsion")
    # The comparison legs run after the timed region; a failure in one is
    # recorded in the line instead of losing it.
    if args.fp64_fraction > 0 and precision != "plain_fp64" and args.attraction == "direct":
        try:
            result["fp64_plain"] = fp64_comparison(spk, torch, w, prm, K, rho,
                                                   args.fp64_fraction, dev)
        except Exception as e:   # noqa: BLE001
            result["fp64_plain"] = {"error": f"{type(e).__name__}: {e}"}

    if args.cpu_seconds > 0:
        try:
            result["cpu_baseline"] = cpu_baseline(w, K, rho, args.cpu_seconds,
                                                  field=args.attraction == "field", eps=eps,
                                                  kernel=args.kernel)
        except Exception as e:   # noqa: BLE001
            result["cpu_baseline"] = {"error": f"{type(e).__name__}: {e}"}

    print(json.dumps(result), flush=True)


def fp64_comparison(spk, torch, w, prm, K, rho, fraction, dev):
    """Plain-FP64 gradient on a leading block of targets, against every source.

    Times the FP64 form on the same stored inputs (widened exactly) and reports
    its rate, the full-gradient time that rate implies, and the relative L2
    difference of the FP32-compensated rows from the FP64 rows.
    """
    p = prm.p
    nt = max(1024, int(p * fraction))
    nt = min(nt, p)
    prm64 = spk.Params(prm.n_shots, prm.n_samples, prm.grid, precision="plain_fp64",
                       half_width=prm.half_width, eps=prm.eps, kernel=prm.kernel)
    K64 = K.double()
    rho64 = rho.double()
    spk.workspace(prm64, dev)
    log(f"fp64 comparison on {nt} targets")
    spk.timing_reset()
    spk.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g64 = spk.grad(K64, rho64, prm64, tgt=(0, nt))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    spk.timing_enable(False)
    rep_ms, _, rep_pairs = spk.timing_query(spk.KIND_REPULSION)
    g32 = spk.grad(K, rho, prm, tgt=(0, nt))
    torch.cuda.synchronize()
    d = (g32.double() - g64).norm().item() / g64.norm().item()
    pairs = float(nt) * (p + w.n_voxels)
    del K64, rho64
    return {"targets": nt, "sample": f"targets [0, {nt}) against all {p} samples and "
            f"{w.n_voxels} cells", "s": dt, "pairs_per_s": pairs / dt,
            "s_per_grad_eval_implied": dt * p / nt,
            "repulsion_pairs_per_s": rep_pairs / (rep_ms * 1e-3),
            "fp32_comp_rel_l2_vs_fp64": d}


def cpu_baseline(w, K, rho, seconds, field=False, eps=0.0, kernel="distance"):
    """The FP64 oracle on a bounded sample of targets (all sources each).

    With field=True the oracle's grid attraction is timed instead (the 8
    surrounding nodes of each target summed over all cells, then the
    trilinear interpolant), and the rate counts the pair interactions the
    step itself performs per target (p, the repulsion)."""
    import oracle
    from paper_2108_02991_amd import inputs

    Kh = K.detach().cpu().double().numpy()
    rh = rho.detach().cpu().double().numpy()
    p = Kh.shape[1]
    fn = oracle.grad_field if field else oracle.grad
    credited = p if field else p + w.n_voxels
    # targets in batches of 64 until the time budget is spent (at least one batch)
    pool = inputs.sample_targets(p, min(p, 65536), seed=100)
    done, dt = 0, 0.0
    while done < pool.size and (done == 0 or dt < seconds):
        batch = pool[done:done + 64]
        t0 = time.perf_counter()
        fn(Kh, rh, w.grid, w.half_width, eps, batch, kernel=kernel)
        dt += time.perf_counter() - t0
        done += batch.size
    targets = pool[:done]
    log(f"cpu baseline: oracle on {done} targets ({oracle.num_threads()} threads), {dt:.1f} s")
    pairs = float(targets.size) * credited
    what = ("the grid attraction of 8 nodes x all cells" if field else f"all {w.n_voxels} cells")
    return {"value": pairs / dt, "unit": "pair-interactions/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": f"{targets.size} random targets of {w.name}, each against "
            f"all {p} samples and {what} ({kernel} kernel, FP64, compensated sums), {dt:.1f} s",
            "s_per_grad_eval_extrapolated": float(p) * dt / targets.size}


if __name__ == "__main__":
    main()
