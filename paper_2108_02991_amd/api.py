"""Python binding of libsparkling.so: argument marshalling over ctypes only.

Every computation runs in the library's HIP kernels; torch supplies device
memory (the trajectory K as a (3, p) tensor, rho, outputs, the workspace) and
the current stream.  The binding raises if the library was not built: there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import dataclasses
from dataclasses import dataclass, field
from pathlib import Path

import numpy as np
import torch

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libsparkling.so"

PRECISIONS = {"plain_fp64": 0, "fp32_comp": 1, "fp32_naive": 2, "fp32_acc64": 3}
FLAG_DISCREPANCY = 1
FLAG_ROTATION_VARIANT = 2
FLAG_LOG_KERNEL = 4
FLAG_FIELD_DIRECT = 8
FLAG_ENERGY_FROM_FORCE = 16
KERNELS = {"distance": 0, "log": FLAG_LOG_KERNEL}
KIND_REPULSION, KIND_ATTRACTION, KIND_PROJECTION, KIND_OTHER, KIND_INTERPOLATION = 0, 1, 2, 3, 4

_i32, _i64, _dbl, _vp, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class SpkParams(ctypes.Structure):
    _fields_ = [("n_shots", _i64), ("n_samples", _i64), ("grid", _i64), ("precision", _i32),
                ("te_index", _i32), ("half_width", _dbl), ("eps", _dbl), ("a_max", _dbl),
                ("b_max", _dbl), ("n_pit", _i32), ("flags", _i32), ("attraction_field", _vp),
                ("far_field_depth", _i32), ("far_field_order", _i32),
                ("far_field_adaptive", _i32), ("far_field_stream", _vp), ("proj_duals", _vp)]


class SpkStepInfo(ctypes.Structure):
    _fields_ = [("iter", _i64), ("eta_fixed", _dbl), ("eta", _dbl), ("F", _dbl), ("Fa", _dbl),
                ("Fr", _dbl), ("viol", _dbl * 4), ("bb_used", _i32), ("reserved", _i32),
                ("bb_quotient", _dbl)]


class SparklingError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None


def load_library(path: Path | str | None = None):
    """Load libsparkling.so (once): `path`, else $SPK_LIBRARY, else the in-tree
    build.  Raises if the file does not exist."""
    global _lib
    if _lib is not None:
        return _lib
    p = Path(path) if path else Path(os.environ.get("SPK_LIBRARY") or LIB_PATH)
    if not p.exists():
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2108_02991_amd.build`")
    lib = ctypes.CDLL(str(p))
    sig = {
        "spk_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "spk_last_error": ([], ctypes.c_char_p),
        "spk_alpha_beta": ([_dbl] * 8 + [_vp, _vp], ctypes.c_int),
        "spk_workspace_size": ([_vp, _vp], ctypes.c_int),
        "spk_field_workspace_size": ([_vp, _vp], ctypes.c_int),
        "spk_lipschitz_bound": ([_i64, _dbl, _dbl, _i32, _vp], ctypes.c_int),
        "sparkling_energy": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
        "sparkling_field": ([_vp, _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
        "sparkling_grad": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _vp,
                            _vp, _sz, _vp], ctypes.c_int),
        "sparkling_project": ([_vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
        "sparkling_constraint_check": ([_vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
        "sparkling_step": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], ctypes.c_int),
        "sparkling_step_async": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _dbl, _vp, _vp, _sz,
                                  _vp], ctypes.c_int),
        "sparkling_upsample": ([_vp] * 8, ctypes.c_int),
        "sparkling_step_async_noalloc": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _dbl, _vp,
                                          _vp], ctypes.c_int),
        "spk_noalloc_scratch_bytes": ([], _sz),
        "spk_probe_pair_mix": ([ctypes.c_int, _i64, _i32, _vp, _sz, _vp, _vp, _vp],
                               ctypes.c_int),
        "spk_timing_enable": ([ctypes.c_int], ctypes.c_int),
        "spk_timing_query": ([ctypes.c_int, _vp, _vp, _vp], ctypes.c_int),
        "spk_timing_reset": ([], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != 0:
        lib = load_library()
        raise SparklingError(rc, where, f"{lib.spk_status_string(rc).decode()}: "
                                        f"{lib.spk_last_error().decode()}")


@dataclass
class Params:
    """Problem description (mirrors spk_params of sparkling.h)."""
    n_shots: int
    n_samples: int
    grid: int
    precision: str = "fp32_comp"
    half_width: float = 0.5
    eps: float = 0.0
    a_max: float = 1.0
    b_max: float = 1.0
    te_index: int = 0
    n_pit: int = 200
    discrepancy: bool = False
    rotation_variant: bool = False                   # per-axis speed/slew bounds
    kernel: str = "distance"                         # "distance" or "log" (needs eps > 0)
    attraction_field: "torch.Tensor | None" = None   # from attraction_field(); None = direct sum
    far_field_depth: int = 0                         # 0: exact repulsion; 2..7: octree depth
    far_field_order: int = 5                         # Chebyshev nodes per axis (3..6)
    far_field_adaptive: int = 0                      # refinement levels of dense cells (0..2)
    far_field_overlap: bool = True                   # near-field sums on a second stream
    proj_duals: "torch.Tensor | None" = None         # warm-start duals (new_duals()); None = cold
    energy_from_force: bool = False                  # F^r = sum_i K[i] . dF^r/dK[i] (H = |d|)
    field_direct: bool = False                       # node field summed directly, not by FFT
    _c: SpkParams = field(default=None, repr=False, compare=False)

    @property
    def p(self) -> int:
        return self.n_shots * self.n_samples

    @property
    def dtype(self) -> torch.dtype:
        return torch.float64 if self.precision == "plain_fp64" else torch.float32

    def c(self, device=None) -> SpkParams:
        """The C struct; with a CUDA device and the far field on, it carries the
        binding's second stream of that device for the far field's near-field sums."""
        f = self.attraction_field
        if f is not None and (not f.is_cuda or f.dtype != self.dtype or not f.is_contiguous()
                              or f.numel() != 4 * (self.grid + 2) ** 3):
            raise ValueError("attraction_field must be a contiguous device tensor of "
                             f"4*(G+2)^3 {self.dtype} values")
        d = self.proj_duals
        if d is not None and (not d.is_cuda or d.dtype != torch.float64 or not d.is_contiguous()
                              or d.numel() != 6 * self.p):
            raise ValueError("proj_duals must be a contiguous float64 device tensor of "
                             "n_shots*6*n_samples values")
        return SpkParams(self.n_shots, self.n_samples, self.grid, PRECISIONS[self.precision],
                         self.te_index, self.half_width, self.eps, self.a_max, self.b_max,
                         self.n_pit,
                         (FLAG_DISCREPANCY if self.discrepancy else 0)
                         | (FLAG_ROTATION_VARIANT if self.rotation_variant else 0)
                         | KERNELS[self.kernel]
                         | (FLAG_FIELD_DIRECT if self.field_direct else 0)
                         | (FLAG_ENERGY_FROM_FORCE if self.energy_from_force else 0),
                         _vp(f.data_ptr()) if f is not None else None,
                         self.far_field_depth, self.far_field_order if self.far_field_depth else 0,
                         int(self.far_field_adaptive),
                         _far_field_stream(device)
                         if self.far_field_depth and self.far_field_overlap else None,
                         _vp(d.data_ptr()) if d is not None else None)


_SIDE_STREAMS: dict = {}


def _far_field_stream(device):
    """A second stream per device (default priority), created once by the
    binding and passed to the library, which holds no stream of its own."""
    if device is None:
        return None
    device = torch.device(device)
    if device.type != "cuda":
        return None
    idx = device.index if device.index is not None else torch.cuda.current_device()
    st = _SIDE_STREAMS.get(idx)
    if st is None:
        st = _SIDE_STREAMS[idx] = torch.cuda.Stream(device=idx)
    return _vp(st.cuda_stream)


def lipschitz_bound(p: int, eps: float, rho_mass: float = 1.0, kernel: str = "distance") -> float:
    """Upper bound on the Lipschitz constant of grad F (the fixed step 1/L guarantees descent)."""
    out = _dbl()
    _check(load_library().spk_lipschitz_bound(p, eps, rho_mass, KERNELS[kernel],
                                              ctypes.byref(out)), "spk_lipschitz_bound")
    return out.value


def alpha_beta(gmax, smax, raster_dt, dwell_dt, fov, kmax, gamma_bar, half_width):
    a, b = _dbl(), _dbl()
    _check(load_library().spk_alpha_beta(gmax, smax, raster_dt, dwell_dt, fov, kmax, gamma_bar,
                                         half_width, ctypes.byref(a), ctypes.byref(b)),
           "spk_alpha_beta")
    return a.value, b.value


def workspace_size(prm: Params) -> int:
    n = _sz()
    c = prm.c()
    _check(load_library().spk_workspace_size(ctypes.byref(c), ctypes.byref(n)), "spk_workspace_size")
    return n.value


_ws_cache: dict = {}


def workspace(prm: Params, device) -> torch.Tensor:
    """A cached device workspace large enough for prm (one per device and stream)."""
    n = workspace_size(prm)
    stream = torch.cuda.current_stream(device).cuda_stream
    key = (torch.device(device).index, stream)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < n:
        _ws_cache.pop(key, None)
        ws = torch.empty(n, dtype=torch.uint8, device=device)
        _ws_cache[key] = ws
    return ws


def release_workspaces():
    """Drop the cached device workspaces (they only grow otherwise)."""
    _ws_cache.clear()


def _stream(t: torch.Tensor):
    return _vp(torch.cuda.current_stream(t.device).cuda_stream)


def _check_k(K: torch.Tensor, prm: Params, name="K"):
    if not K.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if K.dtype != prm.dtype:
        raise ValueError(f"{name} must be {prm.dtype} for precision {prm.precision}")
    if K.dim() != 2 or K.shape[0] != 3 or K.shape[1] != prm.p or not K.is_contiguous():
        raise ValueError(f"{name} must be a contiguous (3, {prm.p}) tensor")


def _check_rho(rho: torch.Tensor, prm: Params):
    if not rho.is_cuda or rho.dtype != prm.dtype or rho.numel() != prm.grid ** 3 or not rho.is_contiguous():
        raise ValueError(f"rho must be a contiguous {prm.dtype} device tensor of {prm.grid ** 3} weights")


def _rows(K: torch.Tensor):
    return [_vp(K[c].data_ptr()) for c in range(3)]


def attraction_field(rho: torch.Tensor, prm: Params) -> torch.Tensor:
    """Node field of the grid attraction, a ((G+2)^3, 4) tensor of rho's dtype.

    Assign it to prm.attraction_field to evaluate the attraction by trilinear
    interpolation instead of the direct sum over the cells.
    """
    _check_rho(rho, prm)
    out = torch.empty(((prm.grid + 2) ** 3, 4), dtype=prm.dtype, device=rho.device)
    c = prm.c()
    n = _sz()
    _check(load_library().spk_field_workspace_size(ctypes.byref(c), ctypes.byref(n)),
           "spk_field_workspace_size")
    if n.value <= workspace_size(prm):
        ws = workspace(prm, rho.device)
    else:   # the FFT buffers: a temporary workspace, freed on return
        ws = torch.empty(n.value, dtype=torch.uint8, device=rho.device)
    _check(load_library().sparkling_field(ctypes.byref(c), _vp(rho.data_ptr()),
                                          _vp(out.data_ptr()), _vp(ws.data_ptr()), ws.numel(),
                                          _stream(rho)), "sparkling_field")
    return out


def energy(K: torch.Tensor, rho: torch.Tensor, prm: Params):
    """(F, Fa, Fr, D) as Python floats; D is NaN unless prm.discrepancy."""
    _check_k(K, prm)
    _check_rho(rho, prm)
    ws = workspace(prm, K.device)
    out = (_dbl * 4)()
    c = prm.c(K.device)
    _check(load_library().sparkling_energy(ctypes.byref(c), *_rows(K), _vp(rho.data_ptr()), out,
                                           _vp(ws.data_ptr()), ws.numel(), _stream(K)),
           "sparkling_energy")
    return tuple(out)


def grad(K: torch.Tensor, rho: torch.Tensor, prm: Params, tgt=None, out: torch.Tensor | None = None,
         potentials: bool = False, with_energy: bool = False):
    """Gradient rows [b, e) (default all) as a (3, e-b) tensor of K's dtype.

    With potentials=True also returns (pot_a, pot_r) float64 tensors of the
    unscaled per-target sums of H; with_energy=True also returns (F, Fa, Fr).
    """
    _check_k(K, prm)
    _check_rho(rho, prm)
    b, e = (0, prm.p) if tgt is None else (int(tgt[0]), int(tgt[1]))
    nt = e - b
    if out is None:
        out = torch.empty((3, nt), dtype=K.dtype, device=K.device)
    elif out.shape != (3, nt) or out.dtype != K.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous (3, e-b) tensor of K's dtype")
    pa = pr = None
    if potentials:
        pa = torch.empty(nt, dtype=torch.float64, device=K.device)
        pr = torch.empty(nt, dtype=torch.float64, device=K.device)
    en = (_dbl * 3)() if with_energy else None
    ws = workspace(prm, K.device)
    c = prm.c(K.device)
    _check(load_library().sparkling_grad(
        ctypes.byref(c), *_rows(K), _vp(rho.data_ptr()), *_rows(out), b, e,
        _vp(pa.data_ptr()) if pa is not None else None,
        _vp(pr.data_ptr()) if pr is not None else None,
        en, _vp(ws.data_ptr()), ws.numel(), _stream(K)), "sparkling_grad")
    res = [out]
    if potentials:
        res.append((pa, pr))
    if with_energy:
        res.append(tuple(en))
    return res[0] if len(res) == 1 else tuple(res)


def project_(K: torch.Tensor, prm: Params, check: bool = True):
    """Project every shot of K in place; returns the constraint check (numpy, 4)."""
    _check_k(K, prm)
    ws = workspace(prm, K.device)
    viol = (_dbl * 4)() if check else None
    c = prm.c()
    _check(load_library().sparkling_project(ctypes.byref(c), *_rows(K), viol, _vp(ws.data_ptr()),
                                            ws.numel(), _stream(K)), "sparkling_project")
    return np.array(viol[:]) if check else None


def constraint_check(K: torch.Tensor, prm: Params):
    _check_k(K, prm)
    ws = workspace(prm, K.device)
    viol = (_dbl * 4)()
    c = prm.c()
    _check(load_library().sparkling_constraint_check(ctypes.byref(c), *_rows(K), viol,
                                                     _vp(ws.data_ptr()), ws.numel(), _stream(K)),
           "sparkling_constraint_check")
    return np.array(viol[:])


def upsample(K: torch.Tensor, prm: Params) -> torch.Tensor:
    """Dyadic linear up-sampling of every shot of K (prm describes the coarse
    trajectory); returns a (3, 2p) tensor."""
    _check_k(K, prm)
    out = torch.empty((3, 2 * prm.p), dtype=K.dtype, device=K.device)
    c = prm.c()
    _check(load_library().sparkling_upsample(ctypes.byref(c), *_rows(K), *_rows(out), _stream(K)),
           "sparkling_upsample")
    return out


def new_duals(prm: Params, device) -> torch.Tensor:
    """Zeroed warm-start dual state for prm.proj_duals: (n_shots, 6, n_samples) doubles."""
    return torch.zeros((prm.n_shots, 6, prm.n_samples), dtype=torch.float64, device=device)


class StepState:
    """Caller-owned state of the step-size policy: previous K and gradient, (3, p) each."""

    def __init__(self, prm: Params, device):
        self.k_prev = torch.zeros((3, prm.p), dtype=prm.dtype, device=device)
        self.g_prev = torch.zeros((3, prm.p), dtype=prm.dtype, device=device)


def step_(K: torch.Tensor, rho: torch.Tensor, prm: Params, state: StepState, it: int,
          eta_fixed: float):
    """One projected gradient step in place on K; returns the step info as a dict."""
    _check_k(K, prm)
    _check_rho(rho, prm)
    _check_k(state.k_prev, prm, "k_prev")
    _check_k(state.g_prev, prm, "g_prev")
    ws = workspace(prm, K.device)
    info = SpkStepInfo()
    info.iter = it
    info.eta_fixed = eta_fixed
    c = prm.c(K.device)
    rc = load_library().sparkling_step(ctypes.byref(c), *_rows(K), _vp(rho.data_ptr()),
                                       _vp(state.k_prev.data_ptr()), _vp(state.g_prev.data_ptr()),
                                       ctypes.byref(info), _vp(ws.data_ptr()), ws.numel(), _stream(K))
    _check(rc, "sparkling_step")
    return {"eta": info.eta, "F": info.F, "Fa": info.Fa, "Fr": info.Fr,
            "viol": np.array(info.viol[:]), "bb_used": bool(info.bb_used),
            "bb_quotient": info.bb_quotient}


INFO_FIELDS = ("eta", "F", "Fa", "Fr", "viol0", "viol1", "viol2", "viol3", "bb_used",
               "bb_quotient")


def step_async_(K: torch.Tensor, rho: torch.Tensor, prm: Params, state: StepState, it: int,
                eta_fixed: float, info: torch.Tensor, ws: torch.Tensor | None = None):
    """Enqueue one projected gradient step on K's current stream with no host
    synchronisation; info (a float64 device tensor of 10) receives eta, F, Fa,
    Fr, the 4 violations, bb_used and the unclamped quotient s.s/s.y.  Pass ws to pin the workspace (needed
    when the call is captured into a graph)."""
    _check_k(K, prm)
    _check_rho(rho, prm)
    _check_k(state.k_prev, prm, "k_prev")
    _check_k(state.g_prev, prm, "g_prev")
    if (not info.is_cuda or info.dtype != torch.float64 or info.numel() < 10
            or not info.is_contiguous()):
        raise ValueError("info must be a contiguous float64 device tensor of at least 10")
    ws = workspace(prm, K.device) if ws is None else ws
    c = prm.c(K.device)
    _check(load_library().sparkling_step_async(
        ctypes.byref(c), *_rows(K), _vp(rho.data_ptr()), _vp(state.k_prev.data_ptr()),
        _vp(state.g_prev.data_ptr()), it, eta_fixed, _vp(info.data_ptr()), _vp(ws.data_ptr()),
        ws.numel(), _stream(K)), "sparkling_step_async")


def step_async_noalloc_(K: torch.Tensor, rho: torch.Tensor, prm: Params, state: StepState,
                        it: int, eta_fixed: float, info: torch.Tensor):
    """step_async_ without a workspace: the library's static device scratch
    (spk_noalloc_scratch_bytes()) serves instead; nothing is allocated.  Calls
    that overlap on one device race on that scratch."""
    _check_k(K, prm)
    _check_rho(rho, prm)
    _check_k(state.k_prev, prm, "k_prev")
    _check_k(state.g_prev, prm, "g_prev")
    if (not info.is_cuda or info.dtype != torch.float64 or info.numel() < 10
            or not info.is_contiguous()):
        raise ValueError("info must be a contiguous float64 device tensor of at least 10")
    c = prm.c()
    _check(load_library().sparkling_step_async_noalloc(
        ctypes.byref(c), *_rows(K), _vp(rho.data_ptr()), _vp(state.k_prev.data_ptr()),
        _vp(state.g_prev.data_ptr()), it, eta_fixed, _vp(info.data_ptr()), _stream(K)),
        "sparkling_step_async_noalloc")


def noalloc_scratch_bytes() -> int:
    return int(load_library().spk_noalloc_scratch_bytes())


PROBE_VARIANTS = {"pair": 0, "pair_without_rsqrt": 1, "rsqrt": 2}


def probe_pair_mix(variant: str = "pair", blocks: int = 32768, iters: int = 1024,
                   reps: int = 3, device="cuda:0") -> dict:
    """Issue rate of the repulsion pair's instruction mix (spk_probe_pair_mix):
    the best of `reps` launches, as pairs/s and, for the full pair, TFLOP/s at
    the sweep's 17 flop/pair."""
    v = PROBE_VARIANTS[variant]
    out = torch.empty(blocks * 256, dtype=torch.float32, device=device)
    pairs, ms = _dbl(), _dbl()
    best = None
    for _ in range(max(reps, 1)):
        _check(load_library().spk_probe_pair_mix(
            v, blocks, iters, _vp(out.data_ptr()), out.numel() * 4, ctypes.byref(pairs),
            ctypes.byref(ms), _stream(out)), "spk_probe_pair_mix")
        best = ms.value if best is None else min(best, ms.value)
    rate = pairs.value / (best * 1e-3)
    return {"variant": variant, "blocks": blocks, "iters": iters, "pairs": pairs.value,
            "ms": best, "pairs_per_s": rate, "tflops_at_17": 17.0 * rate / 1e12}


def pair_issue_bound(device="cuda:0") -> dict:
    """Issue bound of the repulsion pair from measured component rates: the
    pair's 10 FP32 instructions at the rate they stream at (probe variant 1)
    plus one reciprocal square root at its cost (variant 2 minus its FMA, one
    tenth of variant 1's pair).  Also the whole mix in one fixed order
    (variant 0), for comparison."""
    fma = probe_pair_mix("pair_without_rsqrt", device=device)
    rsq = probe_pair_mix("rsqrt", device=device)
    mix = probe_pair_mix("pair", device=device)
    t_fma10 = 1.0 / fma["pairs_per_s"]
    t_rsq = 1.0 / rsq["pairs_per_s"] - t_fma10 / 10.0
    rate = 1.0 / (t_fma10 + t_rsq)
    return {"pairs_per_s": rate, "tflops_at_17": 17.0 * rate / 1e12,
            "rsqrt_in_fma_slots": t_rsq / (t_fma10 / 10.0),
            "fma_stream_lane_ops_per_s": 10.0 * fma["pairs_per_s"],
            "fixed_order_mix_pairs_per_s": mix["pairs_per_s"]}


def info_dict(info: torch.Tensor) -> dict:
    """The step info of step_async_ (copied to the host) as step_ returns it."""
    v = info.detach().cpu().double().numpy()
    return {"eta": float(v[0]), "F": float(v[1]), "Fa": float(v[2]), "Fr": float(v[3]),
            "viol": v[4:8].copy(), "bb_used": bool(v[8]), "bb_quotient": float(v[9])}


class StepGraph:
    """One projected gradient step captured in a HIP graph.

    A graph serves one phase of the step-size rule: the fixed step (iterations
    below 20) or Barzilai-Borwein (20 and above).  K, rho, the step state, the
    info tensor and a private workspace are bound at capture and must stay
    alive; every replay advances K in place by one step and overwrites info.
    """

    def __init__(self, K: torch.Tensor, rho: torch.Tensor, prm: Params, state: StepState,
                 eta_fixed: float, barzilai_borwein: bool):
        if prm.far_field_depth:
            raise ValueError("the far-field step is not captured: its leaf sort issues memsets")
        self.K, self.rho, self.prm, self.state = K, rho, dataclasses.replace(prm), state
        self.info = torch.zeros(16, dtype=torch.float64, device=K.device)
        self.ws = torch.empty(workspace_size(prm), dtype=torch.uint8, device=K.device)
        self.graph = torch.cuda.CUDAGraph()
        it = 20 if barzilai_borwein else 0
        with torch.cuda.graph(self.graph):
            step_async_(K, rho, self.prm, state, it, eta_fixed, self.info, self.ws)

    def replay(self):
        self.graph.replay()


def timing_enable(on: bool = True):
    _check(load_library().spk_timing_enable(1 if on else 0), "spk_timing_enable")


def timing_reset():
    _check(load_library().spk_timing_reset(), "spk_timing_reset")


def timing_query(kind: int):
    """(total ms, launches, pair interactions) of one kernel kind since the last reset."""
    ms, n, pairs = _dbl(), _i64(), _dbl()
    _check(load_library().spk_timing_query(kind, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(pairs)),
           "spk_timing_query")
    return ms.value, n.value, pairs.value


class SparklingEnergy(torch.autograd.Function):
    """F(K) as a differentiable function of K.

    forward runs the energy sweep; backward is the gradient kernel itself,
    recomputed chunk by chunk over the targets (no pair terms are stored), then
    scaled by the incoming gradient.  Differentiable in K only.
    """

    @staticmethod
    def forward(ctx, K, rho, prm: Params, chunk: int = 8192):
        F, _, _, _ = energy(K, rho, prm)
        ctx.save_for_backward(K, rho)
        ctx.prm = dataclasses.replace(prm)   # later changes to prm do not reach backward
        ctx.chunk = chunk
        return torch.tensor(F, dtype=torch.float64, device=K.device)

    @staticmethod
    def backward(ctx, g_out):
        K, rho = ctx.saved_tensors
        prm = ctx.prm
        if torch.is_grad_enabled():
            raise RuntimeError("SparklingEnergy does not support double backward")
        g = torch.empty_like(K)
        for b in range(0, prm.p, ctx.chunk):
            e = min(b + ctx.chunk, prm.p)
            part = grad(K, rho, prm, tgt=(b, e))
            g[:, b:e].copy_(part)
        return g * g_out.to(g.dtype), None, None, None


def sparkling_energy(K, rho, prm: Params, chunk: int = 8192):
    return SparklingEnergy.apply(K, rho, prm, chunk)
