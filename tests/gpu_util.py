"""Shared helpers of the GPU tests (inputs to device, error measures)."""
import os
import sys

import numpy as np
import torch

import oracle
import paper_2108_02991_amd as spk
from paper_2108_02991_amd import configs, inputs

DTYPE = {"plain_fp64": torch.float64, "fp32_comp": torch.float32, "fp32_naive": torch.float32,
         "fp32_acc64": torch.float32}

# Relative L2 error bounds of the gradient against the FP64 oracle.  The
# FP32-compensated bound is the target the form is built for; plain FP64
# differs from the oracle only by summation order and the rsqrt rounding.
GRAD_TOL = {"plain_fp64": 1e-12, "fp32_comp": 1e-5, "fp32_acc64": 1e-5, "fp32_naive": 3e-3}
ENERGY_TOL = {"plain_fp64": 1e-12, "fp32_comp": 1e-6, "fp32_acc64": 1e-6, "fp32_naive": 1e-3}


def say(*a):
    """Print progress (shown with -s) and append it to $SPK_TEST_LOG if set."""
    print(*a, flush=True)
    sys.stdout.flush()
    path = os.environ.get("SPK_TEST_LOG")
    if path:
        with open(path, "a") as f:
            f.write(" ".join(str(x) for x in a) + "\n")


def device_problem(K, rho, precision, dev):
    dt = DTYPE[precision]
    Kd = torch.tensor(np.asarray(K), dtype=dt, device=dev).contiguous()
    rd = torch.tensor(np.asarray(rho), dtype=dt, device=dev).contiguous()
    return Kd, rd


def host64(t):
    return t.detach().cpu().double().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def row_rel_max(got, ref, floor_frac=1e-3):
    """Largest per-row error |got_i - ref_i| / max(|ref_i|, floor) over the rows
    (columns of a (3, n) array), floor = floor_frac x the rms row norm of ref: a
    few wrong rows cannot hide inside a relative L2 norm, and rows whose
    gradient nearly cancels (the echo-time samples at the origin) are measured
    against the typical row instead of their own tiny norm."""
    got, ref = np.asarray(got), np.asarray(ref)
    nr = np.linalg.norm(ref, axis=0)
    floor = floor_frac * np.sqrt(np.mean(nr * nr))
    return float((np.linalg.norm(got - ref, axis=0) / np.maximum(nr, floor)).max())


# Per-row bounds (row_rel_max) of the gradient against the FP64 oracle.
ROW_TOL = {"plain_fp64": 1e-11, "fp32_comp": 1e-4, "fp32_acc64": 1e-4, "fp32_naive": 3e-2}


def with_te_rows(t, n_shots, n_samples, count=8):
    """Sampled targets plus the echo-time samples (sample 0) of `count` spread
    shots, where n_shots samples coincide at the origin."""
    te = (np.linspace(0, n_shots - 1, count).astype(np.int64)) * n_samples
    return np.unique(np.concatenate([np.asarray(t, dtype=np.int64), te]))


def bounds(w):
    return spk.alpha_beta(configs.GMAX, configs.SMAX, configs.RASTER_DT, configs.DWELL_DT, w.fov,
                          w.kmax, configs.GAMMA_BAR, w.half_width)


def params_for(w, precision=None, **kw):
    a, b = bounds(w)
    base = dict(n_shots=w.n_shots, n_samples=w.n_samples, grid=w.grid,
                precision=precision or w.precision, half_width=w.half_width, a_max=a, b_max=b,
                te_index=0, n_pit=w.n_pit)
    base.update(kw)
    return spk.Params(**base)


__all__ = ["oracle", "spk", "configs", "inputs", "np", "torch"]
