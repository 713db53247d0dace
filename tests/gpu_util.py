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
