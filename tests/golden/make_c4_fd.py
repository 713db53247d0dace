"""Writes c4_fd.npy and c4_fd.json: central finite differences of F for the
differentiation workload (128 shots x 512 samples, 32^3 density, coordinates
as stored in FP32), along 200 dense Rademacher directions, from the FP64
oracle only.

Protocol (section "Evaluating F^r and its gradient": the gradient of the
objective; the finite-difference check of the differentiation form): direction
k is e_k = Rademacher +-1 on every coordinate (seed 1000 + k), step h = 1e-4
per coordinate, FD_k = (F(K + h e_k) - F(K - h e_k)) / (2h) evaluated
cancellation-free by the oracle.  Row k of c4_fd.npy holds FD_k and the
oracle's own <grad F, e_k>; the JSON holds h, the seeds, ||grad F||_2 and the
digests of the input bytes.

Run from the repository root:  python3 tests/golden/make_c4_fd.py   (~30 min on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                                    # noqa: E402
from paper_2108_02991_amd import configs, inputs  # noqa: E402

H = 1e-4
N_DIR = 200
SEED0 = 1000


def c4_inputs():
    """The differentiation workload's inputs as the FP32 form stores them, widened."""
    w = configs.C4
    K = w.trajectory().astype(np.float32).astype(np.float64)
    rho = w.density().astype(np.float32).astype(np.float64)
    return w, K, rho


def main():
    w, K, rho = c4_inputs()
    here = os.path.dirname(os.path.abspath(__file__))
    t0 = time.time()
    og = oracle.grad(K, rho, w.grid, w.half_width)["dF"]
    rows = []
    for k in range(N_DIR):
        e = inputs.rademacher(K.shape, SEED0 + k)
        fd = oracle.fd_directional(K, rho, w.grid, w.half_width, e, H)
        rows.append((fd, float((og * e).sum())))
        print(f"direction {k}: FD {fd:.12e} ({time.time() - t0:.0f} s)", flush=True)
    np.save(os.path.join(here, "c4_fd.npy"), np.array(rows))
    meta = {"workload": w.name, "n_shots": w.n_shots, "n_samples": w.n_samples, "grid": w.grid,
            "half_width": w.half_width, "storage": "float32 coordinates and density, widened",
            "h": H, "directions": N_DIR, "seed0": SEED0, "direction_kind": "rademacher",
            "grad_norm": float(np.linalg.norm(og)), "K_digest": inputs.digest(K),
            "rho_digest": inputs.digest(rho),
            "columns": ["FD_k (oracle, central, cancellation-free)", "<oracle grad F, e_k>"]}
    with open(os.path.join(here, "c4_fd.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(f"wrote c4_fd.npy and c4_fd.json in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
