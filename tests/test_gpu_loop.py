"""The projected-gradient loop on the 2048 x 1024 workload: FP32-compensated
against the plain-FP64 GPU run, iteration by iteration (the first 22 of the
100 iterations `paper_2108_02991_amd.driver` runs: the 20 fixed steps and two
Barzilai-Borwein steps), with the per-iteration records' metrics."""
import numpy as np
import pytest

from gpu_util import configs, say, spk
from paper_2108_02991_amd import driver

pytestmark = pytest.mark.gpu

ITERS = 22


def test_c5_loop_fp32_comp_tracks_plain_fp64(gpu):
    w = configs.C5
    say(f"  c5 loop fp32_comp, {ITERS} iterations")
    r32, K32 = driver.run(w, "fp32_comp", ITERS, log_every=0)
    say(f"  c5 loop plain_fp64, {ITERS} iterations")
    r64, K64 = driver.run(w, "plain_fp64", ITERS, log_every=0)
    for a, b in zip(r32[:-1], r64[:-1]):
        say(f"  iter {a['iter']}: F32 {a['F']:.12e} F64 {b['F']:.12e} eta32 {a['eta']:.6g} "
            f"eta64 {b['eta']:.6g} quotient64 {b['bb_quotient']:.6g} "
            f"viol32 {np.round(a['viol'], 4).tolist()}")
        assert a["F"] == pytest.approx(b["F"], rel=1e-6)
        assert a["D"] == pytest.approx(b["D"], rel=1e-5)
        assert a["grad_norm"] == pytest.approx(b["grad_norm"], rel=1e-4)
        if a["iter"] < 20:
            assert a["eta"] == b["eta"] == w.eta_fixed and not a["bb_used"]
            assert np.isnan(a["bb_quotient"]) and np.isnan(b["bb_quotient"])
        else:
            # the Barzilai-Borwein phase: both runs take the BB step, from quotients that
            # agree to the FP32 storage of K and the gradient
            assert a["bb_used"] and b["bb_used"]
            assert a["bb_quotient"] == pytest.approx(b["bb_quotient"], rel=1e-3)
            assert a["eta"] == pytest.approx(b["eta"], rel=1e-3)
            lo, hi = 0.1 * w.eta_fixed, 10.0 * w.eta_fixed
            assert b["eta"] == min(max(b["bb_quotient"], lo), hi)
        assert a["viol"][2] <= 1.0 and a["viol"][3] == 0.0
        assert a["D"] >= 0.0 and b["D"] >= 0.0
        km = a["kernel_ms"]
        assert km["repulsion"] > 0 and km["attraction"] > 0 and km["projection"] > 0
        assert sum(km.values()) <= 1e3 * a["s"] * 1.05
    assert r32[-1]["final_F"] == pytest.approx(r64[-1]["final_F"], rel=1e-6)
    # the energy decreases over the run
    assert r64[-1]["final_F"] < r64[0]["F"]
    d = (K32.double() - K64).abs().max().item()
    say(f"  max |K32 - K64| after {ITERS} steps: {d:.3e}")
    assert d < 1e-3
