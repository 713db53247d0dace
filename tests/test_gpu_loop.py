"""The projected-gradient loop on the 2048 x 1024 workload: FP32-compensated
against the plain-FP64 GPU run, iteration by iteration (a short prefix of the
100-iteration run of `paper_2108_02991_amd.driver`)."""
import numpy as np
import pytest

from gpu_util import configs, say, spk
from paper_2108_02991_amd import driver

pytestmark = pytest.mark.gpu


def test_c5_loop_fp32_comp_tracks_plain_fp64(gpu):
    w = configs.C5
    say("  c5 loop fp32_comp")
    r32, K32 = driver.run(w, "fp32_comp", 3, log_every=0)
    say("  c5 loop plain_fp64")
    r64, K64 = driver.run(w, "plain_fp64", 3, log_every=0)
    for a, b in zip(r32[:-1], r64[:-1]):
        say(f"  iter {a['iter']}: F32 {a['F']:.12e} F64 {b['F']:.12e} "
            f"viol32 {np.round(a['viol'], 4).tolist()}")
        assert a["F"] == pytest.approx(b["F"], rel=1e-6)
        assert a["eta"] == b["eta"]
        assert a["viol"][2] <= 1.0 and a["viol"][3] == 0.0
    assert r32[-1]["final_F"] == pytest.approx(r64[-1]["final_F"], rel=1e-6)
    # the energy decreases over the first steps
    assert r64[-1]["final_F"] < r64[0]["F"]
    d = (K32.double() - K64).abs().max().item()
    say(f"  max |K32 - K64| after 3 steps: {d:.3e}")
    assert d < 1e-4
