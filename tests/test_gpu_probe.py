"""Issue-rate probes of the repulsion pair's instruction mix (a calibration
of the sweep's roofline, not an operation of the paper)."""
import pytest

from gpu_util import say, spk

pytestmark = pytest.mark.gpu


def test_pair_mix_probe_rates(gpu):
    full = spk.probe_pair_mix("pair", blocks=8192, iters=512, device=gpu)
    bare = spk.probe_pair_mix("pair_without_rsqrt", blocks=8192, iters=512, device=gpu)
    rsq = spk.probe_pair_mix("rsqrt", blocks=8192, iters=512, device=gpu)
    say(f"  probe: pair {full['pairs_per_s']:.4g}/s, without rsqrt {bare['pairs_per_s']:.4g}/s, "
        f"rsqrt+fma {rsq['pairs_per_s']:.4g}/s")
    assert full["pairs"] == 8192 * 256 * 512 * 8
    # the reciprocal square root costs time: the mix without it is faster
    assert bare["pairs_per_s"] > full["pairs_per_s"] > 0
    # ten FP32 instructions per pair stream at no more than the chip's issue peak
    assert 10 * bare["pairs_per_s"] * 2 < 157.3e12


def test_pair_issue_bound(gpu):
    b = spk.pair_issue_bound(device=gpu)
    say(f"  pair issue bound {b['pairs_per_s']:.4g}/s = {b['tflops_at_17']:.1f} TFLOP/s at 17, "
        f"rsqrt = {b['rsqrt_in_fma_slots']:.2f} FMA slots")
    # between what the repulsion sweep sustains (about 74 TFLOP/s) and the FP32 peak
    assert 70.0 < b["tflops_at_17"] < 157.3
    assert 2.0 < b["rsqrt_in_fma_slots"] < 8.0
