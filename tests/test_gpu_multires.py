"""Algorithm 1 (multi-resolution) on the GPU against the oracle's Algorithm 1."""
import numpy as np
import pytest
import torch

from gpu_util import configs, device_problem, host64, inputs, oracle, say, spk
from paper_2108_02991_amd import driver

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["plain_fp64", "fp32_comp"])
def test_upsample_matches_oracle(gpu, precision):
    Nc, N = 5, 37
    K = inputs.radial_spokes(Nc, N, 0.5, seed=9, jitter=0.05)
    prm = spk.Params(Nc, N, 1, precision=precision)
    Kd, _ = device_problem(K, [1.0], precision, gpu)
    got = host64(spk.upsample(Kd, prm))
    want = oracle.upsample(host64(Kd), Nc, N)
    if precision == "plain_fp64":
        assert np.array_equal(got, want)
    else:
        assert np.array_equal(got, want.astype(np.float32).astype(np.float64))


def test_multiresolution_plain_fp64_matches_oracle(gpu):
    """Three levels of 22 iterations each: the 20 fixed steps and two
    Barzilai-Borwein steps per level, step by step against the oracle."""
    w = configs.C1
    Nc, Ns, levels, n_git, G = 6, 64, 2, 22, 8
    a, b = spk.alpha_beta(configs.GMAX, configs.SMAX, configs.RASTER_DT, configs.DWELL_DT, w.fov,
                          w.kmax, configs.GAMMA_BAR, 0.5)
    K0 = inputs.radial_spokes(Nc, Ns >> levels, 0.5, seed=3, jitter=0.02)
    rho = inputs.radial_density(G, 0.5, 0.05, 2.0)
    prm = spk.Params(Nc, Ns, G, precision="plain_fp64", a_max=a, b_max=b, n_pit=100)
    Kd, rd = device_problem(K0, rho, "plain_fp64", gpu)
    say("  multires GPU")
    Kg, recs = driver.multiresolution(Kd, rd, prm, levels, n_git)
    say("  multires oracle")
    Ko, orecs = oracle.multiresolution(K0, rho, Nc, Ns >> levels, levels, G, 0.5, a, b, 0, 100,
                                       n_git)
    assert len(recs) == len(orecs) == (levels + 1) * n_git
    for r, o in zip(recs, orecs):
        assert r["level"] == o["level"] and r["iter"] == o["iter"]
        assert r["F"] == pytest.approx(o["F"], rel=1e-11)
        assert r["eta"] == pytest.approx(o["eta"], rel=1e-12)
        assert r["bb_used"] == o["bb_used"] == (o["iter"] >= 20)
        if o["iter"] >= 20:
            assert r["bb_quotient"] == pytest.approx(o["bb_quotient"], rel=1e-9)
    assert Kg.shape == (3, Nc * Ns)
    assert np.abs(host64(Kg) - Ko).max() <= 1e-9


def test_multiresolution_with_the_far_field(gpu):
    """Algorithm 1 with the far field requested: levels of at most exact_max_p
    samples take the exact sums (by default every level of this small problem,
    so the run equals the exact one bit for bit); with the threshold at 0 every
    level takes the far field, and F stays within its accuracy of the exact run."""
    w = configs.C1
    Nc, Ns, levels, n_git, G = 64, 256, 2, 4, 8
    a, b = spk.alpha_beta(configs.GMAX, configs.SMAX, configs.RASTER_DT, configs.DWELL_DT, w.fov,
                          w.kmax, configs.GAMMA_BAR, 0.5)
    K0 = inputs.radial_spokes(Nc, Ns >> levels, 0.5, seed=5, jitter=0.05)
    rho = inputs.radial_density(G, 0.5, 0.05, 2.0)

    def run(depth, exact_max_p=driver.EXACT_MAX_P):
        prm = spk.Params(Nc, Ns, G, precision="fp32_comp", a_max=a, b_max=b, n_pit=100,
                         far_field_depth=depth, far_field_order=6,
                         far_field_adaptive=1 if depth else 0)
        Kd, rd = device_problem(K0, rho, "fp32_comp", gpu)
        say(f"  multires far field depth {depth}, exact up to {exact_max_p} samples")
        Kg, recs = driver.multiresolution(Kd, rd, prm, levels, n_git, exact_max_p=exact_max_p)
        return host64(Kg), recs

    K_exact, r_exact = run(0)
    K_small, r_small = run(3)
    assert np.array_equal(K_small, K_exact)
    assert [r["F"] for r in r_small] == [r["F"] for r in r_exact]
    K_ff, r_ff = run(3, exact_max_p=0)
    assert len(r_ff) == len(r_exact) == (levels + 1) * n_git
    for r, e in zip(r_ff, r_exact):
        assert r["F"] == pytest.approx(e["F"], rel=1e-6)
    assert np.abs(K_ff - K_exact).max() <= 1e-5
