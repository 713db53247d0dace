"""Seeded synthetic inputs: determinism, shapes and the structure the workloads assume."""
import numpy as np
import pytest

from paper_2108_02991_amd import configs, inputs


def test_spokes_deterministic_and_shaped():
    a = inputs.radial_spokes(16, 32, 0.5, seed=3, jitter=0.05)
    b = inputs.radial_spokes(16, 32, 0.5, seed=3, jitter=0.05)
    c = inputs.radial_spokes(16, 32, 0.5, seed=4, jitter=0.05)
    assert a.shape == (3, 512) and a.dtype == np.float64
    assert inputs.digest(a) == inputs.digest(b) != inputs.digest(c)
    assert np.abs(a).max() <= 0.5
    assert np.all(a[:, ::32] == 0.0)                    # sample 0 of every shot at the origin


def test_plain_spokes_are_straight_centre_out():
    K = inputs.radial_spokes(8, 64, 0.5, seed=1, jitter=0.0)
    shot = K[:, :64]
    r = np.linalg.norm(shot, axis=0)
    np.testing.assert_allclose(r, 0.5 * np.arange(64) / 63, atol=1e-15)
    d = shot[:, 1:] - shot[:, :-1]
    np.testing.assert_allclose(d, np.repeat(d[:, :1], 63, axis=1), atol=1e-15)


def test_density_normalised_and_radial():
    rho = inputs.radial_density(32, 0.5, 0.05, 2.0)
    assert rho.shape == (32 ** 3,)
    assert rho.sum() == pytest.approx(1.0, rel=1e-14)
    r3 = rho.reshape(32, 32, 32)
    # symmetric under axis flips and x<->y swap (radial law on a symmetric grid)
    assert np.allclose(r3, r3[::-1], rtol=1e-14)
    assert np.allclose(r3, r3.transpose(0, 2, 1), rtol=1e-14)
    # min(1, (0.05/r)^2): the centre cells are on the plateau, corners decay as r^-2
    ax = inputs.voxel_axis(32, 0.5)
    rc = np.sqrt(3) * abs(ax[0])
    assert r3[0, 0, 0] / r3.max() == pytest.approx((0.05 / rc) ** 2, rel=1e-12)


def test_workload_sizes():
    assert configs.C3.p == 8_388_608 and configs.C3.n_voxels == 192 ** 3
    assert configs.C1.p == 4096 and configs.C4.p == 65536
    assert configs.C5.p == 2_097_152 and configs.C2.p == 524_288
    assert configs.C1.eta_fixed == pytest.approx(64.0)
    assert configs.C5.eta_fixed == pytest.approx(4096.0)
    assert configs.C3.kmax == pytest.approx(833.3333333, rel=1e-9)


def test_sample_targets():
    t = inputs.sample_targets(1000, 64, seed=5)
    assert t[0] == 0 and t[-1] == 999 and np.all(np.diff(t) > 0) and t.size == 64
