"""Largest sizes and multi-pass paths: the maximum grid (G = 1024), a sample
count whose workspace offsets pass 2^32, and the node field and self-energy
when their grid targets need more than one pass."""
import numpy as np
import pytest
import torch

from gpu_util import (ENERGY_TOL, GRAD_TOL, device_problem, host64, inputs, oracle, rel_l2,
                      say, spk)

pytestmark = pytest.mark.gpu

GRID_PASS = 1 << 21   # grid targets per pass of the field and self-energy sweeps


def node_coords(idx, G, L=0.5):
    """Coordinates of field nodes n = kx + (G+2)(ky + (G+2) kz): -L + (k - 1/2) 2L/G."""
    Gn = G + 2
    k = np.stack([idx % Gn, (idx // Gn) % Gn, idx // (Gn * Gn)]).astype(np.float64)
    return -L + (k - 0.5) * (2 * L / G)


def test_field_in_two_passes(gpu):
    """(G+2)^3 = 129^3 > 2^21 nodes: rows of both passes against the oracle's direct
    sums at the node coordinates."""
    G, L = 127, 0.5
    Mn = (G + 2) ** 3
    assert Mn > GRID_PASS
    rho = inputs.radial_density(G, L, 0.1, 2.0)
    prm = spk.Params(1, 8, G, precision="plain_fp64")
    _, rd = device_problem(np.zeros((3, 8)), rho, "plain_fp64", gpu)
    say(f"  field G={G}: {Mn} nodes")
    f = host64(spk.attraction_field(rd, prm))
    idx = np.unique(np.concatenate([np.arange(4), GRID_PASS + np.arange(-4, 4), Mn - 1 - np.arange(4),
                                    np.random.default_rng(3).integers(0, Mn, 20)]))
    P = node_coords(idx, G)
    ref = oracle.grad(P, rho, G, L)
    n = P.shape[1]
    assert rel_l2(f[idx, 0], ref["ua"]) <= 1e-12
    assert rel_l2(f[idx, 1:].T, ref["dFa"] * n) <= 1e-12


def test_discrepancy_in_two_passes_vanishes_at_equilibrium(gpu):
    """G^3 = 130^3 > 2^21 cells, samples at the cell centres, uniform density: D = 0
    exactly in real arithmetic, with the self-energy summed in two passes."""
    G = 130
    M = G ** 3
    assert M > GRID_PASS
    ax = inputs.voxel_axis(G, 0.5)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    K = np.stack([x.ravel(), y.ravel(), z.ravel()])
    rho = inputs.uniform_density(G)
    prm = spk.Params(G * G, G, G, precision="plain_fp64", discrepancy=True)
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    say(f"  discrepancy G={G}: {M} samples and cells")
    F, Fa, Fr, D = spk.energy(Kd, rd, prm)
    say(f"  F={F:.15e} D={D:.3e}")
    assert abs(D) <= 1e-12 * Fa
    assert Fa == pytest.approx(2 * Fr, rel=1e-12)


def test_maximum_grid_1024(gpu):
    """G = 1024 (1.07e9 cells, the largest grid accepted) against 300 samples."""
    G, Nc, Ns = 1024, 3, 100
    say("  building a separable 1024^3 density")
    rho = inputs.separable_density(G, seed=7)
    K = inputs.radial_spokes(Nc, Ns, 0.5, seed=8, jitter=0.05)
    prm = spk.Params(Nc, Ns, G, precision="fp32_comp")
    Kd, rd = device_problem(K, rho.astype(np.float32), "fp32_comp", gpu)
    say(f"  workspace {spk.workspace_size(prm) / 2**30:.3f} GiB")
    g, (pa, pr) = spk.grad(Kd, rd, prm, potentials=True)
    torch.cuda.synchronize()
    t = inputs.sample_targets(prm.p, 16, seed=9)
    rho32 = host64(rd)
    del rd
    say("  oracle on 16 targets x 1.07e9 cells")
    ref = oracle.grad(host64(Kd), rho32, G, 0.5, 0.0, t)
    err = rel_l2(host64(g)[:, t], ref["dF"])
    say(f"  G=1024 rel L2 {err:.3e}")
    assert err <= GRAD_TOL["fp32_comp"]
    assert rel_l2(host64(pa)[t], ref["ua"]) <= ENERGY_TOL["fp32_comp"]


def test_samples_beyond_2_to_the_30(gpu):
    """p = 1,073,743,872 samples (FP32): accumulator offsets pass 2^32; rows at both
    ends and in between against the oracle."""
    Nc, Ns, G = 524289, 2048, 4
    p = Nc * Ns
    prm = spk.Params(Nc, Ns, G, precision="fp32_comp")
    need = spk.workspace_size(prm) + 12 * p + (1 << 30)
    total = torch.cuda.get_device_properties(gpu).total_memory
    if total < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of device memory, {total / 2**30:.0f} present")
    say(f"  p={p}: drawing samples")
    K32 = inputs.uniform_points(p, 0.5, seed=10).astype(np.float32)
    rho = inputs.radial_density(G, 0.5, 0.1, 2.0)
    Kd = torch.from_numpy(K32).to(gpu)
    rd = torch.tensor(rho, dtype=torch.float32, device=gpu)
    say(f"  workspace {spk.workspace_size(prm) / 2**30:.1f} GiB")
    rows = [(0, 256), (p // 2 - 100, p // 2 + 156), (p - 256, p)]
    try:
        got = [host64(spk.grad(Kd, rd, prm, tgt=r)) for r in rows]
        torch.cuda.synchronize()
    finally:
        del Kd
        spk.api.release_workspaces()
        torch.cuda.empty_cache()
    t = np.array([0, 255, p // 2 - 100, p // 2 + 155, p - 256, p - 1], dtype=np.int64)
    g = np.concatenate(got, axis=1)[:, [0, 255, 256, 511, 512, 767]]
    say("  oracle on 6 targets x 1.07e9 samples")
    ref = oracle.grad(K32, host64(rd), G, 0.5, 0.0, t)
    err = rel_l2(g, ref["dF"])
    say(f"  p=2^30+ rel L2 {err:.3e}")
    assert err <= GRAD_TOL["fp32_comp"]
