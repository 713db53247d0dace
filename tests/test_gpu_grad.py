"""GPU energy/gradient parity against the FP64 oracle, through the C ABI.

Small cases compare every target; the full-size workloads compare sampled
targets (the oracle computes them one by one) after a full-size GPU run in the
launch configuration the benchmark times.
"""
import numpy as np
import pytest
import torch

from gpu_util import (ENERGY_TOL, GRAD_TOL, ROW_TOL, bounds, configs, device_problem, host64,
                      inputs, oracle, params_for, rel_l2, row_rel_max, say, spk, with_te_rows)

pytestmark = pytest.mark.gpu

ALL = ["plain_fp64", "fp32_comp", "fp32_acc64", "fp32_naive"]


def run_case(dev, K, rho, G, precision, L=0.5, eps=0.0, targets=None, with_energy=True):
    Nc, Ns = 1, K.shape[1]
    prm = spk.Params(Nc, Ns, G, precision=precision, half_width=L, eps=eps)
    Kd, rd = device_problem(K, rho, precision, dev)
    say(f"  grad {precision} p={prm.p} G={G} eps={eps}")
    g, (pa, pr), en = spk.grad(Kd, rd, prm, potentials=True, with_energy=True)
    torch.cuda.synchronize()
    ref = oracle.grad(host64(Kd), host64(rd), G, L, eps, targets)
    sel = slice(None) if targets is None else ref["targets"]
    return prm, Kd, rd, host64(g)[:, sel], host64(pa)[sel], host64(pr)[sel], en, ref


@pytest.mark.parametrize("precision", ALL)
def test_ragged_multi_tile_all_targets(gpu, precision):
    """p and G not multiples of any tile: ragged target blocks, tiles, rows and slabs."""
    K = inputs.radial_spokes(37, 113, 0.5, seed=17, jitter=0.05)
    rho = inputs.radial_density(13, 0.5, 0.0625, 2.0)
    prm, Kd, rd, g, pa, pr, en, ref = run_case(gpu, K, rho, 13, precision)
    tol = GRAD_TOL[precision]
    assert rel_l2(g, ref["dF"]) <= tol
    assert rel_l2(pa, ref["ua"]) <= ENERGY_TOL[precision]
    assert rel_l2(pr, ref["ur"]) <= ENERGY_TOL[precision]
    F, Fa, Fr = oracle.energy(host64(Kd), host64(rd), 13, 0.5)
    for got, want in zip(en, (F, Fa, Fr)):
        assert abs(got - want) <= ENERGY_TOL[precision] * abs(want)


@pytest.mark.parametrize("G", [3, 4, 8, 20, 21])
def test_cell_sweep_row_lengths(gpu, G):
    """FP32-comp cell sweep on rows of 3 (no whole group of four cells), 4 (one group),
    8, 20 (an odd number of groups) and 21 cells (groups and a remainder): every row
    length the read-ahead distinguishes, against the oracle on every target."""
    K = inputs.radial_spokes(9, 70, 0.5, seed=23, jitter=0.05)
    rho = inputs.radial_density(G, 0.5, 0.0625, 2.0)
    prm, Kd, rd, g, pa, pr, en, ref = run_case(gpu, K, rho, G, "fp32_comp")
    assert rel_l2(g, ref["dF"]) <= GRAD_TOL["fp32_comp"]
    assert rel_l2(pa, ref["ua"]) <= ENERGY_TOL["fp32_comp"]
    assert row_rel_max(g, ref["dF"]) <= ROW_TOL["fp32_comp"]


def test_c1_plain_fp64_every_target(gpu):
    w = configs.C1
    K, rho = w.trajectory(), w.density()
    prm, Kd, rd, g, pa, pr, en, ref = run_case(gpu, K, rho, w.grid, "plain_fp64")
    assert rel_l2(g, ref["dF"]) <= 1e-12
    assert np.abs(g - ref["dF"]).max() <= 1e-12 * np.abs(ref["dF"]).max()
    F, Fa, Fr = oracle.energy(host64(Kd), host64(rd), w.grid, 0.5)
    assert en[0] == pytest.approx(F, rel=1e-12, abs=0)
    assert en[1] == pytest.approx(Fa, rel=1e-13) and en[2] == pytest.approx(Fr, rel=1e-13)


@pytest.mark.parametrize("precision", ["plain_fp64", "fp32_comp"])
def test_regularised_kernel(gpu, precision):
    K = inputs.radial_spokes(9, 50, 0.5, seed=5, jitter=0.02)
    rho = inputs.radial_density(8, 0.5, 0.05, 2.0)
    eps = 2e-3
    prm, Kd, rd, g, pa, pr, en, ref = run_case(gpu, K, rho, 8, precision, eps=eps)
    assert rel_l2(g, ref["dF"]) <= GRAD_TOL[precision]
    F, Fa, Fr = oracle.energy(host64(Kd), host64(rd), 8, 0.5, eps)
    assert abs(en[2] - Fr) <= ENERGY_TOL[precision] * Fr


def test_discrepancy_output(gpu):
    w = configs.C1
    K = inputs.radial_spokes(16, 32, 0.5, seed=8, jitter=0.03)
    rho = inputs.radial_density(12, 0.5, 0.05, 2.0)
    prm = spk.Params(16, 32, 12, precision="plain_fp64", discrepancy=True)
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    F, Fa, Fr, D = spk.energy(Kd, rd, prm)
    oF, oFa, oFr = oracle.energy(K, rho, 12, 0.5)
    Erho = oracle.rho_self_energy(rho, 12, 0.5)
    assert F == pytest.approx(oF, rel=1e-12)
    assert D == pytest.approx(oF - Erho, rel=1e-9, abs=1e-15)
    assert D > 0
    prm.discrepancy = False
    assert np.isnan(spk.energy(Kd, rd, prm)[3])


def test_equilibrium_on_gpu(gpu):
    """Samples at the voxel centres with a uniform density: grad F = 0, D = 0."""
    G = 8
    ax = inputs.voxel_axis(G, 0.5)
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    K = np.stack([x.ravel(), y.ravel(), z.ravel()])
    rho = inputs.uniform_density(G)
    prm = spk.Params(G, G * G, G, precision="plain_fp64", discrepancy=True)
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    g, (pa, pr) = spk.grad(Kd, rd, prm, potentials=True)
    scale = float(host64(pa).max()) / prm.p
    assert np.abs(host64(g)).max() <= 1e-13 * scale
    F, Fa, Fr, D = spk.energy(Kd, rd, prm)
    assert abs(D) <= 1e-14 * Fa


def test_edge_cases(gpu):
    # one sample, one cell
    for precision in ("plain_fp64", "fp32_comp"):
        K = np.array([[0.1], [-0.2], [0.3]])
        prm, Kd, rd, g, pa, pr, en, ref = run_case(gpu, K, np.array([1.0]), 1, precision)
        np.testing.assert_allclose(g, ref["dF"], rtol=1e-6)
        assert pr[0] < 1e-9             # only the self pair: H(0)
    # all samples coincident: no repulsion force at all
    K = np.zeros((3, 300))
    prm, Kd, rd, g, pa, pr, en, ref = run_case(gpu, K, inputs.uniform_density(5), 5, "fp32_comp")
    assert np.abs(ref["dFr"]).max() == 0.0
    # the exact attraction at the centre of a symmetric grid is 0; compare at
    # FP32 rounding of the individual terms, |rho_v u| / p <= 1/(125 * 300)
    assert np.abs(g - ref["dF"]).max() <= 1e-6 / 300
    # empty target range
    prm = spk.Params(1, 300, 5)
    out = torch.empty((3, 0), device=gpu)
    spk.grad(Kd, rd, prm, tgt=(7, 7), out=out)


def test_chunk_invariance_and_rerun_bitwise(gpu):
    w = configs.C4
    K, rho = w.trajectory(), w.density()
    for precision in ("fp32_comp", "plain_fp64"):
        prm = spk.Params(w.n_shots, w.n_samples, w.grid, precision=precision)
        Kd, rd = device_problem(K, rho, precision, gpu)
        say(f"  chunks {precision} p={prm.p}")
        full = spk.grad(Kd, rd, prm)
        again = spk.grad(Kd, rd, prm)
        assert torch.equal(full, again)
        for chunk in (8192, 4096, 5000):
            parts = [spk.grad(Kd, rd, prm, tgt=(b, min(b + chunk, prm.p)))
                     for b in range(0, prm.p, chunk)]
            assert torch.equal(torch.cat(parts, dim=1), full), chunk


def test_repulsion_invariants_on_gpu(gpu):
    """Antisymmetry of the repulsion forces and reflection, on the GPU result."""
    K = np.round(inputs.uniform_points(4000, 0.5, seed=3) * 2 ** 16) / 2 ** 16
    prm = spk.Params(1, 4000, 1, precision="plain_fp64")
    rho = np.array([1.0])
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    Km, _ = device_problem(-K, rho, "plain_fp64", gpu)
    g, (pa, pr) = spk.grad(Kd, rd, prm, potentials=True)
    gm = spk.grad(Km, rd, prm)
    # the attraction to a single cell at the origin flips with K as well
    assert torch.equal(g, -gm)
    # sum of repulsion forces is zero: total force equals total attraction
    ga = oracle.grad(K, rho, 1, 0.5)["dFa"]
    tot = host64(g).sum(axis=1) - ga.sum(axis=1)
    assert np.abs(tot).max() <= 1e-13 * np.abs(ga).sum()


@pytest.mark.parametrize("precision", ["fp32_comp", "plain_fp64"])
def test_c2_sampled_targets(gpu, precision):
    w = configs.C2
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, precision)
    Kd, rd = device_problem(K, rho, precision, gpu)
    say(f"  c2 grad {precision} p={prm.p}")
    g, (pa, pr), en = spk.grad(Kd, rd, prm, potentials=True, with_energy=True)
    torch.cuda.synchronize()
    t = with_te_rows(inputs.sample_targets(prm.p, w.oracle_targets, seed=22), w.n_shots,
                     w.n_samples)
    ref = oracle.grad(host64(Kd), host64(rd), w.grid, 0.5, 0.0, t)
    err = rel_l2(host64(g)[:, t], ref["dF"])
    row = row_rel_max(host64(g)[:, t], ref["dF"])
    say(f"  c2 {precision} rel L2 = {err:.3e}, worst row {row:.3e}")
    assert err <= GRAD_TOL[precision]
    assert row <= ROW_TOL[precision]
    assert rel_l2(host64(pr)[t], ref["ur"]) <= ENERGY_TOL[precision]
    assert rel_l2(host64(pa)[t], ref["ua"]) <= ENERGY_TOL[precision]


def test_c3_full_size_sampled_targets(gpu):
    """8.4 M samples against a 192^3 density: the benchmark's configuration."""
    w = configs.C3
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, "fp32_comp")
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    say(f"  c3 grad fp32_comp p={prm.p} G={w.grid}")
    g, (pa, pr), en = spk.grad(Kd, rd, prm, potentials=True, with_energy=True)
    torch.cuda.synchronize()
    t = with_te_rows(inputs.sample_targets(prm.p, w.oracle_targets, seed=33), w.n_shots,
                     w.n_samples)
    say(f"  c3 oracle on {t.size} targets")
    ref = oracle.grad(host64(Kd), host64(rd), w.grid, 0.5, 0.0, t)
    err = rel_l2(host64(g)[:, t], ref["dF"])
    row = row_rel_max(host64(g)[:, t], ref["dF"])
    say(f"  c3 fp32_comp rel L2 = {err:.3e}, worst row {row:.3e}")
    assert err <= GRAD_TOL["fp32_comp"]
    assert row <= ROW_TOL["fp32_comp"]
    assert rel_l2(host64(pr)[t], ref["ur"]) <= ENERGY_TOL["fp32_comp"]
    assert rel_l2(host64(pa)[t], ref["ua"]) <= ENERGY_TOL["fp32_comp"]
    assert np.isfinite(en).all() and en[1] > en[2] > 0


def test_c2_all_fp32_forms_sampled_targets(gpu):
    """The three FP32 forms on the same stored inputs against one oracle pass."""
    w = configs.C2
    K, rho = w.trajectory(), w.density()
    t = inputs.sample_targets(w.p, 2048, seed=23)
    ref = None
    for precision in ("fp32_comp", "fp32_acc64", "fp32_naive"):
        prm = params_for(w, precision)
        Kd, rd = device_problem(K, rho, precision, gpu)
        g, (pa, pr) = spk.grad(Kd, rd, prm, potentials=True)
        torch.cuda.synchronize()
        if ref is None:
            ref = oracle.grad(host64(Kd), host64(rd), w.grid, 0.5, 0.0, t)
        err = rel_l2(host64(g)[:, t], ref["dF"])
        row = row_rel_max(host64(g)[:, t], ref["dF"])
        say(f"  c2 {precision} rel L2 = {err:.3e}, worst row {row:.3e} "
            f"(potentials {rel_l2(host64(pr)[t], ref['ur']):.3e})")
        assert err <= GRAD_TOL[precision]
        assert row <= ROW_TOL[precision]
