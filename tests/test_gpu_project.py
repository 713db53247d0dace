"""GPU projection and constraint check against the FP64 oracle, through the C ABI.

Both sides run the same dual iteration in the same operation order with no
floating-point contraction, so the FP64 results are compared bit for bit.
"""
import numpy as np
import pytest
import torch

from gpu_util import bounds, configs, device_problem, host64, inputs, oracle, params_for, say, spk

pytestmark = pytest.mark.gpu


def project_both(dev, K, Nc, Ns, a, b, te, n_pit, precision="plain_fp64", L=0.5):
    prm = spk.Params(Nc, Ns, 1, precision=precision, half_width=L, a_max=a, b_max=b,
                     te_index=te, n_pit=n_pit)
    Kd, _ = device_problem(K, [1.0], precision, dev)
    K_in = host64(Kd)
    say(f"  project {precision} Nc={Nc} Ns={Ns} te={te} n_pit={n_pit}")
    viol = spk.project_(Kd, prm)
    ref = oracle.project(K_in, Nc, Ns, L, a, b, te, n_pit)
    return prm, Kd, host64(Kd), ref, viol


@pytest.mark.parametrize("Ns", [2, 3, 5, 64, 1000, 1024, 1025, 2048, 4096])
def test_projection_bitwise_fp64(gpu, Ns):
    Nc = 6
    K = inputs.radial_spokes(Nc, Ns, 0.5, seed=Ns, jitter=0.05)
    a, b = bounds(configs.C5)
    prm, Kd, got, ref, viol = project_both(gpu, K, Nc, Ns, a, b, 0, 200)
    assert np.array_equal(got, ref), np.abs(got - ref).max()
    assert np.array_equal(viol, oracle.constraint_check(got, Nc, Ns, 0.5, a, b, 0))


@pytest.mark.parametrize("te", [-1, 0, 7])
def test_projection_te_and_box_exact(gpu, te):
    Nc, Ns = 5, 40
    rng = np.random.default_rng(3)
    K = rng.uniform(-0.9, 0.9, (3, Nc * Ns))
    prm, Kd, got, ref, viol = project_both(gpu, K, Nc, Ns, 0.05, 0.01, te, 100)
    assert np.array_equal(got, ref)
    assert np.abs(got).max() <= 0.5
    if te >= 0:
        assert np.all(got[:, te::Ns] == 0.0) and viol[3] == 0.0


@pytest.mark.parametrize("Ns,precision", [(64, "plain_fp64"), (1025, "plain_fp64"),
                                          (2048, "plain_fp64"), (300, "fp32_comp")])
def test_warm_started_projection_bitwise(gpu, Ns, precision):
    """Duals carried by the caller (spk_params.proj_duals): two projections in a
    row from a nonzero start, output and dual state equal to the oracle's."""
    Nc = 5
    K = inputs.radial_spokes(Nc, Ns, 0.5, seed=Ns + 1, jitter=0.05)
    a, b = bounds(configs.C5)
    rng = np.random.default_rng(Ns)
    d0 = rng.normal(scale=1e-3, size=(Nc, 6, Ns))
    d0[:, :3, Ns - 1] = 0.0
    d0[:, 3:, Ns - 2:] = 0.0
    duals = torch.tensor(d0, device=gpu)
    prm = spk.Params(Nc, Ns, 1, precision=precision, a_max=a, b_max=b, n_pit=150,
                     proj_duals=duals)
    Kd, _ = device_problem(K, [1.0], precision, gpu)
    ref_d = d0.copy()
    ref = host64(Kd)
    for call in range(2):
        say(f"  warm projection {precision} Ns={Ns} call {call}")
        if call == 1:     # the next input: a small move of the projected shots
            Kd += torch.tensor(rng.uniform(-1e-3, 1e-3, K.shape), dtype=Kd.dtype, device=gpu)
            ref = host64(Kd)
        viol = spk.project_(Kd, prm)
        ref = oracle.project(ref, Nc, Ns, 0.5, a, b, 0, 150, duals=ref_d)
        if precision != "plain_fp64":
            ref = ref.astype(np.float32).astype(np.float64)
        assert np.array_equal(host64(Kd), ref), np.abs(host64(Kd) - ref).max()
        assert np.array_equal(host64(duals), ref_d)
        assert np.array_equal(viol, oracle.constraint_check(host64(Kd), Nc, Ns, 0.5, a, b, 0))


@pytest.mark.parametrize("Ns", [64, 1025, 2048])
def test_warm_start_ignores_entries_past_the_ranges(gpu, Ns):
    """Dual slots past their ranges (q[Ns-1], r[Ns-2], r[Ns-1]) hold NaN on entry:
    the projection reads them as 0 and writes 0 there, like the oracle, and the
    output equals the oracle's bit for bit."""
    Nc = 3
    K = inputs.radial_spokes(Nc, Ns, 0.5, seed=Ns + 7, jitter=0.05)
    a, b = bounds(configs.C5)
    rng = np.random.default_rng(Ns + 7)
    d0 = rng.normal(scale=1e-3, size=(Nc, 6, Ns))
    d0[:, :3, Ns - 1] = np.nan
    d0[:, 3:, Ns - 2:] = np.nan
    duals = torch.tensor(d0, device=gpu)
    prm = spk.Params(Nc, Ns, 1, precision="plain_fp64", a_max=a, b_max=b, n_pit=80,
                     proj_duals=duals)
    Kd, _ = device_problem(K, [1.0], "plain_fp64", gpu)
    ref_d = d0.copy()
    ref = oracle.project(host64(Kd), Nc, Ns, 0.5, a, b, 0, 80, duals=ref_d)
    say(f"  warm projection with NaN past the ranges, Ns={Ns}")
    spk.project_(Kd, prm)
    assert np.array_equal(host64(Kd), ref), np.abs(host64(Kd) - ref).max()
    got_d = host64(duals)
    assert np.array_equal(got_d, ref_d)
    assert not np.isnan(got_d).any()
    assert np.all(got_d[:, :3, Ns - 1] == 0.0) and np.all(got_d[:, 3:, Ns - 2:] == 0.0)


def test_warm_started_per_axis_projection_bitwise(gpu):
    """Warm-started duals with per-axis (rotation-variant) bounds: two
    projections in a row, output and dual state equal to the oracle's."""
    Nc, Ns = 4, 333
    K = inputs.radial_spokes(Nc, Ns, 0.5, seed=81, jitter=0.05)
    a, b = bounds(configs.C5)
    duals = torch.zeros((Nc, 6, Ns), dtype=torch.float64, device=gpu)
    prm = spk.Params(Nc, Ns, 1, precision="plain_fp64", a_max=a, b_max=b, n_pit=120,
                     rotation_variant=True, proj_duals=duals)
    Kd, _ = device_problem(K, [1.0], "plain_fp64", gpu)
    ref, ref_d = host64(Kd), np.zeros((Nc, 6, Ns))
    rng = np.random.default_rng(82)
    for call in range(2):
        if call == 1:
            Kd += torch.tensor(rng.uniform(-1e-3, 1e-3, K.shape), dtype=Kd.dtype, device=gpu)
            ref = host64(Kd)
        spk.project_(Kd, prm)
        ref = oracle.project(ref, Nc, Ns, 0.5, a, b, 0, 120, rotation_variant=True, duals=ref_d)
        assert np.array_equal(host64(Kd), ref)
        assert np.array_equal(host64(duals), ref_d)


def test_warm_started_steps_match_the_oracle(gpu):
    """Projected gradient steps with carried duals, in plain FP64, step by step
    against the oracle's steps with the same dual state."""
    w = configs.C1
    K, rho = w.trajectory(), w.density()
    a, b = bounds(w)
    duals = spk.new_duals(spk.Params(w.n_shots, w.n_samples, w.grid), gpu)
    prm = params_for(w, "plain_fp64", proj_duals=duals)
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    state = spk.StepState(prm, gpu)
    Ko, kp, gp = K.copy(), np.zeros_like(K), np.zeros_like(K)
    od = np.zeros((w.n_shots, 6, w.n_samples))
    for it in range(4):
        info = spk.step_(Kd, rd, prm, state, it, w.eta_fixed)
        Ko, kp, gp, oinfo = oracle.step(Ko, rho, w.n_shots, w.n_samples, w.grid, 0.5, a, b, 0,
                                        w.n_pit, kp, gp, it, w.eta_fixed, duals=od)
        assert info["F"] == pytest.approx(oinfo["F"], rel=1e-12)
        assert np.abs(host64(Kd) - Ko).max() <= 1e-10
        assert np.abs(host64(duals) - od).max() <= 1e-9 * max(np.abs(od).max(), 1e-30)


def test_projection_fp32_storage(gpu):
    """FP32 trajectories: FP64 iteration on the widened values, one rounding on output."""
    Nc, Ns = 8, 300
    K = inputs.radial_spokes(Nc, Ns, 0.5, seed=4, jitter=0.05)
    a, b = bounds(configs.C5)
    prm, Kd, got, ref, viol = project_both(gpu, K, Nc, Ns, a, b, 0, 200, "fp32_comp")
    assert np.array_equal(got, ref.astype(np.float32).astype(np.float64))
    assert np.array_equal(viol, oracle.constraint_check(got, Nc, Ns, 0.5, a, b, 0))


def test_feasible_input_is_unchanged_bitwise(gpu):
    rng = np.random.default_rng(9)
    Nc, Ns, a, b = 4, 128, 0.05, 0.004
    shots = []
    for _ in range(Nc):
        acc = rng.normal(size=(3, Ns))
        acc *= 0.4 * b / np.linalg.norm(acc, axis=0).max()
        vel = np.cumsum(acc, axis=1)
        vel *= min(1.0, 0.4 * a / np.linalg.norm(vel, axis=0).max())
        s = np.concatenate([np.zeros((3, 1)), np.cumsum(vel, axis=1)[:, :-1]], axis=1)
        s *= min(1.0, 0.4 / np.abs(s).max())      # shrinking keeps speed and slew feasible
        shots.append(s)
    K = np.concatenate(shots, axis=1)
    assert oracle.constraint_check(K, Nc, Ns, 0.5, a, b, 0).max() < 1
    prm, Kd, got, ref, viol = project_both(gpu, K, Nc, Ns, a, b, 0, 200)
    assert np.array_equal(got, K) and np.array_equal(ref, K)
    assert viol[0] < 1 and viol[1] < 1 and viol[2] < 1


def test_projection_rerun_bitwise_and_violation(gpu):
    w = configs.C5
    K = inputs.radial_spokes(64, w.n_samples, 0.5, seed=12, jitter=w.jitter)
    a, b = bounds(w)
    outs = []
    for _ in range(2):
        prm, Kd, got, ref, viol = project_both(gpu, K, 64, w.n_samples, a, b, 0, w.n_pit,
                                               "fp32_comp")
        outs.append((got, viol))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    viol = outs[0][1]
    say(f"  violations after {w.n_pit} iterations: {viol}")
    assert viol[2] <= 1.0 and viol[3] == 0.0
    assert viol[0] < 1.5 and viol[1] < 2.0


def test_c5_full_size_projection(gpu):
    """2048 shots x 1024 samples, 200 iterations: every shot matches the oracle."""
    w = configs.C5
    K = w.trajectory()
    a, b = bounds(w)
    prm, Kd, got, ref, viol = project_both(gpu, K, w.n_shots, w.n_samples, a, b, 0, w.n_pit,
                                           "fp32_comp")
    assert np.array_equal(got, ref.astype(np.float32).astype(np.float64))
    want = oracle.constraint_check(got, w.n_shots, w.n_samples, 0.5, a, b, 0)
    assert np.array_equal(viol, want)


def test_constraint_check_bitwise(gpu):
    rng = np.random.default_rng(2)
    Nc, Ns = 33, 257
    K = rng.uniform(-0.6, 0.6, (3, Nc * Ns))
    for precision in ("plain_fp64", "fp32_comp"):
        prm = spk.Params(Nc, Ns, 1, precision=precision, a_max=0.07, b_max=0.011, te_index=5)
        Kd, _ = device_problem(K, [1.0], precision, gpu)
        got = spk.constraint_check(Kd, prm)
        want = oracle.constraint_check(host64(Kd), Nc, Ns, 0.5, 0.07, 0.011, 5)
        assert np.array_equal(got, want)
    K[1, 100] = np.nan
    Kd, _ = device_problem(K, [1.0], "plain_fp64", gpu)
    prm = spk.Params(Nc, Ns, 1, precision="plain_fp64", a_max=0.07, b_max=0.011)
    assert np.isnan(spk.constraint_check(Kd, prm)[:3]).all()


@pytest.mark.parametrize("precision,Ns", [("plain_fp64", 3), ("plain_fp64", 1025),
                                          ("fp32_comp", 1024)])
def test_per_axis_projection_bitwise(gpu, precision, Ns):
    """Rotation-variant bounds: per-coordinate dual prox, per-axis check."""
    Nc = 6
    K = inputs.radial_spokes(Nc, Ns, 0.5, seed=Ns + 1, jitter=0.05)
    a, b = bounds(configs.C5)
    prm = spk.Params(Nc, Ns, 1, precision=precision, a_max=a, b_max=b, te_index=0, n_pit=200,
                     rotation_variant=True)
    Kd, _ = device_problem(K, [1.0], precision, gpu)
    K_in = host64(Kd)
    say(f"  per-axis project {precision} Nc={Nc} Ns={Ns}")
    viol = spk.project_(Kd, prm)
    got = host64(Kd)
    ref = oracle.project(K_in, Nc, Ns, 0.5, a, b, 0, 200, rotation_variant=True)
    if precision == "fp32_comp":
        ref = ref.astype(np.float32).astype(np.float64)
    assert np.array_equal(got, ref), np.abs(got - ref).max()
    want = oracle.constraint_check(got, Nc, Ns, 0.5, a, b, 0, rotation_variant=True)
    assert np.array_equal(viol, want)
    # the Euclidean form gives a different result on the same input
    prm.rotation_variant = False
    Kd2, _ = device_problem(K, [1.0], precision, gpu)
    spk.project_(Kd2, prm)
    assert not np.array_equal(host64(Kd2), got)


def test_per_axis_constraint_check_bitwise(gpu):
    rng = np.random.default_rng(21)
    Nc, Ns = 17, 130
    K = rng.uniform(-0.6, 0.6, (3, Nc * Ns))
    prm = spk.Params(Nc, Ns, 1, precision="plain_fp64", a_max=0.07, b_max=0.011, te_index=3,
                     rotation_variant=True)
    Kd, _ = device_problem(K, [1.0], "plain_fp64", gpu)
    got = spk.constraint_check(Kd, prm)
    want = oracle.constraint_check(K, Nc, Ns, 0.5, 0.07, 0.011, 3, rotation_variant=True)
    assert np.array_equal(got, want)
    assert not np.array_equal(got, oracle.constraint_check(K, Nc, Ns, 0.5, 0.07, 0.011, 3))
