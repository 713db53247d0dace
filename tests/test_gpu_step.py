"""Projected gradient steps on the GPU against the oracle's steps."""
import numpy as np
import pytest
import torch

from gpu_util import bounds, configs, device_problem, host64, inputs, oracle, params_for, say, spk

pytestmark = pytest.mark.gpu


def test_c1_five_iterations_plain_fp64(gpu):
    w = configs.C1
    K, rho = w.trajectory(), w.density()
    a, b = bounds(w)
    prm = params_for(w, "plain_fp64")
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    state = spk.StepState(prm, gpu)
    Ko, kp, gp = K.copy(), np.zeros_like(K), np.zeros_like(K)
    for it in range(w.n_iters):
        say(f"  c1 step {it}")
        info = spk.step_(Kd, rd, prm, state, it, w.eta_fixed)
        Ko, kp, gp, oinfo = oracle.step(Ko, rho, w.n_shots, w.n_samples, w.grid, 0.5, a, b, 0,
                                        w.n_pit, kp, gp, it, w.eta_fixed)
        assert info["eta"] == oinfo["eta"]
        assert info["F"] == pytest.approx(oinfo["F"], rel=1e-12)
        assert np.abs(host64(Kd) - Ko).max() <= 1e-10
        assert np.abs(host64(state.g_prev) - gp).max() <= 1e-12 * np.abs(gp).max()
        np.testing.assert_allclose(info["viol"], oinfo["viol"], rtol=1e-8)
    # the energy decreased over the run
    assert oinfo["F"] < oracle.energy(K, rho, w.grid, 0.5)[0]


def test_barzilai_borwein_iterations(gpu):
    """Iterations 20.. use the BB step: compare eta with the oracle's."""
    w = configs.C1
    K = inputs.radial_spokes(16, 64, 0.5, seed=7, jitter=0.01)
    rho = w.density()
    a, b = bounds(w)
    prm = spk.Params(16, 64, w.grid, precision="plain_fp64", a_max=a, b_max=b, n_pit=200)
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    state = spk.StepState(prm, gpu)
    Ko, kp, gp = K.copy(), np.zeros_like(K), np.zeros_like(K)
    used = 0
    for it in range(18, 24):
        info = spk.step_(Kd, rd, prm, state, it, 16.0)
        Ko, kp, gp, oinfo = oracle.step(Ko, rho, 16, 64, w.grid, 0.5, a, b, 0, 200, kp, gp, it,
                                        16.0)
        assert info["bb_used"] == oinfo["bb_used"]
        assert info["eta"] == pytest.approx(oinfo["eta"], rel=1e-9)
        assert np.isnan(info["bb_quotient"]) == (it < 20)
        if it >= 20:
            assert info["bb_quotient"] == pytest.approx(oinfo["bb_quotient"], rel=1e-9)
        assert np.abs(host64(Kd) - Ko).max() <= 1e-9
        used += info["bb_used"]
    assert used >= 2


@pytest.mark.parametrize("precision", ["plain_fp64", "fp32_comp"])
@pytest.mark.parametrize("c1, c2, want, used", [
    (1 / 64, 1 / 16, 320 / 17, True),         # quotient 320/17 inside [1.6, 160]
    (5.0, 20.0, 1.6, True),                   # quotient 5/85 below: 0.1 * eta_fixed
    (1 / 6400, 1 / 1600, 160.0, True),        # quotient 32000/17 above: 10 * eta_fixed
    (-1 / 64, -1 / 16, 16.0, False),          # s.y < 0: the fixed step
])
def test_barzilai_borwein_known_quotient(gpu, precision, c1, c2, want, used):
    """States with a quotient s.s/s.y fixed by construction (tests/bb_states.py),
    through sparkling_step and sparkling_step_async: the device dots and the
    step rule give the quotient inside the clamp range, and the oracle's step."""
    from bb_states import bb_expected, bb_state, quantise
    w = configs.C1
    # a 2^-24 grid keeps K, k_prev = K - s and s exact in FP32 storage too
    K = quantise(inputs.radial_spokes(16, 64, 0.5, seed=7, jitter=0.01), bits=24)
    rho = w.density()
    a, b = bounds(w)
    prm = spk.Params(16, 64, w.grid, precision=precision, a_max=a, b_max=b, n_pit=200)
    Kd, rd = device_problem(K, rho, precision, gpu)
    Kh, rh = host64(Kd), host64(rd)
    g = oracle.grad(Kh, rh, w.grid, 0.5)["dF"]
    kp_exact, gp = bb_state(Kh, g, c1, c2, bits=24)
    # the state as the device stores it: k_prev stays exact in FP32, g_prev rounds once more
    kp = host64(torch.tensor(kp_exact, dtype=prm.dtype))
    gp = host64(torch.tensor(gp, dtype=prm.dtype))
    assert np.array_equal(kp, kp_exact)
    K1, _, _, oinfo = oracle.step(Kh, rh, 16, 64, w.grid, 0.5, a, b, 0, 200, kp, gp, 25, 16.0)
    assert oinfo["bb_used"] == used
    tol = 1e-12 if precision == "plain_fp64" else 2e-5
    if precision == "plain_fp64":
        assert oinfo["eta"] == pytest.approx(want, rel=1e-13)
    for mode in ("sync", "async"):
        say(f"  BB state c=({c1:.4g}, {c2:.4g}) {precision} {mode}")
        Kg = torch.tensor(Kh, dtype=prm.dtype, device=gpu)
        state = spk.StepState(prm, gpu)
        state.k_prev.copy_(torch.tensor(kp, dtype=prm.dtype))
        state.g_prev.copy_(torch.tensor(gp, dtype=prm.dtype))
        if mode == "sync":
            info = spk.step_(Kg, rd, prm, state, 25, 16.0)
        else:
            dinfo = torch.zeros(16, dtype=torch.float64, device=gpu)
            spk.step_async_(Kg, rd, prm, state, 25, 16.0, dinfo)
            torch.cuda.synchronize()
            info = spk.info_dict(dinfo)
        assert info["bb_used"] == used
        assert info["eta"] == pytest.approx(oinfo["eta"], rel=tol)
        assert info["bb_quotient"] == pytest.approx(oinfo["bb_quotient"], rel=tol)
        assert info["bb_quotient"] == pytest.approx(bb_expected(c1, c2), rel=tol)
        if used and 1.6 < want < 160.0:
            assert info["eta"] == pytest.approx(bb_expected(c1, c2), rel=tol)
        step = info["eta"] * np.abs(g).max()
        assert np.abs(host64(Kg) - K1).max() <= (1e-10 if precision == "plain_fp64"
                                                 else 1e-5 * step + 1e-7)


def test_fp32_step_and_resume_bitwise(gpu):
    """Saving the caller-owned state and resuming continues bit-identically."""
    w = configs.C4
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, "fp32_comp")
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    spk.project_(Kd, prm)
    state = spk.StepState(prm, gpu)
    for it in range(3):
        spk.step_(Kd, rd, prm, state, it, w.eta_fixed)
    saved = [Kd.clone(), state.k_prev.clone(), state.g_prev.clone()]
    ref = [spk.step_(Kd, rd, prm, state, it, w.eta_fixed) for it in (3, 4)]
    K2 = saved[0].clone()
    st2 = spk.StepState(prm, gpu)
    st2.k_prev.copy_(saved[1])
    st2.g_prev.copy_(saved[2])
    again = [spk.step_(K2, rd, prm, st2, it, w.eta_fixed) for it in (3, 4)]
    assert torch.equal(K2, Kd)
    for x, y in zip(ref, again):
        assert x["F"] == y["F"] and x["eta"] == y["eta"]
        assert np.array_equal(x["viol"], y["viol"])


def test_nonfinite_energy_reported(gpu):
    w = configs.C1
    prm = spk.Params(4, 16, 4, precision="fp32_comp", a_max=0.1, b_max=0.01)
    K = inputs.radial_spokes(4, 16, 0.5, seed=1)
    K[0, 5] = np.nan
    Kd, rd = device_problem(K, inputs.radial_density(4, 0.5, 0.05, 2.0), "fp32_comp", gpu)
    state = spk.StepState(prm, gpu)
    before = host64(Kd)
    kp, gp = state.k_prev.clone(), state.g_prev.clone()
    with pytest.raises(spk.SparklingError) as e:
        spk.step_(Kd, rd, prm, state, 0, 1.0)
    assert e.value.status == -5
    # nothing was updated
    np.testing.assert_array_equal(host64(Kd), before)
    assert torch.equal(state.k_prev, kp) and torch.equal(state.g_prev, gp)


def test_per_axis_steps_plain_fp64(gpu):
    """Three projected steps with rotation-variant bounds against the oracle."""
    w = configs.C1
    K, rho = w.trajectory(), w.density()
    a, b = bounds(w)
    prm = params_for(w, "plain_fp64")
    prm.rotation_variant = True
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    state = spk.StepState(prm, gpu)
    Ko, kp, gp = K.copy(), np.zeros_like(K), np.zeros_like(K)
    for it in range(3):
        say(f"  c1 per-axis step {it}")
        info = spk.step_(Kd, rd, prm, state, it, w.eta_fixed)
        Ko, kp, gp, oinfo = oracle.step(Ko, rho, w.n_shots, w.n_samples, w.grid, 0.5, a, b, 0,
                                        w.n_pit, kp, gp, it, w.eta_fixed, rotation_variant=True)
        assert info["F"] == pytest.approx(oinfo["F"], rel=1e-12)
        assert np.abs(host64(Kd) - Ko).max() <= 1e-10
        np.testing.assert_allclose(info["viol"], oinfo["viol"], rtol=1e-8)


def test_c3_step_sampled_shots(gpu):
    """One step of the benchmark's configuration (4096 x 2048 samples, 192^3 density,
    FP32-compensated, n_pit = 200), checked on two whole shots: the oracle's gradient
    rows of those shots, the same descent, and the oracle's projection of each shot."""
    w = configs.C3
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, "fp32_comp")
    a, b = prm.a_max, prm.b_max
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    K0 = host64(Kd)
    state = spk.StepState(prm, gpu)
    say("  c3 step")
    info = spk.step_(Kd, rd, prm, state, 0, w.eta_fixed)
    K1 = host64(Kd)
    Ns, last = w.n_samples, w.n_shots - 1
    t = np.concatenate([np.arange(Ns), last * Ns + np.arange(Ns)])
    say("  c3 oracle gradient on 2 shots (4096 targets)")
    g = oracle.grad(K0, host64(rd), w.grid, 0.5, 0.0, t)["dF"]
    half = K0[:, t] - info["eta"] * g
    want = oracle.project(half, 2, Ns, 0.5, a, b, 0, w.n_pit)
    got = K1[:, t]
    diff = np.abs(got - want).max()
    say(f"  c3 step: eta {info['eta']:.6g}, max |K_gpu - K_oracle| on 2 shots {diff:.3e}")
    assert info["eta"] == w.eta_fixed
    assert diff <= 1e-6     # FP32 storage of K (about 3e-8 at |k| <= 0.5) plus FP32-comp rows
    assert np.all(got[:, [0, Ns]] == 0.0) and np.abs(got).max() <= 0.5
    # Feasibility after n_pit = 200 from the jittered start (slew 540x over the
    # bound): box and TE exact, speed within its bound, slew left above it at
    # the levels measured with the oracle (2.20 on these two shots, 4.22 over
    # all 4096; about 3000 iterations bring these shots within 1%).  Bounds
    # that catch a regression of the projection or of the step before it.
    v2 = oracle.constraint_check(got, 2, Ns, 0.5, a, b, 0)
    say(f"  c3 step violations: all shots {np.round(info['viol'], 4).tolist()}, two shots "
        f"{np.round(v2, 4).tolist()}")
    assert info["viol"][2] <= 1.0 and info["viol"][3] == 0.0
    assert info["viol"][0] <= 1.0 and info["viol"][1] <= 4.5
    assert v2[0] <= 1.0 and v2[1] <= 2.3
