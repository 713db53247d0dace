"""The logarithmic kernel H(d) = log(|d|^2 + eps^2)/2 and the regularised-kernel
step policy on the GPU, through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest
import torch

from gpu_util import (ENERGY_TOL, GRAD_TOL, configs, device_problem, host64, inputs, oracle,
                      params_for, rel_l2, say, spk)

pytestmark = pytest.mark.gpu


def spacing(p, L=0.5):
    """Mean sample spacing of p samples spread over [-L, L]^3."""
    return 2 * L / p ** (1.0 / 3.0)


@pytest.mark.parametrize("precision", ["plain_fp64", "fp32_comp"])
def test_log_kernel_ragged_all_targets(gpu, precision):
    K = inputs.radial_spokes(37, 113, 0.5, seed=23, jitter=0.05)
    rho = inputs.radial_density(13, 0.5, 0.0625, 2.0)
    eps = 0.25 * spacing(K.shape[1])
    prm = spk.Params(37, 113, 13, precision=precision, eps=eps, kernel="log")
    Kd, rd = device_problem(K, rho, precision, gpu)
    say(f"  log kernel {precision} p={prm.p} eps={eps:.4g}")
    g, (pa, pr), en = spk.grad(Kd, rd, prm, potentials=True, with_energy=True)
    ref = oracle.grad(host64(Kd), host64(rd), 13, 0.5, eps, kernel="log")
    assert rel_l2(host64(g), ref["dF"]) <= GRAD_TOL[precision]
    assert rel_l2(host64(pa), ref["ua"]) <= ENERGY_TOL[precision]
    assert rel_l2(host64(pr), ref["ur"]) <= ENERGY_TOL[precision]
    F, Fa, Fr = oracle.energy(host64(Kd), host64(rd), 13, 0.5, eps, kernel="log")
    for got, want in zip(en, (F, Fa, Fr)):
        assert abs(got - want) <= ENERGY_TOL[precision] * abs(want)
    # the distance kernel gives a different gradient on the same input
    prm.kernel = "distance"
    assert rel_l2(host64(spk.grad(Kd, rd, prm)), ref["dF"]) > 1e-2


def test_log_kernel_c1_plain_fp64_and_discrepancy(gpu):
    w = configs.C1
    K, rho = w.trajectory(), w.density()
    eps = 0.25 * spacing(K.shape[1])
    prm = params_for(w, "plain_fp64", eps=eps, kernel="log", discrepancy=True)
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    g = host64(spk.grad(Kd, rd, prm))
    ref = oracle.grad(K, rho, w.grid, 0.5, eps, kernel="log")
    assert rel_l2(g, ref["dF"]) <= 1e-12
    F, Fa, Fr, D = spk.energy(Kd, rd, prm)
    oF, oFa, oFr = oracle.energy(K, rho, w.grid, 0.5, eps, kernel="log")
    assert F == pytest.approx(oF, rel=1e-12) and Fr == pytest.approx(oFr, rel=1e-12)
    Erho = oracle.rho_self_energy(rho, w.grid, 0.5, eps, kernel="log")
    assert D == pytest.approx(oF - Erho, rel=1e-9, abs=1e-12)


def test_log_kernel_c2_sampled_targets(gpu):
    """524,288 samples on 128^3 in the compensated FP32 form, 512 oracle targets."""
    w = configs.C2
    K, rho = w.trajectory(), w.density()
    eps = 0.25 * spacing(K.shape[1])
    prm = params_for(w, "fp32_comp", eps=eps, kernel="log")
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    say("  c2 log kernel gradient")
    g = host64(spk.grad(Kd, rd, prm))
    t = inputs.sample_targets(prm.p, 512, seed=3)
    say("  c2 log kernel oracle on 512 targets")
    ref = oracle.grad(host64(Kd), host64(rd), w.grid, 0.5, eps, targets=t, kernel="log")
    err = rel_l2(g[:, t], ref["dF"])
    say(f"  c2 log kernel rel L2 {err:.3e}")
    assert err <= GRAD_TOL["fp32_comp"]


@pytest.mark.parametrize("precision,tol", [("plain_fp64", 1e-12), ("fp32_comp", 1e-6)])
def test_log_kernel_node_field(gpu, precision, tol):
    G, L = 7, 0.5
    eps = 0.05
    rho = inputs.radial_density(G, L, 0.1, 2.0)
    prm = spk.Params(1, 8, G, precision=precision, eps=eps, kernel="log")
    _, rd = device_problem(np.zeros((3, 8)), rho, precision, gpu)
    f = host64(spk.attraction_field(rd, prm))
    want = oracle.field(host64(rd), G, L, eps, kernel="log")
    assert rel_l2(f, want) <= tol
    K = inputs.radial_spokes(11, 30, L, seed=4, jitter=0.05)
    Kd, _ = device_problem(K, rho, precision, gpu)
    prm = spk.Params(11, 30, G, precision=precision, eps=eps, kernel="log")
    prm.attraction_field = spk.attraction_field(rd, prm)
    g = host64(spk.grad(Kd, rd, prm))
    ref = oracle.grad_field(host64(Kd), host64(rd), G, L, eps, kernel="log")
    assert rel_l2(g, ref["dF"]) <= 10 * GRAD_TOL[precision]


def test_log_kernel_steps_plain_fp64(gpu):
    w = configs.C1
    K, rho = w.trajectory(), w.density()
    eps = 0.25 * spacing(K.shape[1])
    prm = params_for(w, "plain_fp64", eps=eps, kernel="log")
    a, b = prm.a_max, prm.b_max
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    state = spk.StepState(prm, gpu)
    eta = 1.0 / spk.lipschitz_bound(prm.p, eps, float(rho.sum()), "log")
    Ko, kp, gp = K.copy(), np.zeros_like(K), np.zeros_like(K)
    for it in range(3):
        say(f"  c1 log-kernel step {it}")
        info = spk.step_(Kd, rd, prm, state, it, eta)
        Ko, kp, gp, oinfo = oracle.step(Ko, rho, w.n_shots, w.n_samples, w.grid, 0.5, a, b, 0,
                                        w.n_pit, kp, gp, it, eta, eps, kernel="log")
        assert info["F"] == pytest.approx(oinfo["F"], rel=1e-12)
        assert np.abs(host64(Kd) - Ko).max() <= 1e-10


@pytest.mark.parametrize("wname,precision,kernel", [("c5_loop", "fp32_comp", "distance"),
                                                    ("c2_fp32_grad", "fp32_comp", "log"),
                                                    ("c1_plain_fp64_loop", "plain_fp64", "log")])
def test_lipschitz_step_decreases_f(gpu, wname, precision, kernel):
    """Fixed step 1/L with the library's bound and an exact projection (box and TE:
    n_pit = 0, unbounded speed and slew): every step lowers F by at least
    (L/2)|K+ - K|^2.  At full size this checks the regularised step end to end."""
    w = configs.WORKLOADS[wname]
    K, rho = w.trajectory(), w.density()
    eps = spacing(K.shape[1])
    prm = params_for(w, precision, eps=eps, kernel=kernel, a_max=1e3, b_max=1e3, n_pit=0)
    lip = spk.lipschitz_bound(prm.p, eps, float(rho.sum()), kernel)
    Kd, rd = device_problem(K, rho, precision, gpu)
    state = spk.StepState(prm, gpu)
    F_prev, K_prev = None, None
    for it in range(4):
        say(f"  {wname} {kernel} step {it} (eta = 1/L = {1 / lip:.4g})")
        K_in = host64(Kd)
        info = spk.step_(Kd, rd, prm, state, it, 1.0 / lip)
        if F_prev is not None:
            drop = 0.5 * lip * float(((K_in - K_prev) ** 2).sum())
            slack = ENERGY_TOL[precision] * abs(F_prev) * 4
            say(f"    F {F_prev:.12e} -> {info['F']:.12e}, guaranteed drop {drop:.3e}")
            assert drop > 10 * slack
            assert info["F"] <= F_prev - drop + slack
        F_prev, K_prev = info["F"], K_in
