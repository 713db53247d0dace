"""The projected gradient step without host synchronisation (sparkling_step_async)
and its capture in a HIP graph, against the synchronous step."""
import numpy as np
import pytest
import torch

from gpu_util import configs, device_problem, host64, inputs, params_for, say, spk

pytestmark = pytest.mark.gpu


def same_info(a, b):
    assert a["eta"] == b["eta"] and a["F"] == b["F"] and a["Fa"] == b["Fa"]
    assert a["Fr"] == b["Fr"] and a["bb_used"] == b["bb_used"]
    assert np.array_equal(a["viol"], b["viol"])
    assert np.array_equal([a["bb_quotient"]], [b["bb_quotient"]], equal_nan=True)


@pytest.mark.parametrize("wname,precision", [("c1_plain_fp64_loop", "plain_fp64"),
                                             ("c4_autograd", "fp32_comp")])
def test_async_step_matches_sync_bitwise(gpu, wname, precision):
    """24 steps (the fixed step, then Barzilai-Borwein): same K, state and info bits."""
    w = configs.WORKLOADS[wname]
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, precision)
    KA, rd = device_problem(K, rho, precision, gpu)
    KB = KA.clone()
    sA, sB = spk.StepState(prm, gpu), spk.StepState(prm, gpu)
    info = torch.zeros(10, dtype=torch.float64, device=gpu)
    eta = w.eta_fixed
    used = 0
    for it in range(24):
        ia = spk.step_(KA, rd, prm, sA, it, eta)
        spk.step_async_(KB, rd, prm, sB, it, eta, info)
        ib = spk.info_dict(info)
        same_info(ia, ib)
        assert torch.equal(KA, KB)
        assert torch.equal(sA.k_prev, sB.k_prev) and torch.equal(sA.g_prev, sB.g_prev)
        used += ia["bb_used"]
    say(f"  {wname} {precision}: 24 async steps bit-identical, BB used {used} times")
    assert used >= 1


def test_graph_replays_match_eager_steps(gpu):
    """Two captured graphs (fixed-step phase, BB phase) replayed 24 times with eager
    work and synchronisations between replays; every replay against the eager step."""
    w = configs.C4
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, "fp32_comp")
    KA, rd = device_problem(K, rho, "fp32_comp", gpu)
    KB = KA.clone()
    sA, sB = spk.StepState(prm, gpu), spk.StepState(prm, gpu)
    eta = w.eta_fixed
    fixed = spk.StepGraph(KB, rd, prm, sB, eta, barzilai_borwein=False)
    bb = spk.StepGraph(KB, rd, prm, sB, eta, barzilai_borwein=True)
    assert torch.equal(KA, KB)             # capturing runs nothing
    for it in range(24):
        ia = spk.step_(KA, rd, prm, sA, it, eta)
        g = bb if it >= 20 else fixed
        g.replay()
        noise = torch.randn(1000, device=gpu).sum().item()   # eager work between replays
        torch.cuda.synchronize()
        ib = spk.info_dict(g.info)
        same_info(ia, ib)
        assert torch.equal(KA, KB), it
        assert torch.equal(sA.g_prev, sB.g_prev), it
    say(f"  24 graph replays bit-identical to eager steps ({noise:.3f})")


def test_async_step_with_nonfinite_energy_changes_nothing(gpu):
    prm = spk.Params(4, 16, 4, precision="fp32_comp", a_max=0.1, b_max=0.01)
    K = inputs.radial_spokes(4, 16, 0.5, seed=1)
    K[1, 7] = np.nan
    Kd, rd = device_problem(K, inputs.radial_density(4, 0.5, 0.05, 2.0), "fp32_comp", gpu)
    state = spk.StepState(prm, gpu)
    state.k_prev.fill_(0.25)
    before, kp = host64(Kd), state.k_prev.clone()
    info = torch.zeros(10, dtype=torch.float64, device=gpu)
    spk.step_async_(Kd, rd, prm, state, 3, 1.0, info)
    d = spk.info_dict(info)
    assert np.isnan(d["F"]) and np.isnan(d["eta"]) and not d["bb_used"]
    np.testing.assert_array_equal(host64(Kd), before)
    assert torch.equal(state.k_prev, kp)
