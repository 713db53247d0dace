"""The allocation-free step (sparkling_step_async_noalloc, static device
scratch) against sparkling_step_async with a caller's workspace: two calls in
a row, the second on a smaller problem, every output bit for bit."""
import numpy as np
import pytest
import torch

from gpu_util import bounds, configs, device_problem, host64, inputs, say, spk

pytestmark = pytest.mark.gpu


def both_steps(K, rho, prm, it, eta, kp, gp, dev):
    """One step through each entry point from the same inputs and state."""
    out = []
    for noalloc in (False, True):
        Kd, rd = device_problem(K, rho, prm.precision, dev)
        state = spk.StepState(prm, dev)
        state.k_prev.copy_(torch.tensor(kp, dtype=prm.dtype))
        state.g_prev.copy_(torch.tensor(gp, dtype=prm.dtype))
        info = torch.full((16,), -1.0, dtype=torch.float64, device=dev)
        if noalloc:
            spk.step_async_noalloc_(Kd, rd, prm, state, it, eta, info)
        else:
            spk.step_async_(Kd, rd, prm, state, it, eta, info)
        torch.cuda.synchronize()
        out.append((Kd, state.k_prev, state.g_prev, info[:10]))
    return out


def assert_same(a, b):
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)
    assert np.array_equal(host64(a[3]), host64(b[3]), equal_nan=True)


def test_noalloc_step_matches_the_workspace_step(gpu):
    assert spk.noalloc_scratch_bytes() == 64 << 20
    # call 1: 128 x 512 samples on a 32^3 density, FP32-compensated, fixed step
    w = configs.C4
    a, b = bounds(w)
    prm = spk.Params(w.n_shots, w.n_samples, w.grid, precision="fp32_comp", a_max=a, b_max=b,
                     n_pit=w.n_pit)
    assert spk.workspace_size(prm) <= spk.noalloc_scratch_bytes()
    K = w.trajectory()
    z = np.zeros_like(K)
    say(f"  noalloc call 1: p = {prm.p}, {prm.precision}, iteration 0")
    ref, got = both_steps(K, w.density(), prm, 0, w.eta_fixed, z, z, gpu)
    assert_same(ref, got)
    assert np.isfinite(host64(got[3])[1])
    # call 2: a smaller problem in plain FP64, in the Barzilai-Borwein phase
    K2 = inputs.radial_spokes(16, 64, 0.5, seed=7, jitter=0.01)
    rho2 = inputs.radial_density(8, 0.5, 0.05, 2.0)
    prm2 = spk.Params(16, 64, 8, precision="plain_fp64", a_max=a, b_max=b, n_pit=200)
    kp = K2 + 1e-3 * inputs.uniform_points(K2.shape[1], 0.5, seed=8)
    gp = 1e-4 * inputs.uniform_points(K2.shape[1], 0.5, seed=9)
    say(f"  noalloc call 2: p = {prm2.p}, {prm2.precision}, iteration 21")
    ref, got = both_steps(K2, rho2, prm2, 21, 16.0, kp, gp, gpu)
    assert_same(ref, got)
    assert host64(got[3])[8] in (0.0, 1.0) and not np.isnan(host64(got[3])[9])


def test_noalloc_step_replayed_from_captured_graphs(gpu):
    """The allocation-free step captured in HIP graphs (fixed-step and
    Barzilai-Borwein phases), replayed 22 times with eager work and
    synchronisations between the replays: every replay bit for bit as the
    eager sparkling_step_async with a caller's workspace."""
    w = configs.C4
    a, b = bounds(w)
    prm = spk.Params(w.n_shots, w.n_samples, w.grid, precision="fp32_comp", a_max=a, b_max=b,
                     n_pit=w.n_pit)
    KA, rd = device_problem(w.trajectory(), w.density(), "fp32_comp", gpu)
    KB = KA.clone()
    sA, sB = spk.StepState(prm, gpu), spk.StepState(prm, gpu)
    ia = torch.zeros(16, dtype=torch.float64, device=gpu)
    ib = torch.zeros(16, dtype=torch.float64, device=gpu)
    # the first call on a device looks up the static scratch: made outside capture
    spk.step_async_noalloc_(KB.clone(), rd, prm, spk.StepState(prm, gpu), 0, w.eta_fixed, ib)
    torch.cuda.synchronize()
    graphs = {}
    for bb in (False, True):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            spk.step_async_noalloc_(KB, rd, prm, sB, 20 if bb else 0, w.eta_fixed, ib)
        graphs[bb] = g
    torch.cuda.synchronize()
    for it in range(22):
        spk.step_async_(KA, rd, prm, sA, it, w.eta_fixed, ia)
        graphs[it >= 20].replay()
        noise = torch.randn(1000, device=gpu).sum().item()   # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(KA, KB), it
        assert torch.equal(sA.g_prev, sB.g_prev), it
        assert np.array_equal(host64(ia[:10]), host64(ib[:10]), equal_nan=True), it
    say(f"  22 graph replays of the allocation-free step bit-identical ({noise:.3f})")


def test_noalloc_rejects_a_problem_beyond_its_scratch(gpu):
    w = configs.C2
    prm = spk.Params(w.n_shots, w.n_samples, w.grid, precision="fp32_comp", a_max=0.1,
                     b_max=0.01)
    Kd, rd = device_problem(np.zeros((3, prm.p)), np.zeros(w.grid ** 3), "fp32_comp", gpu)
    state = spk.StepState(prm, gpu)
    info = torch.zeros(16, dtype=torch.float64, device=gpu)
    with pytest.raises(spk.SparklingError) as e:
        spk.step_async_noalloc_(Kd, rd, prm, state, 0, 1.0, info)
    assert e.value.status == -2 and "static scratch" in str(e.value)
