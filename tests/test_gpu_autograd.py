"""F as a torch.autograd.Function: backward is the gradient kernel, recomputed in chunks."""
import json
import os

import numpy as np
import pytest
import torch

from gpu_util import configs, device_problem, host64, inputs, oracle, rel_l2, say, spk

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def c4_fd_golden():
    with open(os.path.join(GOLDEN, "c4_fd.json")) as f:
        meta = json.load(f)
    return meta, np.load(os.path.join(GOLDEN, "c4_fd.npy"))

pytestmark = pytest.mark.gpu


def test_gradcheck_plain_fp64(gpu):
    K = inputs.uniform_points(48, 0.5, seed=4)
    rho = inputs.radial_density(4, 0.5, 0.1, 2.0)
    prm = spk.Params(3, 16, 4, precision="plain_fp64")
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    Kd.requires_grad_(True)
    f = lambda k: spk.SparklingEnergy.apply(k, rd, prm, 16)
    assert torch.autograd.gradcheck(f, (Kd,), eps=1e-6, atol=1e-9, rtol=1e-6)


def test_gradcheck_log_kernel(gpu):
    K = inputs.uniform_points(48, 0.5, seed=5)
    rho = inputs.radial_density(4, 0.5, 0.1, 2.0)
    prm = spk.Params(3, 16, 4, precision="plain_fp64", eps=0.05, kernel="log")
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    Kd.requires_grad_(True)
    f = lambda k: spk.SparklingEnergy.apply(k, rd, prm, 16)
    assert torch.autograd.gradcheck(f, (Kd,), eps=1e-6, atol=1e-9, rtol=1e-6)
    F = f(Kd)
    prm.kernel = "distance"        # a later change of prm does not reach backward
    F.backward()
    ref = oracle.grad(K, rho, 4, 0.5, 0.05, kernel="log")["dF"]
    assert rel_l2(host64(Kd.grad), ref) <= 1e-12


def test_coincident_samples_backward_matches_central_differences(gpu):
    """Every shot starts at the origin: the zero subgradient is what central FD sees."""
    K = inputs.radial_spokes(4, 8, 0.5, seed=2, jitter=0.05)
    rho = inputs.radial_density(4, 0.5, 0.1, 2.0)
    prm = spk.Params(4, 8, 4, precision="plain_fp64")
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    Kd.requires_grad_(True)
    F = spk.SparklingEnergy.apply(Kd, rd, prm, 8)
    F.backward()
    g = host64(Kd.grad)
    for k in range(5):
        e = inputs.rademacher(K.shape, 40 + k)
        fd = oracle.fd_directional(K, rho, 4, 0.5, e, 1e-6)
        assert fd == pytest.approx(float((g * e).sum()), rel=1e-7, abs=1e-12)


def test_double_backward_unsupported(gpu):
    prm = spk.Params(2, 8, 2, precision="plain_fp64")
    Kd, rd = device_problem(inputs.uniform_points(16, 0.5, 1), inputs.uniform_density(2),
                            "plain_fp64", gpu)
    Kd.requires_grad_(True)
    F = spk.SparklingEnergy.apply(Kd, rd, prm, 8)
    (g,) = torch.autograd.grad(F, Kd, create_graph=False)
    with pytest.raises(RuntimeError):
        F2 = spk.SparklingEnergy.apply(Kd, rd, prm, 8)
        torch.autograd.grad(F2, Kd, create_graph=True)


def test_c4_autograd_fp32(gpu):
    """p = 65,536 in FP32, chunks of 8192: forward vs oracle energy, backward vs the
    oracle gradient, and 200 central finite differences of the FP64 oracle along
    dense Rademacher directions (h = 1e-4), error_k = |FD_k - <g, e_k>| / ||grad F||."""
    w = configs.C4
    K, rho = w.trajectory(), w.density()
    prm = spk.Params(w.n_shots, w.n_samples, w.grid, precision="fp32_comp")
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    K64, r64 = host64(Kd), host64(rd)
    Kd.requires_grad_(True)
    say(f"  c4 forward/backward p={prm.p}")
    F = spk.sparkling_energy(Kd, rd, prm, chunk=8192)
    F.backward()
    g = host64(Kd.grad)
    # the chunked backward is the full gradient kernel, bit for bit
    assert torch.equal(Kd.grad, spk.grad(Kd.detach(), rd, prm))

    say("  c4 oracle energy and gradient")
    oF = oracle.energy(K64, r64, w.grid, 0.5)[0]
    assert float(F.detach()) == pytest.approx(oF, rel=1e-6)
    og = oracle.grad(K64, r64, w.grid, 0.5)["dF"]
    err = rel_l2(g, og)
    say(f"  c4 backward rel L2 vs oracle = {err:.3e}")
    assert err <= 1e-5

    # 200 dense Rademacher directions (h = 1e-4 per coordinate): the FP64
    # oracle's central differences, stored by tests/golden/make_c4_fd.py
    meta, fd = c4_fd_golden()
    assert meta["K_digest"] == inputs.digest(K64) and meta["rho_digest"] == inputs.digest(r64)
    scale = meta["grad_norm"]
    errs_gpu, errs_orc = [], []
    for k in range(meta["directions"]):
        e = inputs.rademacher(K.shape, meta["seed0"] + k)
        errs_gpu.append(abs(fd[k, 0] - float((g * e).sum())) / scale)
        errs_orc.append(abs(fd[k, 0] - float((og * e).sum())) / scale)
    errs_gpu, errs_orc = np.array(errs_gpu), np.array(errs_orc)
    say(f"  c4 FD ({meta['directions']} dense directions): max err GPU {errs_gpu.max():.3e}  "
        f"oracle floor {errs_orc.max():.3e}  median GPU {np.median(errs_gpu):.3e}")
    assert errs_orc.max() <= 1e-4          # FD of the FP64 oracle agrees with its gradient
    assert errs_gpu.max() <= errs_orc.max() + 2e-5
