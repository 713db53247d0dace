"""Grid attraction on the GPU against the oracle: node field, interpolated
gradient and energy, chunk invariance, and its distance from the direct sum."""
import time

import numpy as np
import pytest
import torch

from gpu_util import (GRAD_TOL, configs, device_problem, host64, inputs, oracle, params_for,
                      rel_l2, say, spk)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("direct", [False, True])
@pytest.mark.parametrize("precision,tol", [("plain_fp64", 1e-12), ("fp32_comp", 1e-6)])
def test_node_field_matches_oracle(gpu, precision, tol, direct):
    """Both ways of taking the node field: FP64 FFT convolution, and the direct
    sum over the cells in the precision form."""
    G, L = 7, 0.5
    rho = inputs.radial_density(G, L, 0.1, 2.0)
    prm = spk.Params(1, 8, G, precision=precision, field_direct=direct)
    _, rd = device_problem(np.zeros((3, 8)), rho, precision, gpu)
    f = host64(spk.attraction_field(rd, prm))
    want = oracle.field(host64(rd), G, L)
    assert f.shape == want.shape
    assert rel_l2(f[:, 0], want[:, 0]) <= tol
    assert rel_l2(f[:, 1:], want[:, 1:]) <= tol


@pytest.mark.parametrize("precision", ["plain_fp64", "fp32_comp"])
def test_interpolated_gradient_matches_oracle(gpu, precision):
    G, L = 9, 0.5
    K = inputs.radial_spokes(21, 47, L, seed=31, jitter=0.05)
    rho = inputs.radial_density(G, L, 0.08, 2.0)
    prm = spk.Params(21, 47, G, precision=precision)
    Kd, rd = device_problem(K, rho, precision, gpu)
    prm.attraction_field = spk.attraction_field(rd, prm)
    g, (pa, pr), en = spk.grad(Kd, rd, prm, potentials=True, with_energy=True)
    ref = oracle.grad_field(host64(Kd), host64(rd), G, L)
    tol = GRAD_TOL[precision] * (10 if precision == "fp32_comp" else 1)
    assert rel_l2(host64(g), ref["dF"]) <= tol
    assert rel_l2(host64(pa), ref["ua"]) <= tol
    Fa = ref["ua"].sum() / prm.p
    assert en[1] == pytest.approx(Fa, rel=tol)
    # chunked calls give the same rows
    parts = [spk.grad(Kd, rd, prm, tgt=(b, min(b + 300, prm.p))) for b in range(0, prm.p, 300)]
    assert torch.equal(torch.cat(parts, dim=1), g)


def test_c2_grid_attraction_vs_direct(gpu):
    """At 524k samples on 128^3: interpolated attraction against the oracle's
    interpolant on sampled targets, and its distance from the direct sum."""
    w = configs.C2
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, "fp32_comp")
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    say("  c2 field precompute")
    fld = spk.attraction_field(rd, prm)
    g_direct = spk.grad(Kd, rd, prm)
    prm.attraction_field = fld
    g_field = spk.grad(Kd, rd, prm)
    torch.cuda.synchronize()
    t = inputs.sample_targets(prm.p, 256, seed=5)
    say("  c2 oracle grid attraction on 256 targets")
    ref = oracle.grad_field(host64(Kd), host64(rd), w.grid, 0.5, 0.0, t)
    err = rel_l2(host64(g_field)[:, t], ref["dF"])
    dist = rel_l2(host64(g_field), host64(g_direct))
    say(f"  c2 grid attraction: rel L2 vs oracle {err:.3e}, vs direct sum {dist:.3e}")
    assert err <= 1e-5
    assert dist <= 5e-2


@pytest.mark.parametrize("G,kernel,eps", [(24, "distance", 0.0), (31, "log", 0.02), (40, "distance", 0.01)])
def test_fft_field_against_direct_fp64(gpu, G, kernel, eps):
    """FP64: the FFT convolution and the direct sum agree to rounding (odd, even
    and non-power-of-two grids; both kernels; a regularised distance)."""
    rho = inputs.separable_density(G, seed=G)
    out = []
    for direct in (False, True):
        prm = spk.Params(1, 8, G, precision="plain_fp64", kernel=kernel, eps=eps,
                         field_direct=direct)
        _, rd = device_problem(np.zeros((3, 8)), rho, "plain_fp64", gpu)
        out.append(host64(spk.attraction_field(rd, prm)))
    err = rel_l2(out[0], out[1])
    say(f"  G = {G} {kernel}: FFT vs direct node field, rel L2 {err:.3e}")
    assert err <= 1e-12


def test_fft_field_c2_against_direct(gpu):
    """128^3 cells (FFT of 512^3): the FP64 FFT field against the FP32-compensated
    direct sum, and the time of both."""
    w = configs.C2
    rho = w.density()
    res = []
    for direct in (False, True):
        prm = params_for(w, "fp32_comp", field_direct=direct)
        _, rd = device_problem(np.zeros((3, prm.p)), rho, "fp32_comp", gpu)
        spk.attraction_field(rd, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = spk.attraction_field(rd, prm)
        torch.cuda.synchronize()
        res.append((host64(f), time.perf_counter() - t0))
    err = rel_l2(res[0][0], res[1][0])
    say(f"  c2 node field: FFT {res[0][1] * 1e3:.1f} ms, direct {res[1][1] * 1e3:.1f} ms, "
        f"rel L2 {err:.3e}")
    assert err <= 1e-6


def test_fft_field_c3_sampled_nodes(gpu):
    """192^3 cells: the FFT node field on sampled nodes against the oracle's
    attraction potential and gradient at those nodes."""
    w = configs.C3
    rho = w.density()
    G, L = w.grid, w.half_width
    prm = params_for(w, "fp32_comp")
    _, rd = device_problem(np.zeros((3, 8)), rho, "fp32_comp", gpu)
    spk.attraction_field(rd, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = host64(spk.attraction_field(rd, prm))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    Gn = G + 2
    nodes = inputs.sample_targets(Gn ** 3, 48, seed=9)
    k = np.stack([nodes % Gn, (nodes // Gn) % Gn, nodes // (Gn * Gn)])
    X = -L + (k - 0.5) * (2 * L / G)
    ref = oracle.grad(X, host64(rd), G, L)
    n = X.shape[1]
    err_u = rel_l2(f[nodes, 0], ref["ua"])
    err_g = rel_l2(f[nodes, 1:].T, ref["dFa"] * n)
    say(f"  c3 FFT node field {ms:.1f} ms; sampled nodes rel L2 U {err_u:.3e}, grad {err_g:.3e}")
    assert err_u <= 1e-6 and err_g <= 1e-6


def test_fft_field_largest_transform_sampled_nodes(gpu):
    """300^3 cells take transforms of 1024^3 (4 lines per block): sampled nodes
    against the oracle's attraction potential and gradient."""
    G, L = 300, 0.5
    rho = inputs.separable_density(G, seed=3)
    prm = spk.Params(1, 8, G, precision="plain_fp64")
    _, rd = device_problem(np.zeros((3, 8)), rho, "plain_fp64", gpu)
    t0 = time.perf_counter()
    f = spk.attraction_field(rd, prm)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    Gn = G + 2
    nodes = inputs.sample_targets(Gn ** 3, 24, seed=10)
    fs = host64(f[torch.as_tensor(nodes, device=f.device)])
    del f
    k = np.stack([nodes % Gn, (nodes // Gn) % Gn, nodes // (Gn * Gn)])
    X = -L + (k - 0.5) * (2 * L / G)
    ref = oracle.grad(X, rho, G, L)
    err_u = rel_l2(fs[:, 0], ref["ua"])
    err_g = rel_l2(fs[:, 1:].T, ref["dFa"] * X.shape[1])
    say(f"  G = 300 FFT node field {ms:.0f} ms; sampled nodes rel L2 U {err_u:.3e}, grad {err_g:.3e}")
    assert err_u <= 1e-12 and err_g <= 1e-12
