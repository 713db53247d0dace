"""The far field of the repulsion (Chebyshev fast multipole method on a uniform
octree, exact near field) against the oracle and the exact all-pairs sweep."""
import numpy as np
import pytest
import torch

from gpu_util import (ENERGY_TOL, GRAD_TOL, configs, device_problem, host64, inputs, oracle,
                      params_for, rel_l2, row_rel_max, say, spk, with_te_rows)

# Order-6 far field at 8.4M samples against the FP64 oracle's exact sums:
# relative L2 over the sampled rows, and the worst single row (row_rel_max).
C3_FAR_L2 = 1e-5
C3_FAR_ROW = 1e-3

pytestmark = pytest.mark.gpu


def grad_pair(dev, K, rho, G, precision, depth, order, eps=0.0, kernel="distance"):
    Nc, Ns = 1, K.shape[1]
    exact = spk.Params(Nc, Ns, G, precision=precision, eps=eps, kernel=kernel)
    far = spk.Params(Nc, Ns, G, precision=precision, eps=eps, kernel=kernel,
                     far_field_depth=depth, far_field_order=order)
    Kd, rd = device_problem(K, rho, precision, dev)
    g0, (pa0, pr0), e0 = spk.grad(Kd, rd, exact, potentials=True, with_energy=True)
    g1, (pa1, pr1), e1 = spk.grad(Kd, rd, far, potentials=True, with_energy=True)
    torch.cuda.synchronize()
    return Kd, rd, far, (host64(g0), host64(pr0), e0), (host64(g1), host64(pr1), e1)


def test_small_ragged_against_oracle(gpu):
    K = inputs.radial_spokes(37, 113, 0.5, seed=41, jitter=0.05)
    rho = inputs.radial_density(9, 0.5, 0.0625, 2.0)
    for precision in ("plain_fp64", "fp32_comp"):
        for depth, order in ((2, 4), (3, 6)):
            say(f"  far field {precision} depth {depth} order {order}, p = {K.shape[1]}")
            Kd, rd, prm, ex, ff = grad_pair(gpu, K, rho, 9, precision, depth, order)
            ref = oracle.grad(host64(Kd), host64(rd), 9, 0.5)
            e_far = rel_l2(ff[0], ref["dF"])
            e_pot = rel_l2(ff[1], ref["ur"])
            say(f"    grad rel L2 {e_far:.3e}, repulsion potential {e_pot:.3e}")
            assert rel_l2(ex[0], ref["dF"]) <= GRAD_TOL[precision]
            assert e_far <= (3e-3 if order == 4 else 3e-5)
            assert e_pot <= (1e-4 if order == 4 else 1e-6)


def test_rerun_and_chunks_bitwise(gpu):
    w = configs.C4
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, "fp32_comp", far_field_depth=4, far_field_order=5)
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    full = spk.grad(Kd, rd, prm)
    assert torch.equal(full, spk.grad(Kd, rd, prm))
    parts = [spk.grad(Kd, rd, prm, tgt=(b, min(b + 5000, prm.p))) for b in range(0, prm.p, 5000)]
    assert torch.equal(torch.cat(parts, dim=1), full)


def test_side_stream_or_none_same_bits(gpu):
    """The near-field sums on the caller's second stream (beside the M2L) or on
    the call's own stream give the same bits, uniform and adaptive trees."""
    K = inputs.radial_spokes(64, 500, 0.5, seed=44, jitter=0.05)
    rho = inputs.radial_density(8, 0.5, 0.0625, 2.0)
    for R in (0, 2):
        got = []
        for overlap in (True, False):
            prm = spk.Params(64, 500, 8, precision="fp32_comp", far_field_depth=3,
                             far_field_order=5, far_field_adaptive=R, far_field_overlap=overlap)
            Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
            g, (pa, pr), en = spk.grad(Kd, rd, prm, potentials=True, with_energy=True)
            torch.cuda.synchronize()
            got.append((g, pr, en))
        assert torch.equal(got[0][0], got[1][0]) and torch.equal(got[0][1], got[1][1])
        assert got[0][2] == got[1][2]


def test_coincident_and_outside_the_box(gpu):
    # every sample at one point: all pairs are near, the far field is empty
    K = np.full((3, 700), 0.125)
    Kd, rd, prm, ex, ff = grad_pair(gpu, K, inputs.uniform_density(4), 4, "plain_fp64", 3, 5)
    assert np.array_equal(ff[0], ex[0])
    # samples outside [-L, L]^3: the octree spans the samples' own bounding cube
    K = inputs.uniform_points(3000, 0.5, seed=5) * np.array([[3.0], [0.7], [1.5]])
    Kd, rd, prm, ex, ff = grad_pair(gpu, K, inputs.uniform_density(4), 4, "plain_fp64", 4, 6)
    say(f"  outside the box: grad rel L2 vs exact {rel_l2(ff[0], ex[0]):.3e}")
    assert rel_l2(ff[0], ex[0]) <= 3e-5


def test_c2_against_exact_sweep(gpu):
    """524,288 samples on 128^3: the far field against the exact all-pairs sweep."""
    w = configs.C2
    K, rho = w.trajectory(), w.density()
    for precision, depth, order, tol in (("fp32_comp", 5, 5, 3e-4), ("fp32_comp", 5, 6, 5e-5),
                                         ("plain_fp64", 5, 6, 5e-5)):
        Kd, rd, prm, ex, ff = grad_pair(gpu, K, rho, w.grid, precision, depth, order)
        eg, ep = rel_l2(ff[0], ex[0]), rel_l2(ff[1], ex[1])
        eF = abs(ff[2][0] - ex[2][0]) / abs(ex[2][0])
        say(f"  c2 {precision} depth {depth} order {order}: grad F rel L2 {eg:.3e}, "
            f"repulsion potential {ep:.3e}, F {eF:.3e}")
        assert eg <= tol and ep <= tol / 10 and eF <= tol / 10


def test_log_kernel_far_field(gpu):
    K = inputs.radial_spokes(64, 128, 0.5, seed=42, jitter=0.05)
    rho = inputs.radial_density(16, 0.5, 0.0625, 2.0)
    eps = 0.01
    Kd, rd, prm, ex, ff = grad_pair(gpu, K, rho, 16, "plain_fp64", 4, 6, eps=eps, kernel="log")
    say(f"  log kernel: grad rel L2 vs exact {rel_l2(ff[0], ex[0]):.3e}")
    assert rel_l2(ff[0], ex[0]) <= 1e-4


def test_c3_far_field_sampled_against_oracle(gpu):
    """8.4M samples, depth 5, order 6: rows against the oracle, and the time of both methods."""
    w = configs.C3
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, "fp32_comp", far_field_depth=5, far_field_order=6)
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    spk.grad(Kd, rd, prm)                       # warm-up
    torch.cuda.synchronize()
    spk.timing_reset()
    spk.timing_enable(True)
    g = spk.grad(Kd, rd, prm)
    torch.cuda.synchronize()
    spk.timing_enable(False)
    rep_ms = spk.timing_query(spk.KIND_REPULSION)[0]
    att_ms = spk.timing_query(spk.KIND_ATTRACTION)[0]
    t = with_te_rows(inputs.sample_targets(prm.p, 256, seed=43), w.n_shots, w.n_samples)
    say(f"  c3 far-field repulsion {rep_ms:.1f} ms, attraction {att_ms:.1f} ms; oracle on "
        f"{t.size} targets")
    ref = oracle.grad(host64(Kd), host64(rd), w.grid, 0.5, 0.0, t)
    err = rel_l2(host64(g)[:, t], ref["dF"])
    row = row_rel_max(host64(g)[:, t], ref["dF"])
    say(f"  c3 far field: grad rel L2 vs oracle {err:.3e}, worst row {row:.3e}")
    assert err <= C3_FAR_L2
    assert row <= C3_FAR_ROW


def test_step_with_far_field_tracks_the_exact_step(gpu):
    """One projected step at 2048 x 1024 samples with the far field against the exact step."""
    w = configs.C5
    K, rho = w.trajectory(), w.density()
    out = []
    for depth in (0, 5):
        prm = params_for(w, "fp32_comp", far_field_depth=depth, far_field_order=6)
        Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
        spk.project_(Kd, prm)
        info = spk.step_(Kd, rd, prm, spk.StepState(prm, gpu), 0, w.eta_fixed)
        out.append((host64(Kd), info))
    d = np.abs(out[0][0] - out[1][0]).max()
    say(f"  c5 step, far field vs exact: max |dK| {d:.3e}, F {out[1][1]['F']:.12e} vs "
        f"{out[0][1]['F']:.12e}")
    assert d <= 1e-5
    assert out[1][1]["F"] == pytest.approx(out[0][1]["F"], rel=1e-7)


@pytest.mark.parametrize("depth,order", [(2, 4), (3, 5)])
def test_matches_the_reference_fmm(gpu, depth, order):
    """Plain FP64 GPU far field against the NumPy reference of the same method:
    equal up to summation order."""
    from oracle import fmm
    K = inputs.radial_spokes(20, 90, 0.5, seed=53, jitter=0.05)
    prm = spk.Params(20, 90, 1, precision="plain_fp64", far_field_depth=depth,
                     far_field_order=order)
    Kd, rd = device_problem(K, [0.0], "plain_fp64", gpu)       # no attraction
    g, (pa, pr) = spk.grad(Kd, rd, prm, potentials=True)
    gr, ur = fmm.fmm(K.T, depth, order, fmm.distance_kernel())
    p = K.shape[1]
    got = -host64(g) * p * p                                     # grad F = -sum grad H / p^2
    err = np.abs(got - gr.T).max() / np.abs(gr).max()
    say(f"  GPU vs reference FMM, depth {depth} order {order}: {err:.3e}")
    assert err <= 1e-13
    assert np.abs(host64(pr) - ur).max() <= 1e-13 * np.abs(ur).max()


# --------------------------------------------------------------------------
# Adaptive tree: dense leaves refined once more
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dense,sparse,depth,order,R", [(12000, 1000, 2, 3, 1),
                                                      (40000, 2000, 2, 4, 1),
                                                      (48000, 2000, 2, 3, 2)])
def test_adaptive_matches_the_reference_fmm(gpu, dense, sparse, depth, order, R):
    from oracle import fmm
    K = inputs.two_density_points(dense, sparse, 0.5, seed=57)
    p = K.shape[1]
    prm = spk.Params(1, p, 1, precision="plain_fp64", far_field_depth=depth,
                     far_field_order=order, far_field_adaptive=R)
    Kd, rd = device_problem(K, [0.0], "plain_fp64", gpu)
    g, (pa, pr) = spk.grad(Kd, rd, prm, potentials=True)
    info = {}
    gr, ur = fmm.fmm(K.T, depth, order, fmm.distance_kernel(), adaptive=R, info=info)
    final = info["final_level"]
    got = -host64(g) * p * p
    err = np.abs(got - gr.T).max() / np.abs(gr).max()
    counts = [int((final == depth + q).sum()) for q in range(R + 1)]
    say(f"  adaptive (R = {R}) GPU vs reference FMM, depth {depth} order {order}: {err:.3e} "
        f"(targets per final level {counts})")
    assert all(c > 0 for c in counts)
    assert err <= 1e-13
    assert np.abs(host64(pr) - ur).max() <= 1e-13 * np.abs(ur).max()


@pytest.mark.parametrize("R", [1, 2])
def test_adaptive_rerun_and_chunks_bitwise(gpu, R):
    K = inputs.two_density_points(60000, 5000, 0.5, seed=58)
    p = K.shape[1]
    prm = spk.Params(1, p, 1, precision="fp32_comp", far_field_depth=2, far_field_order=4,
                     far_field_adaptive=R)
    Kd, rd = device_problem(K, [0.0], "fp32_comp", gpu)
    full = spk.grad(Kd, rd, prm)
    assert torch.equal(full, spk.grad(Kd, rd, prm))
    parts = [spk.grad(Kd, rd, prm, tgt=(b, min(b + 7000, p))) for b in range(0, p, 7000)]
    assert torch.equal(torch.cat(parts, dim=1), full)


def test_adaptive_c2_against_exact_sweep(gpu):
    w = configs.C2
    K, rho = w.trajectory(), w.density()
    for precision, kernel, eps, tol, R in (("fp32_comp", "distance", 0.0, 5e-5, 1),
                                           ("plain_fp64", "log", 0.01, 1e-4, 1),
                                           ("fp32_comp", "distance", 0.0, 5e-5, 2)):
        Nc, Ns = w.n_shots, w.n_samples
        exact = spk.Params(Nc, Ns, w.grid, precision=precision, eps=eps, kernel=kernel)
        far = spk.Params(Nc, Ns, w.grid, precision=precision, eps=eps, kernel=kernel,
                         far_field_depth=4, far_field_order=6, far_field_adaptive=R)
        Kd, rd = device_problem(K, rho, precision, gpu)
        g0, (pa0, pr0), e0 = spk.grad(Kd, rd, exact, potentials=True, with_energy=True)
        g1, (pa1, pr1), e1 = spk.grad(Kd, rd, far, potentials=True, with_energy=True)
        eg, ep = rel_l2(host64(g1), host64(g0)), rel_l2(host64(pr1), host64(pr0))
        say(f"  c2 adaptive (R = {R}) {precision} {kernel}: grad F rel L2 {eg:.3e}, "
            f"potential {ep:.3e}")
        assert eg <= tol and ep <= tol / 10


@pytest.mark.parametrize("R", [1, 2])
def test_adaptive_c3_sampled_against_oracle(gpu, R):
    """8.4M samples, depth 5 refined once or twice where dense, order 6: rows
    against the oracle."""
    w = configs.C3
    K, rho = w.trajectory(), w.density()
    prm = params_for(w, "fp32_comp", far_field_depth=5, far_field_order=6,
                     far_field_adaptive=R)
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    spk.grad(Kd, rd, prm)                       # warm-up
    torch.cuda.synchronize()
    spk.timing_reset()
    spk.timing_enable(True)
    g = spk.grad(Kd, rd, prm)
    torch.cuda.synchronize()
    spk.timing_enable(False)
    rep_ms = spk.timing_query(spk.KIND_REPULSION)[0]
    t = with_te_rows(inputs.sample_targets(prm.p, 256, seed=43), w.n_shots, w.n_samples)
    ref = oracle.grad(host64(Kd), host64(rd), w.grid, 0.5, 0.0, t)
    err = rel_l2(host64(g)[:, t], ref["dF"])
    row = row_rel_max(host64(g)[:, t], ref["dF"])
    say(f"  c3 adaptive (R = {R}) far field: repulsion {rep_ms:.1f} ms, grad rel L2 vs "
        f"oracle {err:.3e}, worst row {row:.3e}")
    assert err <= C3_FAR_L2
    assert row <= C3_FAR_ROW


def test_adaptive_edge_cases(gpu):
    """Adaptive trees on degenerate inputs: coincident samples (nothing is
    refined, all pairs are near: the exact sum), samples outside [-L, L]^3,
    and tiny p."""
    def pair(K, depth, order, R, precision="plain_fp64"):
        Nc, Ns = 1, K.shape[1]
        exact = spk.Params(Nc, Ns, 4, precision=precision)
        far = spk.Params(Nc, Ns, 4, precision=precision, far_field_depth=depth,
                         far_field_order=order, far_field_adaptive=R)
        Kd, rd = device_problem(K, inputs.uniform_density(4), precision, gpu)
        g0 = host64(spk.grad(Kd, rd, exact))
        g1 = host64(spk.grad(Kd, rd, far))
        return g0, g1

    for R in (1, 2):
        g0, g1 = pair(np.full((3, 700), 0.125), 3, 5, R)
        assert np.array_equal(g0, g1), R
        K = inputs.uniform_points(3000, 0.5, seed=5) * np.array([[3.0], [0.7], [1.5]])
        g0, g1 = pair(K, 3, 6, R)
        say(f"  adaptive R = {R}, outside the box: grad rel L2 vs exact {rel_l2(g1, g0):.3e}")
        assert rel_l2(g1, g0) <= 3e-5
        # one sample: no pair at all; a few: far pairs are interpolated (order 4)
        g0, g1 = pair(inputs.uniform_points(1, 0.5, seed=1), 2, 4, R)
        assert np.array_equal(g0, g1), R
        for p in (2, 5):
            g0, g1 = pair(inputs.uniform_points(p, 0.5, seed=p), 2, 4, R)
            assert rel_l2(g1, g0) <= 1e-3, (R, p)


def test_adaptive_two_levels_fp64_against_the_oracle(gpu):
    """Plain FP64 with two refinement levels on a dense two-density input,
    against the FP64 oracle's exact sums."""
    K = inputs.two_density_points(48000, 2000, 0.5, seed=59)
    p = K.shape[1]
    prm = spk.Params(1, p, 1, precision="plain_fp64", far_field_depth=3, far_field_order=6,
                     far_field_adaptive=2)
    Kd, rd = device_problem(K, [1.0], "plain_fp64", gpu)
    g = host64(spk.grad(Kd, rd, prm))
    t = inputs.sample_targets(p, 400, seed=60)
    ref = oracle.grad(host64(Kd), host64(rd), 1, 0.5, 0.0, t)
    err = rel_l2(g[:, t], ref["dF"])
    say(f"  adaptive R = 2, FP64, 50k samples: grad rel L2 vs oracle {err:.3e}")
    assert err <= 3e-5
