"""F^r from the repulsion forces (SPK_FLAG_ENERGY_FROM_FORCE): with H = |d|,
F^r = sum_i K[i] . dF^r/dK[i] (Euler's theorem for the degree-1 homogeneous
repulsion term), so the sweep skips its per-pair distances.  Checked against
the oracle's pair sums and against the per-pair energy of the same kernels."""
import numpy as np
import pytest
import torch

from gpu_util import (ENERGY_TOL, bounds, configs, device_problem, host64, inputs, oracle,
                      params_for, say, spk)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["plain_fp64", "fp32_comp", "fp32_acc64"])
def test_energies_against_the_oracle(gpu, precision):
    K = inputs.radial_spokes(37, 113, 0.5, seed=71, jitter=0.05)
    rho = inputs.radial_density(13, 0.5, 0.0625, 2.0)
    prm = spk.Params(37, 113, 13, precision=precision, energy_from_force=True)
    Kd, rd = device_problem(K, rho, precision, gpu)
    F, Fa, Fr, _ = spk.energy(Kd, rd, prm)
    oF, oFa, oFr = oracle.energy(host64(Kd), host64(rd), 13, 0.5)
    say(f"  energy from force {precision}: F^r {Fr:.15e} vs {oFr:.15e}")
    tol = ENERGY_TOL[precision]
    assert Fr == pytest.approx(oFr, rel=tol) and F == pytest.approx(oF, rel=tol)
    assert Fa == pytest.approx(oFa, rel=tol)


@pytest.mark.parametrize("precision", ["plain_fp64", "fp32_comp"])
def test_gradient_unchanged_and_energy_close(gpu, precision):
    """The same gradient bits as with the per-pair energy; F within rounding."""
    w = configs.C4
    K, rho = w.trajectory(), w.density()
    Kd, rd = device_problem(K, rho, precision, gpu)
    out = []
    for flag in (False, True):
        prm = params_for(w, precision, energy_from_force=flag)
        g, en = spk.grad(Kd, rd, prm, with_energy=True)
        torch.cuda.synchronize()
        out.append((g, en))
    assert torch.equal(out[0][0], out[1][0])
    say(f"  c4 {precision}: F^r per pair {out[0][1][2]:.15e}, from force {out[1][1][2]:.15e}")
    assert out[1][1][2] == pytest.approx(out[0][1][2], rel=1e-13 if precision == "plain_fp64"
                                         else 1e-7)


def test_steps_unchanged(gpu):
    """Projected steps with the energy from the forces: K and the step state
    bit for bit as with the per-pair energy, into the Barzilai-Borwein phase."""
    w = configs.C1
    K, rho = w.trajectory(), w.density()
    res = []
    for flag in (False, True):
        prm = params_for(w, "plain_fp64", energy_from_force=flag)
        Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
        state = spk.StepState(prm, gpu)
        infos = [spk.step_(Kd, rd, prm, state, it, 16.0) for it in range(18, 22)]
        res.append((Kd, state, infos))
    assert torch.equal(res[0][0], res[1][0])
    assert torch.equal(res[0][1].g_prev, res[1][1].g_prev)
    for a, b in zip(res[0][2], res[1][2]):
        assert a["eta"] == b["eta"] and a["bb_used"] == b["bb_used"]
        assert a["F"] == pytest.approx(b["F"], rel=1e-13)


def test_c2_energy_from_force(gpu):
    w = configs.C2
    K, rho = w.trajectory(), w.density()
    Kd, rd = device_problem(K, rho, "fp32_comp", gpu)
    e = []
    for flag in (False, True):
        prm = params_for(w, "fp32_comp", energy_from_force=flag)
        spk.timing_reset()
        spk.timing_enable(True)
        F, Fa, Fr, _ = spk.energy(Kd, rd, prm)
        torch.cuda.synchronize()
        spk.timing_enable(False)
        e.append((Fr, spk.timing_query(spk.KIND_REPULSION)[0]))
    say(f"  c2: F^r per pair {e[0][0]:.12e} ({e[0][1]:.1f} ms), from force {e[1][0]:.12e} "
        f"({e[1][1]:.1f} ms)")
    assert e[1][0] == pytest.approx(e[0][0], rel=1e-7)


def test_discrepancy_with_energy_from_force(gpu):
    """D = F - (1/2) sum rho rho H with F^r from the forces, against the oracle."""
    K = inputs.radial_spokes(12, 40, 0.5, seed=73, jitter=0.05)
    rho = inputs.radial_density(8, 0.5, 0.0625, 2.0)
    prm = spk.Params(12, 40, 8, precision="plain_fp64", energy_from_force=True,
                     discrepancy=True)
    Kd, rd = device_problem(K, rho, "plain_fp64", gpu)
    F, Fa, Fr, D = spk.energy(Kd, rd, prm)
    oF = oracle.energy(K, rho, 8, 0.5)[0]
    oD = oF - oracle.rho_self_energy(rho, 8, 0.5)
    assert F == pytest.approx(oF, rel=1e-12) and D == pytest.approx(oD, rel=1e-9, abs=1e-15)
