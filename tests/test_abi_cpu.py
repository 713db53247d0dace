"""The C ABI without a GPU: exported symbols, host helpers and argument validation.

Validation runs before any HIP call, so every rejected call below returns its
status without touching a device.  No compute entry point is run here.
"""
import ctypes
import json
import os
import re

import pytest

import oracle
import paper_2108_02991_amd as spk
from paper_2108_02991_amd import api, configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sparkling.h")
EINVAL, EWORKSPACE, EUNSUPPORTED = -1, -2, -4


@pytest.fixture(scope="module")
def lib():
    if not api.LIB_PATH.exists():
        from paper_2108_02991_amd import build
        build.build()
    return spk.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"sparkling_energy", "sparkling_grad", "sparkling_project", "sparkling_step",
            "spk_workspace_size", "spk_alpha_beta"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n


def test_only_the_c_abi_is_exported(lib):
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm is not available")
    out = subprocess.run([nm, "-D", "--defined-only", str(api.LIB_PATH)], capture_output=True,
                         text=True, check=True).stdout
    text = {ln.split()[-1] for ln in out.splitlines() if len(ln.split()) == 3
            and ln.split()[1] == "T"}
    assert text == set(declared_functions())


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.spk_status_string(code)
    assert lib.spk_status_string(99) == b"unknown status"


def test_alpha_beta_matches_oracle_and_golden(lib):
    with open(os.path.join(ROOT, "tests", "golden", "alpha_beta.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        a, b = spk.alpha_beta(*case["args"])
        oa, ob = oracle.alpha_beta(*case["args"])
        assert a == pytest.approx(case["a"], rel=1e-5) and b == pytest.approx(case["b"], rel=1e-5)
        assert a == pytest.approx(oa, rel=1e-15) and b == pytest.approx(ob, rel=1e-15)
    with pytest.raises(spk.SparklingError):
        spk.alpha_beta(0.04, 180, 1e-5, 2e-6, 0.0, 66.0, 42.576e6, 0.5)


def good_params(**kw):
    base = dict(n_shots=4, n_samples=16, grid=8, precision="fp32_comp", a_max=0.1, b_max=0.01)
    base.update(kw)
    return spk.Params(**base)


def test_workspace_size_monotone(lib):
    small = spk.workspace_size(good_params())
    big = spk.workspace_size(good_params(n_shots=64))
    disc = spk.workspace_size(good_params(discrepancy=True, grid=32))
    assert 0 < small < big and disc > small
    assert spk.workspace_size(spk.Params(4096, 2048, 192)) < 2 * 2 ** 30


def test_workspace_does_not_scale_with_grid_times_slabs(lib):
    """Few samples on the largest grid: partials are sized per sweep kind and the
    grid-target sweeps run in passes, so the workspace stays small."""
    for prec in ("fp32_comp", "plain_fp64"):
        for disc in (False, True):
            n = spk.workspace_size(good_params(n_shots=3, n_samples=100, grid=1024,
                                               precision=prec, discrepancy=disc))
            assert n < 2 ** 30, (prec, disc, n)
    # the samples' accumulators dominate at large p: about 100 bytes per sample
    big = spk.workspace_size(spk.Params(524289, 2048, 4))
    assert 90 * 524289 * 2048 < big < 120 * 524289 * 2048


@pytest.mark.parametrize("bad", [
    dict(n_shots=0), dict(n_samples=0), dict(grid=0), dict(grid=2000), dict(te_index=16),
    dict(te_index=-2), dict(half_width=0.0), dict(half_width=float("nan")), dict(eps=-1.0),
    dict(n_shots=2 ** 20, n_samples=2 ** 12),
])
def test_bad_params_rejected(lib, bad):
    prm = good_params(**bad)
    n = ctypes.c_size_t()
    c = prm.c()
    assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == EINVAL
    assert lib.spk_last_error()


def test_unknown_precision_and_flags(lib):
    c = good_params().c()
    c.precision = 7
    n = ctypes.c_size_t()
    assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == EINVAL
    c = good_params().c()
    c.flags = 32
    assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == EINVAL
    assert lib.spk_workspace_size(None, ctypes.byref(n)) == EINVAL


def test_energy_from_force_validation(lib):
    """The energy from the forces needs H = |d|: eps = 0, the distance kernel,
    the exact repulsion; and no per-target repulsion potentials."""
    n = ctypes.c_size_t()
    ok = good_params(energy_from_force=True)
    assert lib.spk_workspace_size(ctypes.byref(ok.c()), ctypes.byref(n)) == 0
    for kw in (dict(eps=0.01), dict(kernel="log", eps=0.01),
               dict(far_field_depth=3, far_field_order=4)):
        c = good_params(energy_from_force=True, **kw).c()
        assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == EINVAL, kw
    v = ctypes.c_void_p
    c = ok.c()
    args = [v(FAKE)] * 7
    assert lib.sparkling_grad(ctypes.byref(c), *args, 0, ok.p, None, v(FAKE), None, v(FAKE),
                              spk.workspace_size(ok), None) == EINVAL
    assert "potentials" in lib.spk_last_error().decode()


def test_far_field_validation_and_workspace(lib):
    n = ctypes.c_size_t()
    base = spk.workspace_size(good_params())
    sizes = []
    for depth, order in ((2, 3), (3, 4), (4, 6)):
        c = good_params(far_field_depth=depth, far_field_order=order).c()
        assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == 0
        sizes.append(n.value)
    assert base < sizes[0] < sizes[1] < sizes[2]
    for bad, code in [(dict(far_field_depth=1), EINVAL), (dict(far_field_depth=8), EINVAL),
                      (dict(far_field_depth=3, far_field_order=2), EINVAL),
                      (dict(far_field_depth=3, far_field_order=7), EINVAL),
                      (dict(far_field_depth=3, precision="fp32_naive"), EUNSUPPORTED),
                      (dict(far_field_depth=3, precision="fp32_acc64"), EUNSUPPORTED)]:
        c = good_params(**bad).c()
        assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == code, bad


def test_adaptive_far_field_validation(lib):
    n = ctypes.c_size_t()
    sizes = []
    for R in (0, 1, 2):
        c = good_params(far_field_depth=4, far_field_order=5, far_field_adaptive=R).c()
        assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == 0
        sizes.append(n.value)
    assert sizes[0] < sizes[1] < sizes[2]
    c = good_params(far_field_depth=5, far_field_adaptive=2).c()
    assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == 0
    for bad in [dict(far_field_depth=7, far_field_adaptive=1),
                dict(far_field_depth=6, far_field_adaptive=2),
                dict(far_field_depth=0, far_field_adaptive=1)]:
        c = good_params(**bad).c()
        assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == EINVAL, bad
    for R in (3, -1):
        c = good_params(far_field_depth=3).c()
        c.far_field_adaptive = R
        assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == EINVAL, R


def test_field_workspace_size(lib):
    n = ctypes.c_size_t()
    # G = 7: FFT length M = 16 (>= 2G + 1): two M^3 complex doubles and M/2 twiddles,
    # each rounded up to 256 bytes, plus 256 bytes of alignment slack
    c = good_params(grid=7).c()
    assert lib.spk_field_workspace_size(ctypes.byref(c), ctypes.byref(n)) == 0
    assert n.value == 2 * 16 ** 3 * 16 + 256 + 256
    # G = 300 needs M = 1024
    c = good_params(grid=300).c()
    assert lib.spk_field_workspace_size(ctypes.byref(c), ctypes.byref(n)) == 0
    assert n.value == 2 * 1024 ** 3 * 16 + 8192 + 256
    # the direct sum, and grids beyond the largest transform, use the ordinary workspace
    for prm in (good_params(grid=7, field_direct=True), good_params(grid=600)):
        c = prm.c()
        assert lib.spk_field_workspace_size(ctypes.byref(c), ctypes.byref(n)) == 0
        assert n.value == spk.workspace_size(prm)


def test_log_kernel_validation(lib):
    n = ctypes.c_size_t()
    ok = good_params(kernel="log", eps=0.01).c()
    assert ok.flags == api.FLAG_LOG_KERNEL
    assert lib.spk_workspace_size(ctypes.byref(ok), ctypes.byref(n)) == 0
    for bad, code in [(dict(eps=0.0), EINVAL), (dict(eps=1e-30), EINVAL),
                      (dict(eps=0.01, precision="fp32_naive"), EUNSUPPORTED),
                      (dict(eps=0.01, precision="fp32_acc64"), EUNSUPPORTED)]:
        c = good_params(kernel="log", **bad).c()
        assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == code, bad
    # FP64 accepts an eps whose square is below the float range
    c = good_params(kernel="log", eps=1e-30, precision="plain_fp64").c()
    assert lib.spk_workspace_size(ctypes.byref(c), ctypes.byref(n)) == 0


FAKE = 0x10000   # an aligned, never dereferenced address


def grad_call(lib, prm, ptrs=None, b=0, e=None, ws=FAKE, ws_bytes=None, energy=None):
    c = prm.c()
    ptrs = ptrs or [FAKE] * 7
    e = prm.p if e is None else e
    ws_bytes = spk.workspace_size(prm) if ws_bytes is None else ws_bytes
    return lib.sparkling_grad(ctypes.byref(c), *[ctypes.c_void_p(x) for x in ptrs[:4]],
                              *[ctypes.c_void_p(x) for x in ptrs[4:7]], b, e, None, None, energy,
                              ctypes.c_void_p(ws), ws_bytes, None)


def test_grad_validation(lib):
    prm = good_params()
    ptrs = [FAKE] * 7
    for k in range(7):
        bad = list(ptrs)
        bad[k] = 0
        assert grad_call(lib, prm, bad) == EINVAL
    bad = list(ptrs)
    bad[2] = FAKE + 2        # misaligned float array
    assert grad_call(lib, prm, bad) == EINVAL
    assert grad_call(lib, prm, b=-1) == EINVAL
    assert grad_call(lib, prm, b=10, e=5) == EINVAL
    assert grad_call(lib, prm, e=prm.p + 1) == EINVAL
    assert grad_call(lib, prm, b=3, e=9, energy=(ctypes.c_double * 3)()) == EINVAL
    assert grad_call(lib, prm, ws_bytes=16) == EWORKSPACE
    assert grad_call(lib, prm, ws=0) == EWORKSPACE
    # an empty target range is valid, launches nothing and takes NULL outputs
    assert grad_call(lib, prm, b=5, e=5) == 0
    assert grad_call(lib, prm, [FAKE] * 4 + [0, 0, 0], b=5, e=5) == 0


def test_plain_fp64_needs_8_byte_alignment(lib):
    prm = good_params(precision="plain_fp64")
    bad = [FAKE] * 7
    bad[0] = FAKE + 4
    assert grad_call(lib, prm, bad) == EINVAL


def test_energy_project_step_validation(lib):
    prm = good_params()
    c = prm.c()
    out = (ctypes.c_double * 4)()
    n = spk.workspace_size(prm)
    v = ctypes.c_void_p
    assert lib.sparkling_energy(ctypes.byref(c), v(FAKE), v(FAKE), v(FAKE), v(FAKE), None,
                                v(FAKE), n, None) == EINVAL
    assert lib.sparkling_energy(ctypes.byref(c), v(FAKE), v(0), v(FAKE), v(FAKE), out,
                                v(FAKE), n, None) == EINVAL
    assert lib.sparkling_energy(ctypes.byref(c), v(FAKE), v(FAKE), v(FAKE), v(FAKE), out,
                                v(FAKE), 8, None) == EWORKSPACE
    # projection needs positive bounds, 2 <= Ns <= 4096
    for kw, want in [(dict(a_max=0.0), EINVAL), (dict(b_max=-1.0), EINVAL),
                     (dict(n_samples=1, te_index=0), EINVAL), (dict(n_pit=-1), EINVAL),
                     (dict(n_shots=1, n_samples=5000), EUNSUPPORTED)]:
        cp = good_params(**kw).c()
        assert lib.sparkling_project(ctypes.byref(cp), v(FAKE), v(FAKE), v(FAKE), None, v(FAKE),
                                     1 << 40, None) == want, kw
        assert lib.sparkling_constraint_check(ctypes.byref(cp), v(FAKE), v(FAKE), v(FAKE), out,
                                              v(FAKE), 1 << 40, None) == want, kw
    info = api.SpkStepInfo()
    info.iter = 0
    info.eta_fixed = 0.0
    assert lib.sparkling_step(ctypes.byref(c), v(FAKE), v(FAKE), v(FAKE), v(FAKE), v(FAKE),
                              v(FAKE), ctypes.byref(info), v(FAKE), n, None) == EINVAL
    info.eta_fixed = 1.0
    info.iter = -3
    assert lib.sparkling_step(ctypes.byref(c), v(FAKE), v(FAKE), v(FAKE), v(FAKE), v(FAKE),
                              v(FAKE), ctypes.byref(info), v(FAKE), n, None) == EINVAL
    assert lib.sparkling_step(ctypes.byref(c), v(FAKE), v(FAKE), v(FAKE), v(FAKE), v(0),
                              v(FAKE), ctypes.byref(info), v(FAKE), n, None) == EINVAL


def test_noalloc_step_validation(lib):
    """The allocation-free step rejects bad arguments, problems whose workspace
    exceeds its static scratch and the far field before any HIP call."""
    v = ctypes.c_void_p
    assert lib.spk_noalloc_scratch_bytes() == 64 << 20

    def call(prm, ptrs=None, it=0, eta=1.0):
        c = prm.c()
        a = ptrs or [FAKE] * 7
        return lib.sparkling_step_async_noalloc(ctypes.byref(c), *map(v, a[:6]), it, eta,
                                                v(a[6]), None)
    prm = good_params()
    assert spk.workspace_size(prm) <= 64 << 20
    assert call(prm, eta=0.0) == EINVAL
    assert call(prm, it=-1) == EINVAL
    for k in range(7):
        bad = [FAKE] * 7
        bad[k] = 0
        assert call(prm, bad) == EINVAL, k
    big = good_params(n_shots=1024, n_samples=512, grid=128)
    assert spk.workspace_size(big) > 64 << 20
    assert call(big) == EWORKSPACE
    assert "static scratch" in lib.spk_last_error().decode()
    assert call(good_params(far_field_depth=3, far_field_order=4)) == EUNSUPPORTED


def test_probe_validation(lib):
    v = ctypes.c_void_p
    pairs, ms = ctypes.c_double(), ctypes.c_double()

    def call(variant=0, blocks=4, iters=1, scratch=FAKE, nbytes=1 << 20, p=True):
        return lib.spk_probe_pair_mix(variant, blocks, iters, v(scratch), nbytes,
                                      ctypes.byref(pairs) if p else None, ctypes.byref(ms), None)
    assert call(variant=3) == EINVAL and call(variant=-1) == EINVAL
    assert call(blocks=0) == EINVAL and call(blocks=(1 << 20) + 1) == EINVAL
    assert call(iters=0) == EINVAL and call(p=False) == EINVAL
    assert call(scratch=0) == EINVAL
    assert call(blocks=4, nbytes=4 * 256 * 4 - 1) == EWORKSPACE


def test_timing_query_rejects_unknown_kind(lib):
    assert lib.spk_timing_query(9, None, None, None) == EINVAL


def test_python_binding_checks_shapes():
    import torch
    prm = good_params()
    with pytest.raises(ValueError):
        spk.grad(torch.zeros(3, prm.p), torch.zeros(prm.grid ** 3), prm)


def test_workloads_have_consistent_bounds(lib):
    for w in configs.WORKLOADS.values():
        a, b = spk.alpha_beta(configs.GMAX, configs.SMAX, configs.RASTER_DT, configs.DWELL_DT,
                              w.fov, w.kmax, configs.GAMMA_BAR, w.half_width)
        # gradient-amplitude bound binds at a 2 us dwell for every workload
        assert a == pytest.approx(configs.GAMMA_BAR * configs.GMAX * configs.RASTER_DT
                                  * w.half_width / w.kmax, rel=1e-14)
        assert a / b == pytest.approx(configs.GMAX / configs.SMAX / configs.RASTER_DT, rel=1e-12)
