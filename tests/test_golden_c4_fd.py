"""The stored central differences of the differentiation workload
(tests/golden/c4_fd.*, written by tests/golden/make_c4_fd.py from the oracle):
the inputs they were taken on, two entries recomputed, and the oracle's own
gradient agreeing with all 200 of them."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2108_02991_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load():
    with open(os.path.join(GOLDEN, "c4_fd.json")) as f:
        meta = json.load(f)
    return meta, np.load(os.path.join(GOLDEN, "c4_fd.npy"))


def c4_inputs():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_c4_fd",
                                                  os.path.join(GOLDEN, "make_c4_fd.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.c4_inputs()


def test_inputs_match_the_stored_digests():
    meta, fd = load()
    w, K, rho = c4_inputs()
    assert fd.shape == (meta["directions"], 2) and meta["directions"] == 200
    assert meta["K_digest"] == inputs.digest(K) and meta["rho_digest"] == inputs.digest(rho)
    assert meta["h"] == 1e-4 and meta["direction_kind"] == "rademacher"


def test_oracle_gradient_agrees_with_every_difference():
    """|FD_k - <grad F, e_k>| / ||grad F|| small for all 200 dense directions:
    the O(h^2) truncation only (the differences are cancellation-free)."""
    meta, fd = load()
    err = np.abs(fd[:, 0] - fd[:, 1]) / meta["grad_norm"]
    assert err.max() <= 1e-4
    # the directional derivatives are not all tiny: the check has something to compare
    assert np.median(np.abs(fd[:, 1])) >= 0.05 * meta["grad_norm"]


@pytest.mark.parametrize("k", [0, 199])
def test_two_entries_recomputed(k):
    meta, fd = load()
    w, K, rho = c4_inputs()
    e = inputs.rademacher(K.shape, meta["seed0"] + k)
    got = oracle.fd_directional(K, rho, w.grid, w.half_width, e, meta["h"])
    assert got == pytest.approx(fd[k, 0], rel=1e-12, abs=1e-18)
