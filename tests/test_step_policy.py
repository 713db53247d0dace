"""Regularised-kernel step policy (Sec. "Choice of step size"): the library's
bound on the Lipschitz constant of grad F, checked on the CPU against Hessian
eigenvalues measured by finite differences of the oracle gradient, and the
descent it guarantees in the oracle's projected gradient steps."""
import numpy as np
import pytest

import oracle
from paper_2108_02991_amd import api, inputs


def _hv(K, rho, G, L, eps, kernel, v, h=1e-6):
    gp = oracle.grad(K + h * v, rho, G, L, eps, kernel=kernel)["dF"]
    gm = oracle.grad(K - h * v, rho, G, L, eps, kernel=kernel)["dF"]
    return (gp - gm) / (2 * h)


def _largest_eigenvalue(K, rho, G, L, eps, kernel, iters=80, seed=0):
    """Largest-magnitude Hessian eigenvalue of F by power iteration (signed)."""
    v = np.random.default_rng(seed).normal(size=K.shape)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = _hv(K, rho, G, L, eps, kernel, v)
        lam = float((v * w).sum())
        v = w / np.linalg.norm(w)
    return lam


@pytest.mark.parametrize("kernel,eps", [("distance", 0.05), ("distance", 0.01),
                                        ("log", 0.05), ("log", 0.02)])
@pytest.mark.parametrize("seed", [0, 1])
def test_bound_holds_on_random_configurations(kernel, eps, seed):
    rng = np.random.default_rng(seed)
    G, L, p = 3, 0.5, 24
    K = rng.uniform(-L, L, (3, p)) * rng.uniform(0.05, 1.0)
    rho = rng.uniform(0, 1, G ** 3) ** 2
    rho /= rho.sum()
    lam = _largest_eigenvalue(K, rho, G, L, eps, kernel, seed=seed)
    bound = api.lipschitz_bound(p, eps, 1.0, kernel)
    assert abs(lam) <= bound * (1 + 1e-6), (lam, bound)


@pytest.mark.parametrize("kernel,ratio", [("distance", 0.95), ("log", 0.85)])
def test_bound_is_nearly_attained(kernel, ratio):
    """Coincident samples far from the density mass: the repulsion's Hessian reaches
    -1/(p eps) (distance) or -1/(p eps^2) (log) on zero-mean directions."""
    G, L, p, eps = 3, 0.5, 12, 0.01
    K = np.full((3, p), 0.4)
    rho = np.zeros(G ** 3)
    rho[0] = 1.0                                   # the cell at (-1/3, -1/3, -1/3)
    lam = _largest_eigenvalue(K, rho, G, L, eps, kernel, iters=40)
    bound = api.lipschitz_bound(p, eps, 1.0, kernel)
    assert lam < 0 and ratio * bound <= -lam <= bound * (1 + 1e-6), (lam, bound)


def test_bound_formula_scaling_and_validation():
    # 1/p and 1/eps (distance), 1/eps^2 (log); a heavier density raises the bound
    assert api.lipschitz_bound(100, 0.1) == pytest.approx(2 * api.lipschitz_bound(200, 0.1))
    assert api.lipschitz_bound(100, 0.1) == pytest.approx(2 * api.lipschitz_bound(100, 0.2))
    assert api.lipschitz_bound(100, 0.1, kernel="log") == pytest.approx(
        4 * api.lipschitz_bound(100, 0.2, kernel="log"))
    assert api.lipschitz_bound(10, 0.1, 3.0) == pytest.approx(3 * api.lipschitz_bound(10, 0.1))
    for bad in [(0, 0.1, 1.0), (10, 0.0, 1.0), (10, -1.0, 1.0), (10, 0.1, -1.0),
                (10, float("nan"), 1.0), (10, 0.1, float("inf"))]:
        with pytest.raises(api.SparklingError):
            api.lipschitz_bound(*bad)


@pytest.mark.parametrize("kernel,eps", [("distance", 0.03), ("log", 0.03)])
def test_fixed_step_one_over_lipschitz_decreases_f(kernel, eps):
    """Exact projection (box and TE only): F(K+) <= F(K) - (L/2) |K+ - K|^2."""
    Nc, Ns, G, L = 8, 24, 6, 0.5
    p = Nc * Ns
    K = inputs.radial_spokes(Nc, Ns, L, seed=5, jitter=0.05)
    rho = inputs.radial_density(G, L, 0.1, 2.0)
    lip = api.lipschitz_bound(p, eps, float(rho.sum()), kernel)
    z = np.zeros_like(K)
    kp, gp = z, z
    F_prev, K_prev = None, None
    for it in range(6):
        K_new, kp, gp, info = oracle.step(K, rho, Nc, Ns, G, L, 1e3, 1e3, 0, 0, kp, gp, it,
                                          1.0 / lip, eps, kernel=kernel)
        if F_prev is not None:
            drop = 0.5 * lip * float(((K - K_prev) ** 2).sum())
            assert info["F"] <= F_prev - drop + 1e-13, (it, info["F"], F_prev, drop)
            assert drop > 0
        F_prev, K_prev, K = info["F"], K, K_new
