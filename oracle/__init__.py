"""FP64 CPU oracle for the SPARKLING energy/gradient/projection path.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product package.  It is a
thin ctypes wrapper over ``oracle.c`` (plain C99 + OpenMP, FP64), which
computes every quantity straight from the paper's definitions; inputs in any
float dtype are up-cast exactly to float64 before the call.

Parity pins: closed forms, invariants, brute force and finite differences in
``tests/test_oracle_pins.py``.  The one quantity without a pin is the cost
value printed for the perturbation study (its inputs are not given): parity
unpinned for that number only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "liboracle.so"
_lib = None

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_int = ctypes.c_int
_p = ctypes.c_void_p


def build(force: bool = False) -> Path:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, no FMA contraction)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out_dir) -> Path:
    """oracle.c built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc;
    any undefined behaviour aborts).  Load it by setting SPK_ORACLE_LIB to the
    returned path in a process started with gcc's libasan in LD_PRELOAD."""
    out = Path(out_dir) / "liboracle_asan_ubsan.so"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-Wextra", "-o", str(out), str(_SRC), "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _load():
    global _lib
    if _lib is None:
        override = os.environ.get("SPK_ORACLE_LIB")
        if override:
            lib = ctypes.CDLL(override)
        else:
            build()
            lib = ctypes.CDLL(str(_LIB))
        for name, args in {
            "orc_grad": [_i64, _p, _p, _p, _i64, _dbl, _p, _dbl, _int, _i64, _p, _p, _p, _p, _p, _p],
            "orc_energy": [_i64, _p, _p, _p, _i64, _dbl, _p, _dbl, _int, _p],
            "orc_rho_self_energy": [_i64, _dbl, _p, _dbl, _int, _p],
            "orc_alpha_beta": [_dbl] * 8 + [_p, _p],
            "orc_project": [_i64, _i64, _p, _p, _p, _dbl, _dbl, _dbl, _i64, ctypes.c_int,
                            ctypes.c_int, _p],
            "orc_constraint_check": [_i64, _i64, _p, _p, _p, _dbl, _dbl, _dbl, _i64, ctypes.c_int,
                                     _p],
            "orc_step": [_i64, _i64, _p, _i64, _dbl, _p, _dbl, _int, _dbl, _dbl, _i64, _int, _int,
                         _p, _p, _i64, _dbl, _p, _p],
            "orc_fd_directional": [_i64, _p, _p, _p, _i64, _dbl, _p, _dbl, _int, _p, _dbl, _p],
            "orc_num_threads": [],
            "orc_upsample": [_i64, _i64, _p, _p],
            "orc_field": [_i64, _dbl, _p, _dbl, _int, _p],
            "orc_interpolate": [_i64, _dbl, _p, _i64, _p, _p, _p, _p],
            "orc_grad_field": [_i64, _p, _p, _p, _i64, _dbl, _p, _dbl, _int, _i64, _p, _p, _p, _p, _p, _p],
        }.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


KERNELS = {"distance": 0, "log": 1}


def _kern(name: str) -> int:
    """Kernel selector: "distance" H = sqrt(|d|^2 + eps^2); "log" H = log(|d|^2 + eps^2) / 2."""
    return KERNELS[name]


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, name: str):
    if rc != 0:
        raise ValueError(f"oracle {name} rejected its arguments (status {rc})")


def num_threads() -> int:
    return _load().orc_num_threads()


def grad(K, rho, G: int, L: float, eps: float = 0.0, targets=None, kernel: str = "distance"):
    """Gradient of F at the listed targets (all if None).

    Returns dict with dF, dFa, dFr of shape (3, n_t) and the unscaled
    per-target potentials ua = sum_v rho_v H(K_i - x_v), ur = sum_j H(K_i - K_j).
    """
    K = _f64(K)
    rho = _f64(rho)
    p = K.shape[1]
    if targets is None:
        targets = np.arange(p, dtype=np.int64)
    targets = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    n_t = targets.size
    dF, dFa, dFr = (np.empty((3, n_t)) for _ in range(3))
    ua, ur = np.empty(n_t), np.empty(n_t)
    x, y, z = (np.ascontiguousarray(K[c]) for c in range(3))
    rc = _load().orc_grad(p, _ptr(x), _ptr(y), _ptr(z), G, L, _ptr(rho), eps, _kern(kernel),
                          n_t, _ptr(targets), _ptr(dF), _ptr(dFa), _ptr(dFr), _ptr(ua), _ptr(ur))
    _check(rc, "grad")
    return {"dF": dF, "dFa": dFa, "dFr": dFr, "ua": ua, "ur": ur, "targets": targets}


def energy(K, rho, G: int, L: float, eps: float = 0.0, kernel: str = "distance"):
    """(F, Fa, Fr) of the objective."""
    K = _f64(K)
    rho = _f64(rho)
    out = np.empty(3)
    x, y, z = (np.ascontiguousarray(K[c]) for c in range(3))
    rc = _load().orc_energy(K.shape[1], _ptr(x), _ptr(y), _ptr(z), G, L, _ptr(rho), eps,
                            _kern(kernel), _ptr(out))
    _check(rc, "energy")
    return tuple(float(v) for v in out)


def rho_self_energy(rho, G: int, L: float, eps: float = 0.0, kernel: str = "distance") -> float:
    rho = _f64(rho)
    out = np.empty(1)
    _check(_load().orc_rho_self_energy(G, L, _ptr(rho), eps, _kern(kernel), _ptr(out)), "rho_self_energy")
    return float(out[0])


def alpha_beta(gmax, smax, raster_dt, dwell_dt, fov, kmax, gamma_bar, half_width):
    a, b = np.empty(1), np.empty(1)
    rc = _load().orc_alpha_beta(gmax, smax, raster_dt, dwell_dt, fov, kmax, gamma_bar,
                                half_width, _ptr(a), _ptr(b))
    _check(rc, "alpha_beta")
    return float(a[0]), float(b[0])


def _duals_ptr(duals, n_shots, n_samples):
    """The warm-start dual state: None (cold start) or a C-contiguous float64
    array of n_shots * 6 * n_samples, updated in place."""
    if duals is None:
        return None
    if (not isinstance(duals, np.ndarray) or duals.dtype != np.float64
            or not duals.flags.c_contiguous or duals.size != n_shots * 6 * n_samples):
        raise ValueError("duals must be a C-contiguous float64 array of n_shots*6*n_samples")
    return _ptr(duals)


def project(K, n_shots: int, n_samples: int, L: float, a: float, b: float, te: int,
            n_pit: int, rotation_variant: bool = False, duals=None) -> np.ndarray:
    """Per-shot projection of K (3, Nc*Ns); returns a new float64 array.  With
    duals (shape (Nc, 6, Ns): q then r per coordinate) the dual iteration starts
    from them and leaves its last iterate there."""
    K = _f64(K).copy()
    rc = _load().orc_project(n_shots, n_samples, _ptr(K[0]), _ptr(K[1]), _ptr(K[2]),
                             L, a, b, te, n_pit, int(rotation_variant),
                             _duals_ptr(duals, n_shots, n_samples))
    _check(rc, "project")
    return K


def constraint_check(K, n_shots: int, n_samples: int, L: float, a: float, b: float,
                     te: int, rotation_variant: bool = False) -> np.ndarray:
    K = _f64(K)
    out = np.empty(4)
    x, y, z = (np.ascontiguousarray(K[c]) for c in range(3))
    rc = _load().orc_constraint_check(n_shots, n_samples, _ptr(x), _ptr(y), _ptr(z),
                                      L, a, b, te, int(rotation_variant), _ptr(out))
    _check(rc, "constraint_check")
    return out


def step(K, rho, n_shots, n_samples, G, L, a, b, te, n_pit, k_prev, g_prev, it, eta_fixed,
         eps: float = 0.0, rotation_variant: bool = False, kernel: str = "distance",
         duals=None):
    """One projected gradient step.  Returns (K_new, k_prev, g_prev, info dict).
    duals: the projection's warm-start state (see project), updated in place."""
    K = _f64(K).copy()
    k_prev = _f64(k_prev).copy()
    g_prev = _f64(g_prev).copy()
    rho = _f64(rho)
    info = np.empty(10)
    rc = _load().orc_step(n_shots, n_samples, _ptr(K), G, L, _ptr(rho), eps, _kern(kernel), a, b,
                          te, n_pit, int(rotation_variant), _ptr(k_prev), _ptr(g_prev), it, eta_fixed,
                          _ptr(info), _duals_ptr(duals, n_shots, n_samples))
    _check(rc, "step")
    d = {"eta": info[0], "F": info[1], "Fa": info[2], "Fr": info[3],
         "viol": info[4:8].copy(), "bb_used": bool(info[8]), "bb_quotient": info[9]}
    return K, k_prev, g_prev, d


def fd_directional(K, rho, G, L, delta, h, eps: float = 0.0, kernel: str = "distance") -> float:
    """(F(K + h delta) - F(K - h delta)) / (2h), cancellation-free."""
    K = _f64(K)
    rho = _f64(rho)
    delta = _f64(delta)
    out = np.empty(1)
    x, y, z = (np.ascontiguousarray(K[c]) for c in range(3))
    rc = _load().orc_fd_directional(K.shape[1], _ptr(x), _ptr(y), _ptr(z), G, L, _ptr(rho),
                                    eps, _kern(kernel), _ptr(delta), h, _ptr(out))
    _check(rc, "fd_directional")
    return float(out[0])


def field(rho, G: int, L: float, eps: float = 0.0, kernel: str = "distance") -> np.ndarray:
    """Node field of the grid attraction, shape ((G+2)^3, 4): U, dU/dx, dU/dy, dU/dz."""
    rho = _f64(rho)
    out = np.empty(((G + 2) ** 3, 4))
    _check(_load().orc_field(G, L, _ptr(rho), eps, _kern(kernel), _ptr(out)), "field")
    return out


def interpolate(node_field, G: int, L: float, P) -> np.ndarray:
    """Trilinear interpolant of a ((G+2)^3, 4) node field at points P (3, n) -> (4, n)."""
    f = _f64(node_field)
    P = _f64(P)
    n = P.shape[1]
    out = np.empty((4, n))
    x, y, z = (np.ascontiguousarray(P[c]) for c in range(3))
    _check(_load().orc_interpolate(G, L, _ptr(f), n, _ptr(x), _ptr(y), _ptr(z), _ptr(out)),
           "interpolate")
    return out


def grad_field(K, rho, G: int, L: float, eps: float = 0.0, targets=None,
               kernel: str = "distance"):
    """Gradient with the grid attraction (node field + trilinear interpolant) at targets."""
    K = _f64(K)
    rho = _f64(rho)
    p = K.shape[1]
    if targets is None:
        targets = np.arange(p, dtype=np.int64)
    targets = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    n_t = targets.size
    dF, dFa, dFr = (np.empty((3, n_t)) for _ in range(3))
    ua, ur = np.empty(n_t), np.empty(n_t)
    x, y, z = (np.ascontiguousarray(K[c]) for c in range(3))
    rc = _load().orc_grad_field(p, _ptr(x), _ptr(y), _ptr(z), G, L, _ptr(rho), eps, _kern(kernel),
                                n_t, _ptr(targets), _ptr(dF), _ptr(dFa), _ptr(dFr), _ptr(ua), _ptr(ur))
    _check(rc, "grad_field")
    return {"dF": dF, "dFa": dFa, "dFr": dFr, "ua": ua, "ur": ur, "targets": targets}


def upsample(K, n_shots: int, n_samples: int) -> np.ndarray:
    """Dyadic linear up-sampling of every shot: (3, Nc*N) -> (3, Nc*2N)."""
    K = _f64(K)
    out = np.empty((3, 2 * K.shape[1]))
    _check(_load().orc_upsample(n_shots, n_samples, _ptr(K), _ptr(out)), "upsample")
    return out


def multiresolution(K0, rho, n_shots, n_samples_coarse, levels, G, L, a, b, te, n_pit, n_git,
                    eta_scale=0.25, final_level=True, eps=0.0, kernel="distance"):
    """Algorithm 1: projected gradient iterations on decimated shots, warm restart by
    linear up-sampling, bounds halved per level.  K0 holds the coarsest shots
    (n_samples_coarse each); a, b are the full-resolution per-raster bounds, scaled
    by 2^d at decimation level d.  Returns the final K and the per-level records."""
    K = _f64(K0).copy()
    Ns = n_samples_coarse
    recs = []
    for d in range(levels, -1 if final_level else 0, -1):
        p = n_shots * Ns
        ad, bd = a * 2.0 ** d, b * 2.0 ** d
        eta = eta_scale * (2.0 * L) * p ** (2.0 / 3.0)
        kp, gp = np.zeros_like(K), np.zeros_like(K)
        for it in range(n_git):
            K, kp, gp, info = step(K, rho, n_shots, Ns, G, L, ad, bd, te, n_pit, kp, gp, it, eta,
                                   eps, kernel=kernel)
            recs.append(dict(level=d, iter=it, **info))
        if d > 0:
            K = upsample(K, n_shots, Ns)
            Ns *= 2
    return K, recs
