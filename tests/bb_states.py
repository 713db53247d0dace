"""Step-state inputs with a known Barzilai-Borwein quotient (section "Choice of
step size": BB1, eta = s.s / s.y, over all 3p coordinates).

For a current point K and its gradient g the previous state is built as

    k_prev = K - s,    g_prev = g - c * s,

with s = +-sigma on the first half of the 3p coordinates and +-2 sigma on the
second half, and c = c1 on the first half, c2 on the second.  K is rounded to
a 2^-30 grid and sigma is a power of two no finer than that, so K - k_prev
recovers s exactly; y = g - g_prev equals c * s up to the one rounding of
g_prev.  Then

    s.s / s.y = (n1 + 4 n2) / (c1 n1 + 4 c2 n2)        (n1 = n2 = 3p/2)

whatever g is: a value fixed by construction, not by re-evaluating the
formula.  BB2 (s.y / y.y) gives (c1 + 4 c2) / (c1^2 + 4 c2^2) on the same
state, a different number, so the two variants cannot be confused.
"""
import numpy as np


def quantise(K, bits=30):
    """K rounded to multiples of 2^-bits (exact differences with sigma below)."""
    return np.round(np.asarray(K, dtype=np.float64) * 2.0 ** bits) / 2.0 ** bits


def bb_expected(c1, c2):
    """The quotient s.s/s.y of the state built by bb_state (equal halves)."""
    return 5.0 / (c1 + 4.0 * c2)


def bb2_value(c1, c2):
    """What the other Barzilai-Borwein variant s.y/y.y would give."""
    return (c1 + 4.0 * c2) / (c1 * c1 + 4.0 * c2 * c2)


def bb_state(K, g, c1, c2, seed=5, bits=30):
    """(k_prev, g_prev) for the current point K (on the 2^-bits grid) and its gradient g."""
    K = np.asarray(K, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = K.size
    assert n % 2 == 0 and np.array_equal(K, quantise(K, bits))
    rng = np.random.default_rng(seed)
    # sigma: a power of two with |c s| on the scale of |g|, so y keeps ~1e-16 relative
    # error; at most 1/16, so that |K - s| < 1 keeps K - s exact on the grid
    c_mean = 0.5 * (abs(c1) + abs(c2))
    scale = np.sqrt(np.mean(g * g)) / c_mean
    sigma = 2.0 ** min(-4, max(-bits, int(np.round(np.log2(scale)))))
    half = n // 2
    mag = np.where(np.arange(n) < half, sigma, 2.0 * sigma)
    s = (mag * rng.choice([-1.0, 1.0], size=n)).reshape(K.shape)
    c = np.where(np.arange(n) < half, c1, c2).reshape(K.shape)
    k_prev = K - s
    assert np.array_equal(K - k_prev, s)
    g_prev = g - c * s
    return k_prev, g_prev
