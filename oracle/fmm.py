"""Plain NumPy reference of the repulsion's far field by the Chebyshev fast
multipole method -- TEST INFRASTRUCTURE ONLY (tests import it; the product
never does).  It shares no code with the HIP path.

The method ("Evaluating F^r and its gradient": the FMM for large p; the
kernel-independent Chebyshev variant, with the interpolation order n per axis
as its precision parameter), step by step in its textbook order:

* root cube: centre of the samples' bounding box, half-width R = (largest
  half-extent) * (1 + 2^-20) + 1e-30;
* uniform octree of depth D; sample i sits in leaf floor((x - (c - R)) /
  (2R / 2^D)) per axis, clamped to [0, 2^D - 1];
* upward pass: leaf weights W[m] = sum_i S_m(t_i) at the tensor Chebyshev
  nodes (t: coordinates scaled to the cell's [-1, 1]^3), then parents from
  children by interpolation at the children's nodes;
* interactions, levels 2..D: every cell receives from the cells of its
  interaction list (children of its parent's neighbours that are not its own
  neighbours) the kernel evaluated between node sets, applied to their
  weights;
* downward pass: children add their parent's expansion interpolated at their
  nodes; every sample adds its leaf's expansion interpolated at itself;
* near field: every sample sums the kernel exactly over the samples of the
  27 leaves around its leaf (itself included);
* adaptive tree (optional): leaves whose near field is dense enough
  (refined_leaves) take their targets one level deeper, where the same steps
  apply to them.

S_k(t) = 1/n + (2/n) sum_{i=1}^{n-1} T_i(tbar_k) T_i(t), tbar_k = cos((2k+1) pi
/ 2n).  Parity unpinned except by the pins in the tests (exactness for
polynomial kernels of degree below n, convergence to the exact sum).
"""
import itertools

import numpy as np


def cheb_nodes(n):
    return np.cos((2 * np.arange(n) + 1) * np.pi / (2 * n))


def cheb_S(n, t):
    """S[k, j] = S_k(t_j)."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    Tb = np.cos(np.outer(np.arange(n), np.arccos(cheb_nodes(n))))      # [i, k]
    Tt = np.empty((n, t.size))
    Tt[0] = 1.0
    if n > 1:
        Tt[1] = t
    for i in range(2, n):
        Tt[i] = 2 * t * Tt[i - 1] - Tt[i - 2]
    w = np.full(n, 2.0 / n)
    w[0] = 1.0 / n
    return (Tb * w[:, None]).T @ Tt


def distance_kernel(eps=0.0):
    def k(d):
        s = (d ** 2).sum(axis=-1) + eps * eps
        r = np.sqrt(s)
        with np.errstate(invalid="ignore", divide="ignore"):
            g = np.where(r[..., None] > 0, d / np.where(r > 0, r, 1.0)[..., None], 0.0)
        return r, g
    return k


def log_kernel(eps):
    def k(d):
        s = (d ** 2).sum(axis=-1) + eps * eps
        return 0.5 * np.log(s), d / s[..., None]
    return k


def square_kernel():
    """H(d) = |d|^2 (degree 2): interpolated exactly from order 3 on."""
    def k(d):
        return (d ** 2).sum(axis=-1), 2.0 * d
    return k


def exact(X, kernel):
    """(g (p, 3), u (p,)): sum over all j of grad H(x_i - x_j) and H(x_i - x_j)
    (rows in blocks, to bound the memory of the pair arrays)."""
    g = np.empty((X.shape[0], 3))
    u = np.empty(X.shape[0])
    for a in range(0, X.shape[0], 1024):
        uu, gg = kernel(X[a:a + 1024, None, :] - X[None, :, :])
        g[a:a + 1024] = gg.sum(axis=1)
        u[a:a + 1024] = uu.sum(axis=1)
    return g, u


def refine_threshold(n):
    """Price of refining one leaf, in direct pairs: 8 children x 189
    interactions x 4 components x n^6 multiply-adds at 1/7 of a pair each."""
    return 8 * 189 * 4 * n ** 6 // 7


def _around(counts):
    """Sum of counts over the (existing) 27 cells around every cell."""
    N = counts.shape[0]
    pad = np.zeros((N + 2,) * 3, dtype=np.int64)
    pad[1:-1, 1:-1, 1:-1] = counts
    out = np.zeros_like(counts)
    for o in itertools.product((0, 1, 2), repeat=3):
        out += pad[o[0]:o[0] + N, o[1]:o[1] + N, o[2]:o[2] + N]
    return out


def refined_leaves(leaf, fine, depth, n):
    """Adaptive tree: cells (of level `depth`, coordinates `leaf`) whose targets
    take their near field one level deeper (coordinates `fine`).  A cell is
    refined when the direct pairs this saves, n_L * (samples around L) - sum
    over children c of n_c * (samples around c), exceed refine_threshold(n);
    exact integers."""
    N = 2 ** depth
    cL = np.zeros((N, N, N), dtype=np.int64)
    np.add.at(cL, (leaf[:, 0], leaf[:, 1], leaf[:, 2]), 1)
    cF = np.zeros((2 * N,) * 3, dtype=np.int64)
    np.add.at(cF, (fine[:, 0], fine[:, 1], fine[:, 2]), 1)
    coarse = cL * _around(cL)
    fine_pairs = (cF * _around(cF)).reshape(N, 2, N, 2, N, 2).sum(axis=(1, 3, 5))
    return (cL > 0) & (coarse - fine_pairs > refine_threshold(n))


def fmm(X, depth, n, kernel, adaptive=0, info=None, only=None):
    """Repulsion sums of every sample by the Chebyshev FMM; X is (p, 3).

    adaptive = R (0, 1 or 2; True counts as 1): refinement levels below the
    leaves.  A leaf is refined by refined_leaves; with R = 2 a child of a
    refined leaf is refined again by the same rule one level down.  A
    target's final level is the deepest level its cells reach: its local
    expansion comes from that level (its interactions included) and its
    near field from the 27 cells of that level around it.  A target whose
    leaf is not refined is treated as in the uniform tree of the given
    depth.  info (a dict) receives the final level of every target.  only (a
    boolean mask) limits the near field to those targets; the other rows then
    hold the far field alone.
    """
    X = np.asarray(X, dtype=np.float64)
    p = X.shape[0]
    R_ = int(adaptive)
    lo, hi = X.min(axis=0), X.max(axis=0)
    c0 = 0.5 * (lo + hi)
    R = (0.5 * (hi - lo)).max() * (1.0 + 2.0 ** -20) + 1e-30
    F = depth + R_                                       # deepest level
    tb = cheb_nodes(n)
    n3 = n ** 3
    m = np.arange(n3)
    m3 = np.stack([m % n, (m // n) % n, m // (n * n)], axis=1)          # x fastest

    def Sm(t):                                                           # (q, 3) -> (n^3, q)
        return (cheb_S(n, t[:, 0])[m3[:, 0]] * cheb_S(n, t[:, 1])[m3[:, 1]]
                * cheb_S(n, t[:, 2])[m3[:, 2]])

    def centre(level, cell):
        h = 2 * R / 2 ** level
        return c0 - R + (np.asarray(cell) + 0.5) * h, 0.5 * h

    def cell_of(level):
        Nl = 2 ** level
        return np.clip(np.floor((X - (c0 - R)) / (2 * R / Nl)).astype(np.int64), 0, Nl - 1)

    cell_at = {l: cell_of(l) for l in range(depth, F + 1)}
    leaf, fine = cell_at[depth], cell_at[F]
    final = np.full(p, depth)                            # final level of every target
    refine_go = np.ones(p, dtype=bool)                   # still refining
    for l in range(depth, F):
        rl = refined_leaves(cell_at[l], cell_at[l + 1], l, n)
        hit = refine_go & rl[cell_at[l][:, 0], cell_at[l][:, 1], cell_at[l][:, 2]]
        final[hit] = l + 1
        refine_go = hit
    ref = final > depth
    if info is not None:
        info["final_level"] = final
        info["refined_targets"] = ref

    # upward pass from the deepest level
    NF = 2 ** F
    W = {F: np.zeros((NF, NF, NF, n3))}
    cc, hh = centre(F, fine)
    np.add.at(W[F], (fine[:, 0], fine[:, 1], fine[:, 2]), Sm((X - cc) / hh).T)
    T = np.zeros((8, n3, n3))                                            # [pos, parent m, child l]
    for pos in range(8):
        b = np.array([pos & 1, (pos >> 1) & 1, (pos >> 2) & 1])
        T[pos] = Sm((-0.5 + b[None, :]) + 0.5 * tb[m3])
    for lvl in range(F - 1, 1, -1):
        Nl = 2 ** lvl
        W[lvl] = np.zeros((Nl, Nl, Nl, n3))
        for pos in range(8):
            b = [pos & 1, (pos >> 1) & 1, (pos >> 2) & 1]
            W[lvl] += W[lvl + 1][b[0]::2, b[1]::2, b[2]::2] @ T[pos].T
    # interactions
    Lx = {lvl: np.zeros((2 ** lvl,) * 3 + (4, n3)) for lvl in range(2, F + 1)}
    for lvl in range(2, F + 1):
        Nl = 2 ** lvl
        h = 2 * R / Nl
        cells = np.stack(np.meshgrid(*(np.arange(Nl),) * 3, indexing="ij"), -1).reshape(-1, 3)
        for o in itertools.product(range(-3, 4), repeat=3):
            o = np.array(o)
            if np.abs(o).max() <= 1:
                continue                                  # a neighbour: near field
            src = cells + o
            inside = ((src >= 0) & (src < Nl)).all(axis=1)
            parents_near = np.abs(src // 2 - cells // 2).max(axis=1) <= 1
            ok = inside & parents_near                    # in the cell's interaction list
            if not ok.any():
                continue
            d = 0.5 * h * tb[m3][:, None, :] - (o * h + 0.5 * h * tb[m3])[None, :, :]
            u, g = kernel(d)
            Kc = np.stack([g[..., 0], g[..., 1], g[..., 2], u])          # (4, m, l)
            t, s_ = cells[ok], src[ok]
            w = W[lvl][s_[:, 0], s_[:, 1], s_[:, 2]]                       # (k, l)
            Lx[lvl][t[:, 0], t[:, 1], t[:, 2]] += np.einsum("cml,kl->kcm", Kc, w)
    # downward pass
    for lvl in range(2, F):
        for pos in range(8):
            b = [pos & 1, (pos >> 1) & 1, (pos >> 2) & 1]
            Lx[lvl + 1][b[0]::2, b[1]::2, b[2]::2] += Lx[lvl] @ T[pos]
    far = np.zeros((p, 4))
    for level in range(depth, F + 1):
        cellv, sel = cell_at[level], final == level
        if not sel.any():
            continue
        cs, hs = centre(level, cellv[sel])
        far[sel] = np.einsum("pcm,mp->pc",
                             Lx[level][cellv[sel, 0], cellv[sel, 1], cellv[sel, 2]],
                             Sm((X[sel] - cs) / hs))
    g = far[:, :3].copy()
    u = far[:, 3].copy()
    # near field: the 27 cells of each target's final level around its cell
    for level in range(depth, F + 1):
        cellv, sel = cell_at[level], final == level
        members = {}
        for i, key in enumerate(map(tuple, cellv)):
            members.setdefault(key, []).append(i)
        targets = {}
        for i in np.flatnonzero(sel if only is None else sel & only):
            targets.setdefault(tuple(cellv[i]), []).append(i)
        for key, tgt in targets.items():
            src = [j for o in itertools.product((-1, 0, 1), repeat=3)
                   for j in members.get(tuple(np.array(key) + o), [])]
            uu, gg = kernel(X[tgt][:, None, :] - X[src][None, :, :])
            g[tgt] += gg.sum(axis=1)
            u[tgt] += uu.sum(axis=1)
    return g, u
