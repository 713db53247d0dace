// Far field of the repulsion sums by a Chebyshev-interpolation fast multipole
// method on an octree (the hierarchical far field for very large p; the paper
// uses a CPU FMM of this family, "Evaluating F^r and its gradient").  The
// octree is uniform to depth D; optionally, cells whose near field is dense
// are refined up to R = 2 levels further, and a target then takes its near
// field and its local expansion at the deepest level its cells reach.
//
// For target i and every sample j farther than the 27 leaves around i's leaf,
// H(x_i - x_j) and grad H(x_i - x_j) are replaced by their tensor Chebyshev
// interpolants of order n in both arguments, summed level by level:
//   P2P-free upward pass:  W_leaf[m]   = sum_{j in leaf} S_m(x_j)
//                          W_parent[m] = sum_children sum_l S_m(y_child,l) W_child[l]
//   interactions (M2L):    L_cell[c][m] = sum_{s in IL(cell)} sum_l K_c(x_m - y_l) W_s[l]
//                          with IL = children of the parent's neighbours that
//                          are not neighbours of the cell (189 per cell)
//   downward pass (L2L):   L_child[c][l] += sum_m S_m(x_child,l) L_parent[c][m]
//   evaluation (L2P):      far_c(x_i) = sum_m S_m(x_i) L_leaf[c][m]
// with K_0..2 = the components of grad H and K_3 = H, S_m the product of 1-D
// Chebyshev interpolation polynomials
//   S_k(t) = 1/n + (2/n) sum_{i=1}^{n-1} T_i(tbar_k) T_i(t),  tbar_k = cos((2k+1) pi / 2n),
// and t the coordinate in the cell scaled to [-1, 1].  The near field (27
// cells) is summed exactly by the sample sweep's pair arithmetic (sweep.hip),
// on a second stream beside the M2L.
//
// Layout.  Samples are sorted (stable radix sort) by the composite index of
// their cell R levels below the leaves (comp_index: x-fastest leaf index, then
// child positions), so every cell of every level from the leaves down owns
// one run of the sorted samples.  The cells of level l (2^l per axis) are
// split into 8 parity classes; each class is a sub-grid of side Q = 2^l / 2
// padded by 2 zero cells on every side (side P = Q + 4).  A target class and
// an offset of its interaction list then map every target to its source by
// one constant shift of the padded linear index, so M2L is a GEMM over the
// class's cells, run on the FP64 matrix cores: C[col][row] += A_o[row][k]
// B[col + shift][k], with rows (component, node) and k the source nodes.  M2M
// and L2L use the same GEMM loop with the transfer matrices.  Empty cells (no
// samples) are skipped.  Every stage runs in double precision and in a fixed
// order.

#include <algorithm>
#include <cfloat>
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "spk_internal.h"

namespace spk {
namespace {

constexpr int EW = 256;
constexpr int kMaxOrder = kFmmMaxOrder;
inline unsigned ew_blocks(int64_t n) { return (unsigned)((n + EW - 1) / EW); }

// Host-computed Chebyshev tables passed by value: tb[i][k] = T_i(tbar_k).
struct Cheb {
    int n;
    double tbar[kMaxOrder];
    double tb[kMaxOrder][kMaxOrder];
};

// S_k(t) for k = 0..N-1 (T_i(t) by the three-term recurrence).
template <int N>
__device__ inline void cheb_s(const Cheb &ch, double t, double (&s)[N])
{
    double tp[N];
    tp[0] = 1.0;
    if (N > 1)
        tp[1] = t;
#pragma unroll
    for (int i = 2; i < N; ++i)
        tp[i] = 2.0 * t * tp[i - 1] - tp[i - 2];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double a = 0.0;
#pragma unroll
        for (int i = 1; i < N; ++i)
            a += ch.tb[i][k] * tp[i];
        s[k] = 1.0 / N + (2.0 / N) * a;
    }
}

// S_k(t) for one k.
template <int N>
__device__ inline double cheb_s1(const Cheb &ch, int k, double t)
{
    double a = 0.0, t0 = 1.0, t1 = t;
#pragma unroll
    for (int i = 1; i < N; ++i) {
        a += ch.tb[i][k] * t1;
        const double t2 = 2.0 * t * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    return 1.0 / N + (2.0 / N) * a;
}

// ------------------------------------------------------------------ box
template <typename T>
__global__ __launch_bounds__(EW) void box_stage1(const T *x, const T *y, const T *z, int64_t p,
                                                 double *part)
{
    __shared__ double red[6][EW];
    double v[6] = {DBL_MAX, DBL_MAX, DBL_MAX, -DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x; i < p; i += (int64_t)gridDim.x * EW) {
        const double c[3] = {(double)x[i], (double)y[i], (double)z[i]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = c[a] < v[a] ? c[a] : v[a];
            v[3 + a] = c[a] > v[3 + a] ? c[a] : v[3 + a];
        }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a)
        red[a][threadIdx.x] = v[a];
    __syncthreads();
    for (int w = EW / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double o = red[a][threadIdx.x + w], q = red[3 + a][threadIdx.x + w];
                red[a][threadIdx.x] = o < red[a][threadIdx.x] ? o : red[a][threadIdx.x];
                red[3 + a][threadIdx.x] = q > red[3 + a][threadIdx.x] ? q : red[3 + a][threadIdx.x];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6)
        part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// box[0..2] = centre, box[3] = half-width of the root cube (a little larger
// than the samples' extent, and never zero).
__global__ void box_stage2(const double *part, int nblk, double *box)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int b = 0; b < nblk; ++b)
        for (int a = 0; a < 3; ++a) {
            lo[a] = part[b * 6 + a] < lo[a] ? part[b * 6 + a] : lo[a];
            hi[a] = part[b * 6 + 3 + a] > hi[a] ? part[b * 6 + 3 + a] : hi[a];
        }
    double R = 0.0;
    for (int a = 0; a < 3; ++a) {
        box[a] = 0.5 * (lo[a] + hi[a]);
        const double h = 0.5 * (hi[a] - lo[a]);
        R = h > R ? h : R;
    }
    R = R * (1.0 + 0x1p-20) + 1e-30;
    box[3] = R;
}

// Leaf coordinate along one axis, clamped to [0, N-1] (NaN goes to 0).
__device__ inline int64_t leaf_coord(double x, double c, double R, int64_t N)
{
    double k = floor((x - (c - R)) / (2.0 * R / (double)N));
    k = !(k >= 0.0) ? 0.0 : (k > (double)(N - 1) ? (double)(N - 1) : k);
    return (int64_t)k;
}

// Samples are keyed by the composite index (comp_index) of their cell R levels
// below the leaves (R = 0: the x-fastest leaf index), so every cell of every
// level from the leaves down owns one run of the sorted samples.
template <typename T>
__global__ __launch_bounds__(EW) void leaf_keys_kernel(const T *x, const T *y, const T *z, int64_t p,
                                                       const double *box, int R, int64_t sD,
                                                       uint32_t *key, uint32_t *val)
{
    const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (i >= p)
        return;
    const double R_ = box[3];
    const int64_t N = sD << R;
    const int64_t ix = leaf_coord((double)x[i], box[0], R_, N);
    const int64_t iy = leaf_coord((double)y[i], box[1], R_, N);
    const int64_t iz = leaf_coord((double)z[i], box[2], R_, N);
    key[i] = (uint32_t)comp_index(ix, iy, iz, R, sD);
    val[i] = (uint32_t)i;
}

template <typename T>
__global__ __launch_bounds__(EW) void gather_kernel(const T *x, const T *y, const T *z,
                                                    const uint32_t *order, int64_t p, T *xs, T *ys,
                                                    T *zs)
{
    const int64_t j = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (j >= p)
        return;
    const uint32_t i = order[j];
    xs[j] = x[i];
    ys[j] = y[i];
    zs[j] = z[i];
}

// start[k] = number of sorted keys below k, for k = 0..nleaves.
__global__ __launch_bounds__(EW) void leaf_bounds_kernel(const uint32_t *ks, int64_t p,
                                                         int64_t nleaves, int32_t *start)
{
    const int64_t k = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (k > nleaves)
        return;
    int64_t lo = 0, hi = p;   // first index with ks[index] >= k
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)ks[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    start[k] = (int32_t)lo;
}

// Near-field target chunks of the cells of one level: chunks[k] = ceil(count_k
// / tpb) for the cells k < ncells whose samples are targets of this near field,
// else 0; chunks[ncells] = 0.  Cell k owns [start[stride k], start[stride
// (k+1)]).  It is a target cell when (a null or a[k >> 3] set: its parent is
// refined) and (b null or b[k] clear: it is not refined itself).
__global__ __launch_bounds__(EW) void leaf_chunks_kernel(const int32_t *start, int64_t ncells,
                                                         int64_t stride, int tpb, const int32_t *a,
                                                         const int32_t *b, int32_t *chunks)
{
    const int64_t k = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (k > ncells)
        return;
    int32_t c = 0;
    if (k < ncells && (!a || a[k >> 3]) && (!b || !b[k]))
        c = (start[stride * (k + 1)] - start[stride * k] + tpb - 1) / tpb;
    chunks[k] = c;
}

// Samples in the 27 cells around cell (x, y, z) of level D + q, and their count.
__device__ inline int64_t around_count(const int32_t *start, int64_t x, int64_t y, int64_t z, int q,
                                       int64_t sD, int64_t stride)
{
    const int64_t N = sD << q;
    int64_t a = 0;
    for (int64_t zz = z - 1; zz <= z + 1; ++zz)
        for (int64_t yy = y - 1; yy <= y + 1; ++yy)
            for (int64_t xx = x - 1; xx <= x + 1; ++xx) {
                if (xx < 0 || xx >= N || yy < 0 || yy >= N || zz < 0 || zz >= N)
                    continue;
                const int64_t kk = comp_index(xx, yy, zz, q, sD);
                a += (int64_t)start[stride * (kk + 1)] - start[stride * kk];
            }
    return a;
}

// Refinement of the cells of level D + q (adaptive tree; samples keyed R levels
// below the leaves; q < R).  A cell (whose parent is refined, for q > 0) is
// refined when the direct pairs its targets save by taking their near field
// over the 27 cells one level down around each child instead of the 27 cells
// around it exceed the threshold, a price for the children's interactions in
// units of pairs.  Counts are exact integers.
__global__ __launch_bounds__(EW) void refine_kernel(const int32_t *start, int q, int R, int64_t sD,
                                                    int64_t threshold, const int32_t *parent,
                                                    int32_t *refined)
{
    const int64_t N = sD << q, k = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (k >= N * N * N)
        return;
    int64_t s1 = 1;                  // start stride of the children's level
    for (int r = q + 1; r < R; ++r)
        s1 *= 8;
    const int64_t s0 = 8 * s1;       // start stride of this level
    const int64_t n = (int64_t)start[s0 * (k + 1)] - start[s0 * k];
    int32_t r = 0;
    if (n > 0 && (!parent || parent[k >> 3])) {
        int64_t x, y, z;
        comp_coords(k, q, sD, x, y, z);
        const int64_t coarse = n * around_count(start, x, y, z, q, sD, s0);
        int64_t fine = 0;
        for (int ch = 0; ch < 8; ++ch) {
            const int64_t kc = 8 * k + ch;
            const int64_t nc = (int64_t)start[s1 * (kc + 1)] - start[s1 * kc];
            if (nc == 0)
                continue;
            fine += nc * around_count(start, 2 * x + (ch & 1), 2 * y + ((ch >> 1) & 1),
                                      2 * z + (ch >> 2), q + 1, sD, s1);
        }
        r = coarse - fine > threshold ? 1 : 0;
    }
    refined[k] = r;
}

__global__ __launch_bounds__(EW) void fill_kernel(double *a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (i < n)
        a[i] = 0.0;
}

__global__ __launch_bounds__(EW) void fill_int_kernel(int32_t *a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (i < n)
        a[i] = 0;
}

// ------------------------------------------------------------------ tree geometry
struct Level {
    int64_t side;   // cells per axis, 2^l
    int64_t P;      // padded class side, side/2 + 4
    double *W;      // [8][P^3][n^3]
    double *L;      // [8][P^3][4 n^3]
    int32_t *occ;   // [8][P^3]: 1 if the cell holds samples (padding 0)
    int32_t *tmask; // [8][P^3]: 1 if the cell's local expansion is used (occ, or
                    // at the refined level, occ and a refined parent)
    // Refined level only (else null): the tmask cells of each class as a list
    // of padded indices, class ct's at [tscan[ct Q^3], tscan[(ct+1) Q^3]).
    const int32_t *tlist;
    const int32_t *tscan;
};

__device__ inline int64_t class_of(int64_t ix, int64_t iy, int64_t iz)
{
    return (ix & 1) + 2 * ((iy & 1) + 2 * (iz & 1));
}

__device__ inline int64_t padded(int64_t ix, int64_t iy, int64_t iz, int64_t P)
{
    return ((ix >> 1) + 2) + P * (((iy >> 1) + 2) + P * ((iz >> 1) + 2));
}

__device__ inline int64_t slot(int64_t ix, int64_t iy, int64_t iz, int64_t P)
{
    return class_of(ix, iy, iz) * P * P * P + padded(ix, iy, iz, P);
}

// ------------------------------------------------------------------ P2M
// One block per leaf.  Batches of EW samples first evaluate their 3 N
// one-dimensional interpolation polynomials (one sample per thread, into LDS);
// then thread m adds S_mx(x_j) S_my(y_j) S_mz(z_j) over the batch, so each
// node's weight is summed over the leaf's samples in sorted order.
template <int N, typename T>
__global__ __launch_bounds__(EW) void p2m_kernel(const T *xs, const T *ys, const T *zs,
                                                 const int32_t *start, const double *box,
                                                 int R, int64_t sD, Level lev, Cheb ch)
{
    constexpr int N3 = N * N * N;
    static_assert(N3 <= EW, "one thread per node");
    __shared__ double S[EW][3 * N];
    const int64_t leaf = blockIdx.x;
    const int32_t j0 = start[leaf], j1 = start[leaf + 1];
    if (j0 == j1)
        return;
    int64_t ix, iy, iz;
    comp_coords(leaf, R, sD, ix, iy, iz);
    const double Rb = box[3];
    const double h = 2.0 * Rb / (double)(sD << R), hh = 0.5 * h;
    const double cx = box[0] - Rb + ((double)ix + 0.5) * h;
    const double cy = box[1] - Rb + ((double)iy + 0.5) * h;
    const double cz = box[2] - Rb + ((double)iz + 0.5) * h;
    double *w = lev.W + slot(ix, iy, iz, lev.P) * N3;
    if (threadIdx.x == 0)
        lev.occ[slot(ix, iy, iz, lev.P)] = 1;
    const int m = threadIdx.x;
    const int mx = m % N, my = (m / N) % N, mz = m / (N * N);
    double a = 0.0;
    for (int32_t b = j0; b < j1; b += EW) {
        const int32_t j = b + (int32_t)threadIdx.x;
        if (j < j1) {
            double sv[N];
            cheb_s<N>(ch, ((double)xs[j] - cx) / hh, sv);
#pragma unroll
            for (int k = 0; k < N; ++k)
                S[threadIdx.x][k] = sv[k];
            cheb_s<N>(ch, ((double)ys[j] - cy) / hh, sv);
#pragma unroll
            for (int k = 0; k < N; ++k)
                S[threadIdx.x][N + k] = sv[k];
            cheb_s<N>(ch, ((double)zs[j] - cz) / hh, sv);
#pragma unroll
            for (int k = 0; k < N; ++k)
                S[threadIdx.x][2 * N + k] = sv[k];
        }
        __syncthreads();
        const int cnt = j1 - b < EW ? (int)(j1 - b) : EW;
        if (m < N3)
            for (int q = 0; q < cnt; ++q)
                a += S[q][mx] * S[q][N + my] * S[q][2 * N + mz];
        __syncthreads();
    }
    if (m < N3)
        w[m] = a;
}

// Target mask of a refined level (D + q, q >= 1): occupied cells whose parent
// (composite index at level D + q - 1) is refined.
__global__ __launch_bounds__(EW) void tmask_kernel(Level lev, const int32_t *refined, int q,
                                                   int64_t sD)
{
    const int64_t side = lev.side, k = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (k >= side * side * side)
        return;
    const int64_t ix = k % side, iy = (k / side) % side, iz = k / (side * side);
    const int64_t sl = slot(ix, iy, iz, lev.P);
    const int64_t par = comp_index(ix >> 1, iy >> 1, iz >> 1, q - 1, sD);
    lev.tmask[sl] = lev.occ[sl] && refined[par] ? 1 : 0;
}

// flag[ct Q^3 + c] = tmask of class ct's cell c (sub-grid order, x fastest).
__global__ __launch_bounds__(EW) void tflag_kernel(Level lev, int32_t *flag)
{
    const int64_t Q = lev.side / 2, Q3 = Q * Q * Q, e = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (e >= 8 * Q3)
        return;
    const int64_t ct = e / Q3, c = e % Q3, P = lev.P;
    const int64_t ux = c % Q, uy = (c / Q) % Q, uz = c / (Q * Q);
    flag[e] = lev.tmask[ct * P * P * P + (ux + 2) + P * ((uy + 2) + P * (uz + 2))];
}

// list[scan[e]] = padded index of cell e for every flagged cell.
__global__ __launch_bounds__(EW) void tlist_kernel(Level lev, const int32_t *flag,
                                                   const int32_t *scan, int32_t *list)
{
    const int64_t Q = lev.side / 2, Q3 = Q * Q * Q, e = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (e >= 8 * Q3 || !flag[e])
        return;
    const int64_t c = e % Q3, P = lev.P;
    const int64_t ux = c % Q, uy = (c / Q) % Q, uz = c / (Q * Q);
    list[scan[e]] = (int32_t)((ux + 2) + P * ((uy + 2) + P * (uz + 2)));
}

// T[pos][m][l] = prod_a S_{m_a}(u_a), u = child node l in the parent's frame.
template <int N>
__global__ __launch_bounds__(EW) void transfer_kernel(Cheb ch, double *Tm)
{
    constexpr int N3 = N * N * N;
    const int64_t e = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (e >= 8 * N3 * N3)
        return;
    const int pos = (int)(e / (N3 * N3));
    const int m = (int)((e / N3) % N3), l = (int)(e % N3);
    const int mi[3] = {m % N, (m / N) % N, m / (N * N)};
    const int li[3] = {l % N, (l / N) % N, l / (N * N)};
    double v = 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double u = (-0.5 + (double)((pos >> a) & 1)) + 0.5 * ch.tbar[li[a]];
        v *= cheb_s1<N>(ch, mi[a], u);
    }
    Tm[e] = v;
}

// ------------------------------------------------------------------ M2L tables
// The M2L kernels run on the FP64 matrix cores.  The table of level l holds,
// for every offset o, A_o^T: At[o][k][row] = K_c(x_m - y_k), row = c*n^3 + m,
// with target nodes hl*tbar_m (relative to the target centre) and source nodes
// o*h + hl*tbar_k; rows are padded with zeros to a multiple of the row tile and
// k to a multiple of the k tile, so tile loads need no bounds tests.
#ifndef SPK_M2L_TN
#define SPK_M2L_TN 64
#endif
#ifndef SPK_M2L_TK
#define SPK_M2L_TK 8     // 216 = 27 x 8: no k padding at order 6
#endif
constexpr int TM = 128, TN = SPK_M2L_TN, TK = SPK_M2L_TK;
constexpr int kM2lThreads = 256, kXcds = 8, kOffsets = 343, kMaxList = 189;
static_assert(TN == 64 || TN == 128, "column tile");
static_assert(TK % 4 == 0 && (TK * TM) % (2 * kM2lThreads) == 0 &&
              (TK * TN) % kM2lThreads == 0, "k tile");

template <int N>
struct M2lShape {
    static constexpr int N3 = N * N * N, ROWS = 4 * N3;
    static constexpr int RP = (ROWS + TM - 1) / TM * TM;  // padded rows
    static constexpr int KP = (N3 + TK - 1) / TK * TK;    // padded k
    static constexpr int KT = KP / TK;                    // k tiles per offset
};

template <int N, int KERN>
__global__ __launch_bounds__(EW) void m2l_table_kernel(const double *box, int level, double eps,
                                                       Cheb ch, double *At)
{
    using S = M2lShape<N>;
    constexpr int N3 = S::N3;
    const int64_t e = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (e >= (int64_t)kOffsets * S::KP * S::RP)
        return;
    const int64_t o = e / ((int64_t)S::KP * S::RP);
    const int l = (int)((e / S::RP) % S::KP), row = (int)(e % S::RP);
    if (row >= S::ROWS || l >= N3) {
        At[e] = 0.0;
        return;
    }
    const int c = row / N3, m = row % N3;
    const int ov[3] = {(int)(o % 7) - 3, (int)((o / 7) % 7) - 3, (int)(o / 49) - 3};
    const int mi[3] = {m % N, (m / N) % N, m / (N * N)};
    const int li[3] = {l % N, (l / N) % N, l / (N * N)};
    const double h = 2.0 * box[3] / (double)(int64_t(1) << level), hl = 0.5 * h;
    double d[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        d[a] = hl * ch.tbar[mi[a]] - ((double)ov[a] * h + hl * ch.tbar[li[a]]);
    const double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
    double v;
    if (KERN == kKernelLog)
        v = c < 3 ? d[c] / s : 0.5 * log(s);
    else
        v = c < 3 ? (s > 0.0 ? d[c] / sqrt(s) : 0.0) : sqrt(s);
    At[e] = v;
}

// Offset o (|o_a| <= 3, linear index o = (ox+3) + 7(oy+3) + 49(oz+3)) is in the
// interaction list of target class ct when it is not a neighbour and the
// source's parent is a neighbour of the target's parent.
__device__ inline bool in_list(int o, int ct)
{
    const int ov[3] = {o % 7 - 3, (o / 7) % 7 - 3, o / 49 - 3};
    bool near = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int v = ov[a];
        if (v < -1 || v > 1)
            near = false;
        const bool odd = (ct >> a) & 1;
        if (!odd && (v < -2 || v > 3))
            return false;
        if (odd && (v < -3 || v > 2))
            return false;
    }
    return !near;
}

// Source class and padded-index shift of offset o seen from target class ct.
__device__ inline void offset_shift(int o, int ct, int64_t P, int &cs, int64_t &shift)
{
    const int ov[3] = {o % 7 - 3, (o / 7) % 7 - 3, o / 49 - 3};
    cs = 0;
    shift = 0;
    int64_t mul = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int ca = (ct >> a) & 1;
        const int sa = (ca + ov[a]) & 1;
        cs |= sa << a;
        shift += (int64_t)((ca + ov[a] - sa) / 2) * mul;
        mul *= P;
    }
}

// ------------------------------------------------------------------ M2L (GEMM)
// Block (row tile, column tile, class ct): rows are (component, node) pairs,
// columns the class's cells (Q^3 of them, Q = side/2) in sub-grid order, or,
// at a refined level, the class's listed target cells.  For every offset of
// the interaction list (or of one contiguous part of it, at levels with few
// tiles), in increasing order, the block adds
// A_o[rows][k] W[source][k] with v_mfma_f64_16x16x4 into accumulators held
// by its four waves (wave w: rows 64 (w & 1) .., columns (TN/2)(w >> 1) ..),
// and writes the tile once (a part writes a partial tile, which
// m2l_reduce_kernel adds up in part order).  Tiles of TK k-values go through
// two LDS buffers:
// the next tile is read from global memory into registers while the matrix
// cores work on the current one.  Tiles without an occupied target cell are
// skipped (nothing reads the local expansion of an empty cell), and so are
// offsets whose TN source cells are all empty (their weights are exact zeros).
// One launch covers every level (level 2's tiles first): the levels' M2L
// steps are independent, and the few blocks of the coarse levels then run
// beside the many of the finest.  Hardware block b runs on XCD b % 8; block
// b = 8k + x takes column tile T = 8 floor(k / row_tiles) + x and row tile
// k % row_tiles, so the row tiles of one column tile share an XCD (and its L2
// copy of the column tile's weights) while consecutive column tiles, which
// hold the work when it is concentrated, spread over all XCDs.
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

constexpr int kMaxLevels = kFmmMaxDepth - 1;  // levels 2..depth
struct M2lPlan {
    Level lev[kMaxLevels];
    const double *At[kMaxLevels];  // table of each level
    int64_t ntc[kMaxLevels];       // column tiles per class of each level
    int64_t first[kMaxLevels];     // first tile (all classes and parts) of each level
    int nsplit[kMaxLevels];        // parts of each tile's interaction list
    int64_t pfirst[kMaxLevels];    // first partial tile of each level (nsplit > 1)
    double *part;                  // partial tiles, TM x TN each
    int nlev, ntr;                 // levels, row tiles
    int64_t ntiles;                // tiles of all levels, classes and parts
};

// Parts of every tile's interaction list at a level with `blocks` tile
// blocks: levels with few tiles (the coarse ones) split their lists so that
// the long chain of one tile's offsets runs on several blocks.
inline int m2l_split(int64_t blocks)
{
    int s = 1;
    while (s < 8 && blocks * s * 2 <= 1024)
        s *= 2;
    return s;
}

// Columns of tile (class ct, column tile cti) of a level: colpad (padded
// index of the target cell, -1 for none), colsrc (its weights' offset) and
// outidx (its expansion's offset).  Returns 1 when this thread's column holds
// a target cell.  Threads t < TN only.
template <int N3, int ROWS>
__device__ inline int tile_column(const Level &lev, int ct, int64_t cti, int t, int64_t *colpad,
                                  int64_t *colsrc, int64_t *outidx)
{
    const int64_t P = lev.P, P3 = P * P * P, Q = lev.side / 2, Q3 = Q * Q * Q;
    const int64_t c0 = cti * TN;
    int64_t pc = -1;
    int mine = 0;
    if (lev.tlist) {          // columns from the class's list of target cells
        const int64_t c = lev.tscan[ct * Q3] + c0 + t;
        if (c < lev.tscan[(ct + 1) * Q3]) {
            pc = lev.tlist[c];
            mine = 1;
        }
    } else {
        const int64_t c = c0 + t;
        if (c < Q3) {
            const int64_t ux = c % Q, uy = (c / Q) % Q, uz = c / (Q * Q);
            pc = (ux + 2) + P * ((uy + 2) + P * (uz + 2));
            mine = lev.tmask[(int64_t)ct * P3 + pc];
        }
    }
    colpad[t] = pc;
    colsrc[t] = pc >= 0 ? pc * N3 : -1;
    outidx[t] = pc >= 0 ? ((int64_t)ct * P3 + pc) * ROWS : -1;
    return mine;
}

// The tile of a block in the plan: level i, class ct, column tile cti and
// part a of its interaction list.
__device__ inline int plan_tile(const M2lPlan &plan, int64_t tile, Level &lev, const double *&At,
                                int64_t &cti, int &ct, int &a, int &nsplit, int64_t &pbase)
{
    int li = 0;
#pragma unroll
    for (int i = 1; i < kMaxLevels; ++i)
        if (i < plan.nlev && tile >= plan.first[i])
            li = i;
    // a select, not an index, keeps the plan in SGPRs
    lev = plan.lev[0];
    At = plan.At[0];
    int64_t ntc = plan.ntc[0], first = 0, pfirst = plan.pfirst[0];
    nsplit = plan.nsplit[0];
#pragma unroll
    for (int i = 1; i < kMaxLevels; ++i)
        if (i == li) {
            lev = plan.lev[i];
            At = plan.At[i];
            ntc = plan.ntc[i];
            first = plan.first[i];
            nsplit = plan.nsplit[i];
            pfirst = plan.pfirst[i];
        }
    const int64_t local = tile - first, base = local / nsplit;
    a = (int)(local % nsplit);
    cti = base % ntc;
    ct = (int)(base / ntc);
    pbase = pfirst + base * plan.ntr * nsplit;   // + rt * nsplit + a
    return li;
}

// The matrix-core loop shared by M2L, M2M and L2L: acc += sum over the nlist
// entries a and the k tiles of A_a[rows][k] B_a[k][columns].  A_a is stored
// k-major with row stride RP and padded with zeros to KP values of k;
// abase(a) points at its row row0 for k = 0.  Column cl of B_a holds
// bbase(a)[colsrc[cl] + k] for k < KV (colsrc < 0: a zero column).  Tiles of
// TK k-values go through two LDS buffers; the next tile is read into
// registers while the matrix cores work on the current one.  Wave w holds
// rows 64 (w & 1) .. and columns (TN/2)(w >> 1) .. of the block's tile.
template <int RP, int KP, int KV, typename AFn, typename BFn>
__device__ inline void mfma_gemm(int nlist, AFn abase, BFn bbase, const int64_t *colsrc,
                                 double (*As)[TK][TM], double (*Bs)[TK][TN + 1],
                                 dbl4 (&acc)[4][TN / 32])
{
    constexpr int KT = KP / TK, FM = 4, FN = TN / 32;
    constexpr int LA = TK * TM / (2 * kM2lThreads), LB = TK * TN / kM2lThreads;
    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    const int nit = nlist * KT;
    dbl2 ra[LA];
    double rb[LB];
    auto load = [&](int it) {
        const int a = it / KT, kt = it % KT;
        const double *Ao = abase(a) + (int64_t)kt * TK * RP;
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int e = t + kM2lThreads * i, k = e / (TM / 2), r = 2 * (e % (TM / 2));
            ra[i] = *reinterpret_cast<const dbl2 *>(Ao + (int64_t)k * RP + r);
        }
        const double *Bc = bbase(a);
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int e = t + kM2lThreads * i, k = e % TK, cl = e / TK;
            const int kk = kt * TK + k;
            const int64_t cs = colsrc[cl];
            rb[i] = (cs >= 0 && kk < KV) ? Bc[cs + kk] : 0.0;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int e = t + kM2lThreads * i, k = e / (TM / 2), r = 2 * (e % (TM / 2));
            *reinterpret_cast<dbl2 *>(&As[buf][k][r]) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int e = t + kM2lThreads * i, k = e % TK, cl = e / TK;
            Bs[buf][k][cl] = rb[i];
        }
    };
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
            acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int wr = (wave & 1) * 64, wc = (wave >> 1) * (TN / 2);
    const int fr = lane % 16, fk = lane / 16;
    if (nit > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int it = 0; it < nit; ++it) {
        const int buf = it & 1;
        if (it + 1 < nit)
            load(it + 1);
#pragma unroll
        for (int k0 = 0; k0 < TK; k0 += 4) {
            double a[FM], bb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[i] = As[buf][k0 + fk][wr + 16 * i + fr];
#pragma unroll
            for (int j = 0; j < FN; ++j)
                bb[j] = Bs[buf][k0 + fk][wc + 16 * j + fr];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bb[j], acc[i][j], 0,
                                                                     0, 0);
        }
        if (it + 1 < nit)
            store(buf ^ 1);
        __syncthreads();
    }
}

// Writes the accumulators: out[outidx[column] + row] (= or +=) for rows below
// nrows and columns with outidx >= 0.  Register r of a lane of
// v_mfma_f64_16x16x4 holds row lane/16 + 4r of column lane % 16.
template <bool ADD>
__device__ inline void mfma_store(const dbl4 (&acc)[4][TN / 32], const int64_t *outidx, int row0,
                                  int nrows, double *out)
{
    constexpr int FM = 4, FN = TN / 32;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wr = (wave & 1) * 64, wc = (wave >> 1) * (TN / 2);
    const int fr = lane % 16, fk = lane / 16;
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int64_t o = outidx[wc + 16 * j + fr];
        if (o < 0)
            continue;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + wr + 16 * i + fk + 4 * r;
                if (row < nrows) {
                    if (ADD)
                        out[o + row] += acc[i][j][r];
                    else
                        out[o + row] = acc[i][j][r];
                }
            }
    }
}

// Tile of a block: hardware block b runs on XCD b % 8; block b = 8k + x takes
// column tile 8 floor(k / ntr) + x and row tile k % ntr.
__device__ inline int64_t block_tile(int ntr, int &rt)
{
    const int64_t b = blockIdx.x, kb = b / kXcds;
    rt = (int)(kb % ntr);
    return kXcds * (kb / ntr) + b % kXcds;
}

template <int N>
__global__ __launch_bounds__(kM2lThreads) void m2l_kernel(M2lPlan plan)
{
    using S = M2lShape<N>;
    constexpr int N3 = S::N3, ROWS = S::ROWS, RP = S::RP, KP = S::KP;
    __shared__ __align__(16) double As[2][TK][TM];
    __shared__ __align__(16) double Bs[2][TK][TN + 1];
    __shared__ int64_t colpad[TN], colsrc[TN], outidx[TN];
    __shared__ int64_t list_shift[kMaxList];
    __shared__ int16_t list_o[kMaxList];
    __shared__ int8_t list_cs[kMaxList];
    __shared__ int8_t flag[kOffsets];
    __shared__ int nlist;

    int rt;
    const int64_t tile = block_tile(plan.ntr, rt);
    if (tile >= plan.ntiles)
        return;
    Level lev;
    const double *At;
    int64_t cti, pbase;
    int ct, part, nsplit;
    plan_tile(plan, tile, lev, At, cti, ct, part, nsplit, pbase);
    const int64_t P = lev.P, P3 = P * P * P;
    const int row0 = rt * TM;
    const int t = threadIdx.x, lane = t % 64, wave = t / 64;
    int mine = 0;
    if (t < TN)
        mine = tile_column<N3, ROWS>(lev, ct, cti, t, colpad, colsrc, outidx);
    if (!__syncthreads_or(mine))
        return;

    // interaction list of this tile: offsets with an occupied source cell
    for (int o = wave; o < kOffsets; o += kM2lThreads / 64) {
        int any = 0;
        if (in_list(o, ct)) {
            int cs;
            int64_t shift;
            offset_shift(o, ct, P, cs, shift);
            const int32_t *occ_s = lev.occ + (int64_t)cs * P3 + shift;
            int v = 0;
            for (int c = lane; c < TN; c += 64)
                if (colpad[c] >= 0 && occ_s[colpad[c]])
                    v = 1;
            any = __ballot(v) != 0;
        }
        if (lane == 0)
            flag[o] = (int8_t)any;
    }
    __syncthreads();
    if (wave == 0) {
        int base = 0;
        for (int o0 = 0; o0 < kOffsets; o0 += 64) {
            const int o = o0 + lane;
            const int f = o < kOffsets && flag[o];
            const unsigned long long mask = __ballot(f);
            if (f) {
                const int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
                int cs;
                int64_t shift;
                offset_shift(o, ct, P, cs, shift);
                list_o[pos] = (int16_t)o;
                list_cs[pos] = (int8_t)cs;
                list_shift[pos] = shift;
            }
            base += __popcll(mask);
        }
        if (lane == 0)
            nlist = base;
    }
    __syncthreads();
    // this part's share of the interaction list (no offset at all: zeros)
    const int lo = part * nlist / nsplit, hi = (part + 1) * nlist / nsplit;
    dbl4 acc[4][TN / 32];
    const double *W = lev.W;
    mfma_gemm<RP, KP, N3>(
        hi - lo, [&](int a) { return At + (int64_t)list_o[lo + a] * KP * RP + row0; },
        [&](int a) { return W + ((int64_t)list_cs[lo + a] * P3 + list_shift[lo + a]) * N3; },
        colsrc, As, Bs, acc);
    if (nsplit == 1) {
        mfma_store<false>(acc, outidx, row0, ROWS, lev.L);
        return;
    }
    // partial tile [column][row] (TM rows), summed into the expansions by
    // m2l_reduce_kernel
    __syncthreads();
    if (t < TN)
        outidx[t] = (int64_t)t * TM;
    __syncthreads();
    mfma_store<false>(acc, outidx, 0, TM, plan.part + (pbase + (int64_t)rt * nsplit + part) * TM * TN);
}

// Sums the partial tiles of split levels in part order into the expansions.
template <int N>
__global__ __launch_bounds__(kM2lThreads) void m2l_reduce_kernel(M2lPlan plan, int li)
{
    using S = M2lShape<N>;
    constexpr int N3 = S::N3, ROWS = S::ROWS;
    __shared__ int64_t colpad[TN], colsrc[TN], outidx[TN];
    Level lev = plan.lev[0];
    int64_t ntc = plan.ntc[0], pfirst = plan.pfirst[0];
    int nsplit = plan.nsplit[0];
    for (int i = 1; i < kMaxLevels; ++i)
        if (i == li) {
            lev = plan.lev[i];
            ntc = plan.ntc[i];
            pfirst = plan.pfirst[i];
            nsplit = plan.nsplit[i];
        }
    const int64_t b = blockIdx.x, base = b / plan.ntr;
    const int rt = (int)(b % plan.ntr);
    const int64_t cti = base % ntc;
    const int ct = (int)(base / ntc);
    const int t = threadIdx.x;
    int mine = 0;
    if (t < TN)
        mine = tile_column<N3, ROWS>(lev, ct, cti, t, colpad, colsrc, outidx);
    if (!__syncthreads_or(mine))
        return;                      // the M2L skipped this tile as well
    const double *pp = plan.part + (pfirst + (base * plan.ntr + rt) * nsplit) * TM * TN;
    for (int e = t; e < TM * TN; e += kM2lThreads) {
        const int col = e / TM, row = e % TM;
        const int64_t o = outidx[col];
        if (o < 0 || rt * TM + row >= ROWS)
            continue;
        double v = 0.0;
        for (int a = 0; a < nsplit; ++a)
            v += pp[(int64_t)a * TM * TN + e];
        lev.L[o + rt * TM + row] = v;
    }
}

// ------------------------------------------------------------------ M2M, L2L on the matrix cores
// Both translations are products with the 8 transfer matrices T[pos][m][l]
// (child position pos, parent node m, child node l):
//   M2M  W_parent[m] = sum_pos sum_l T[pos][m][l] W_child(pos)[l]
//   L2L  L_child[c][l] += sum_m T[pos][m][l] L_parent[c][m]
// Their tables, k-major and padded like the M2L tables:
//   Tu[pos][k = l][row = m] and Td[pos][k = m][row = l].
template <int N>
struct TransShape {
    static constexpr int N3 = N * N * N;
    static constexpr int RP = (N3 + TM - 1) / TM * TM;
    static constexpr int KP = (N3 + TK - 1) / TK * TK;
};

template <int N>
__global__ __launch_bounds__(EW) void transfer_tables_kernel(const double *Tm, double *Tu,
                                                             double *Td)
{
    using S = TransShape<N>;
    constexpr int N3 = S::N3;
    const int64_t e = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (e >= (int64_t)8 * S::KP * S::RP)
        return;
    const int pos = (int)(e / ((int64_t)S::KP * S::RP));
    const int k = (int)((e / S::RP) % S::KP), row = (int)(e % S::RP);
    const bool in = k < N3 && row < N3;
    Tu[e] = in ? Tm[((int64_t)pos * N3 + row) * N3 + k] : 0.0;
    Td[e] = in ? Tm[((int64_t)pos * N3 + k) * N3 + row] : 0.0;
}

// M2M of one level: block tiles of parent cells (class ct, sub-grid order) by
// parent nodes.  A parent's 8 children all sit at its own coordinates in the
// children's level sub-grids (class pos).  Marks occupied parents.
template <int N>
__global__ __launch_bounds__(kM2lThreads) void m2m_kernel(Level par, Level chd, const double *Tu,
                                                          int ntr, int64_t ntc)
{
    using S = TransShape<N>;
    constexpr int N3 = S::N3, RP = S::RP, KP = S::KP;
    __shared__ __align__(16) double As[2][TK][TM];
    __shared__ __align__(16) double Bs[2][TK][TN + 1];
    __shared__ int64_t colsrc[TN], outidx[TN];
    __shared__ int list_pos[8];
    __shared__ int nlist;
    int rt;
    const int64_t tile = block_tile(ntr, rt);
    if (tile >= 8 * ntc)
        return;
    const int64_t cti = tile % ntc;
    const int ct = (int)(tile / ntc);
    const int64_t P = par.P, P3 = P * P * P, Q = par.side / 2, Q3 = Q * Q * Q;
    const int64_t Pc = chd.P, Pc3 = Pc * Pc * Pc;
    const int t = threadIdx.x, lane = t % 64;
    const int row0 = rt * TM;
    int mine = 0;
    if (t < TN) {
        const int64_t c = cti * TN + t;
        int64_t src = -1, out = -1;
        if (c < Q3) {
            const int64_t ux = c % Q, uy = (c / Q) % Q, uz = c / (Q * Q);
            const int64_t ix = 2 * ux + (ct & 1), iy = 2 * uy + ((ct >> 1) & 1),
                          iz = 2 * uz + (ct >> 2);
            const int64_t cpad = (ix + 2) + Pc * ((iy + 2) + Pc * (iz + 2));
            for (int pos = 0; pos < 8; ++pos)
                mine |= chd.occ[pos * Pc3 + cpad];
            const int64_t pc = (ux + 2) + P * ((uy + 2) + P * (uz + 2));
            if (mine && rt == 0)
                par.occ[ct * P3 + pc] = 1;
            src = cpad * N3;
            out = ((int64_t)ct * P3 + pc) * N3;
        }
        colsrc[t] = src;
        outidx[t] = out;
    }
    if (!__syncthreads_or(mine))
        return;                      // the tile's weights stay zero
    if (t < 64) {
        int base = 0;
        for (int pos = 0; pos < 8; ++pos) {
            int v = 0;
            for (int c = lane; c < TN; c += 64)
                if (colsrc[c] >= 0 && chd.occ[pos * Pc3 + colsrc[c] / N3])
                    v = 1;
            if (__ballot(v) != 0) {
                if (lane == 0)
                    list_pos[base] = pos;
                ++base;
            }
        }
        if (lane == 0)
            nlist = base;
    }
    __syncthreads();
    dbl4 acc[4][TN / 32];
    const double *Wc = chd.W;
    mfma_gemm<RP, KP, N3>(
        nlist, [&](int a) { return Tu + (int64_t)list_pos[a] * KP * RP + row0; },
        [&](int a) { return Wc + (int64_t)list_pos[a] * Pc3 * N3; }, colsrc, As, Bs, acc);
    mfma_store<false>(acc, outidx, row0, N3, par.W);
}

// L2L into one level: block tiles of (child cell, component) columns, 4 per
// cell, of child class ct (the cells whose expansion is used, from the class's
// list where there is one) by child nodes.  A child at sub-grid coordinates u
// of class ct has its parent at coordinates u of the parents' level.
template <int N>
__global__ __launch_bounds__(kM2lThreads) void l2l_kernel(Level par, Level chd, const double *Td,
                                                          int ntr, int64_t ntc)
{
    using S = TransShape<N>;
    constexpr int N3 = S::N3, RP = S::RP, KP = S::KP;
    __shared__ __align__(16) double As[2][TK][TM];
    __shared__ __align__(16) double Bs[2][TK][TN + 1];
    __shared__ int64_t colsrc[TN], outidx[TN];
    int rt;
    const int64_t tile = block_tile(ntr, rt);
    if (tile >= 8 * ntc)
        return;
    const int64_t cti = tile % ntc;
    const int ct = (int)(tile / ntc);
    const int64_t P = chd.P, P3 = P * P * P, Q = chd.side / 2, Q3 = Q * Q * Q;
    const int64_t Pp = par.P;
    const int t = threadIdx.x;
    const int row0 = rt * TM;
    int mine = 0;
    if (t < TN) {
        const int64_t col = cti * TN + t, c = col / 4, comp = col % 4;
        int64_t pc = -1;
        if (chd.tlist) {
            const int64_t k = chd.tscan[ct * Q3] + c;
            if (k < chd.tscan[(ct + 1) * Q3])
                pc = chd.tlist[k];
        } else if (c < Q3) {
            const int64_t ux = c % Q, uy = (c / Q) % Q, uz = c / (Q * Q);
            pc = (ux + 2) + P * ((uy + 2) + P * (uz + 2));
            if (!chd.tmask[ct * P3 + pc])
                pc = -1;
        }
        int64_t src = -1, out = -1;
        if (pc >= 0) {
            mine = 1;
            const int64_t ux = pc % P - 2, uy = (pc / P) % P - 2, uz = pc / (P * P) - 2;
            src = slot(ux, uy, uz, Pp) * 4 * N3 + comp * N3;
            out = ((int64_t)ct * P3 + pc) * 4 * N3 + comp * N3;
        }
        colsrc[t] = src;
        outidx[t] = out;
    }
    if (!__syncthreads_or(mine))
        return;
    dbl4 acc[4][TN / 32];
    const double *Lp = par.L;
    mfma_gemm<RP, KP, N3>(
        1, [&](int) { return Td + (int64_t)ct * KP * RP + row0; }, [&](int) { return Lp; },
        colsrc, As, Bs, acc);
    mfma_store<true>(acc, outidx, row0, N3, chd.L);
}

// ------------------------------------------------------------------ L2P
// Sample j (sorted, key = composite index R levels below the leaves) evaluates
// the local expansion of its cell at its final level: the leaves' level, or
// one (two) levels down while its cells there are refined.
struct L2pLevels {
    Level lev[kMaxRefine + 1];          // levels D .. D + R
    const int32_t *refined[kMaxRefine]; // refine flags of levels D .. D + R - 1
    int R;
    int64_t sD;
};

template <int N, typename T>
__global__ __launch_bounds__(EW) void l2p_kernel(const T *xs, const T *ys, const T *zs,
                                                 const uint32_t *ks, const uint32_t *order,
                                                 int64_t p, const double *box, L2pLevels lv,
                                                 Cheb ch, int64_t t0, int64_t nt, bool energy,
                                                 double *acc, int64_t ld)
{
    constexpr int N3 = N * N * N;
    const int64_t j = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (j >= p)
        return;
    const int64_t i = (int64_t)order[j] - t0;
    if (i < 0 || i >= nt)
        return;
    const int64_t key = ks[j];
    int q = 0;
    if (lv.R > 0 && lv.refined[0][key >> (3 * lv.R)]) {
        q = 1;
        if (lv.R > 1 && lv.refined[1][key >> (3 * (lv.R - 1))])
            q = 2;
    }
    const Level L = q == 0 ? lv.lev[0] : (q == 1 ? lv.lev[1] : lv.lev[2]);
    int64_t ix, iy, iz;
    comp_coords(key >> (3 * (lv.R - q)), q, lv.sD, ix, iy, iz);
    const double R = box[3];
    const double h = 2.0 * R / (double)L.side, hh = 0.5 * h;
    double sx[N], sy[N], sz[N];
    cheb_s<N>(ch, ((double)xs[j] - (box[0] - R + ((double)ix + 0.5) * h)) / hh, sx);
    cheb_s<N>(ch, ((double)ys[j] - (box[1] - R + ((double)iy + 0.5) * h)) / hh, sy);
    cheb_s<N>(ch, ((double)zs[j] - (box[2] - R + ((double)iz + 0.5) * h)) / hh, sz);
    const double *lf = L.L + slot(ix, iy, iz, L.P) * 4 * N3;
    double f[4] = {0.0, 0.0, 0.0, 0.0};
    for (int mz = 0; mz < N; ++mz)
        for (int my = 0; my < N; ++my) {
            const double syz = sy[my] * sz[mz];
#pragma unroll
            for (int mx = 0; mx < N; ++mx) {
                const int m = mx + N * (my + N * mz);
                const double s = sx[mx] * syz;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    f[c] += lf[c * N3 + m] * s;
            }
        }
    acc[i] += f[0];
    acc[ld + i] += f[1];
    acc[2 * ld + i] += f[2];
    if (energy)
        acc[3 * ld + i] += f[3];
}

template <int N>
hipError_t run_order(const FmmLaunch &f, hipStream_t s);

}  // namespace

int64_t fmm_padded_side(int level) { return (int64_t(1) << level) / 2 + 4; }

size_t fmm_level_cells(int level)
{
    const int64_t P = fmm_padded_side(level);
    return (size_t)(8 * P * P * P);
}

template <int N>
size_t split_doubles(int F)
{
    constexpr int ntr = M2lShape<N>::RP / TM;
    size_t n = 0;
    for (int l = 2; l <= F; ++l) {
        const int64_t Q = (int64_t(1) << l) / 2, ntc = (Q * Q * Q + TN - 1) / TN;
        const int sp = m2l_split(8 * ntc * ntr);
        if (sp > 1)
            n += (size_t)8 * ntc * ntr * sp * TM * TN;
    }
    return n;
}

size_t fmm_split_doubles(int order, int F)
{
    switch (order) {
    case 3: return split_doubles<3>(F);
    case 4: return split_doubles<4>(F);
    case 5: return split_doubles<5>(F);
    case 6: return split_doubles<6>(F);
    default: return 0;
    }
}

size_t fmm_trans_doubles(int order)
{
    switch (order) {
    case 3: return (size_t)8 * TransShape<3>::KP * TransShape<3>::RP;
    case 4: return (size_t)8 * TransShape<4>::KP * TransShape<4>::RP;
    case 5: return (size_t)8 * TransShape<5>::KP * TransShape<5>::RP;
    case 6: return (size_t)8 * TransShape<6>::KP * TransShape<6>::RP;
    default: return 0;
    }
}

size_t fmm_table_doubles(int order)
{
    switch (order) {
    case 3: return (size_t)kOffsets * M2lShape<3>::KP * M2lShape<3>::RP;
    case 4: return (size_t)kOffsets * M2lShape<4>::KP * M2lShape<4>::RP;
    case 5: return (size_t)kOffsets * M2lShape<5>::KP * M2lShape<5>::RP;
    case 6: return (size_t)kOffsets * M2lShape<6>::KP * M2lShape<6>::RP;
    default: return 0;
    }
}

int64_t fmm_refine_threshold(int order)
{
    // 8 children x 189 interactions x 4 components x n^6 multiply-adds, at
    // about 1/7 of a direct pair each (FP64 matrix-core rate over pair rate)
    int64_t n6 = 1;
    for (int i = 0; i < 6; ++i)
        n6 *= order;
    return 8 * 189 * 4 * n6 / 7;
}

size_t fmm_sort_temp_bytes(int64_t p, int depth)
{
    const int64_t nleaves = int64_t(1) << (3 * depth);
    size_t a = 0, b = 0;
    // a failed query leaves 0; the sort or scan then reports the short buffer
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const uint32_t *)nullptr,
                                           (uint32_t *)nullptr, (const uint32_t *)nullptr,
                                           (uint32_t *)nullptr, (int)p, 0,
                                           3 * depth) != hipSuccess)
        a = 0;
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, b, (const int32_t *)nullptr, (int32_t *)nullptr,
                                         (int)(nleaves + 1)) != hipSuccess)
        b = 0;
    return a > b ? a : b;
}

namespace {

Cheb make_cheb(int n)
{
    Cheb ch{};
    ch.n = n;
    for (int k = 0; k < n; ++k) {
        const double th = (2.0 * k + 1.0) * 3.14159265358979323846 / (2.0 * n);
        ch.tbar[k] = std::cos(th);
        for (int i = 0; i < n; ++i)
            ch.tb[i][k] = std::cos(i * th);
    }
    return ch;
}

// 1: the near field runs on a second stream beside the interactions (0: on
// the caller's stream, in order).
#ifndef SPK_FMM_OVERLAP
#define SPK_FMM_OVERLAP 1
#endif

template <int N, typename T>
hipError_t run_typed(const FmmLaunch &f, hipStream_t s)
{
    constexpr int N3 = N * N * N;
    const T *x = static_cast<const T *>(f.x), *y = static_cast<const T *>(f.y),
            *z = static_cast<const T *>(f.z);
    T *xs = static_cast<T *>(f.xs), *ys = static_cast<T *>(f.ys), *zs = static_cast<T *>(f.zs);
    const int D = f.depth, R = f.adaptive, F = D + R;
    const int64_t p = f.p, sD = int64_t(1) << D;
    auto ncells_at = [&](int q) { return int64_t(1) << (3 * (D + q)); };
    auto stride_at = [&](int q) { return int64_t(1) << (3 * (R - q)); };
    const int64_t ncellsF = ncells_at(R);
    const Cheb ch = make_cheb(N);
    hipError_t e;
    // root box
    const int nb = (int)std::min<int64_t>(kFmmBoxBlocks, (p + EW - 1) / EW);
    hipLaunchKernelGGL(box_stage1<T>, dim3(nb), dim3(EW), 0, s, x, y, z, p, f.box_part);
    hipLaunchKernelGGL(box_stage2, dim3(1), dim3(64), 0, s, f.box_part, nb, f.box);
    // cell keys at the deepest level, stable sort, sorted coordinates, cell ranges
    hipLaunchKernelGGL(leaf_keys_kernel<T>, dim3(ew_blocks(p)), dim3(EW), 0, s, x, y, z, p, f.box,
                       R, sD, f.keys_in, f.vals_in);
    size_t tb = f.temp_bytes;
    if ((e = hipcub::DeviceRadixSort::SortPairs(f.temp, tb, f.keys_in, f.keys_out, f.vals_in,
                                                f.vals_out, (int)p, 0, 3 * F, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(gather_kernel<T>, dim3(ew_blocks(p)), dim3(EW), 0, s, x, y, z, f.vals_out,
                       p, xs, ys, zs);
    hipLaunchKernelGGL(leaf_bounds_kernel, dim3(ew_blocks(ncellsF + 1)), dim3(EW), 0, s,
                       f.keys_out, p, ncellsF, f.start);
    // refinement, level by level, and the near-field target chunks of every level
    for (int q = 0; q < R; ++q)
        hipLaunchKernelGGL(refine_kernel, dim3(ew_blocks(ncells_at(q))), dim3(EW), 0, s, f.start,
                           q, R, sD, fmm_refine_threshold(N), q > 0 ? f.refined[q - 1] : nullptr,
                           f.refined[q]);
    for (int q = 0; q <= R; ++q) {
        const int64_t nc = ncells_at(q);
        hipLaunchKernelGGL(leaf_chunks_kernel, dim3(ew_blocks(nc + 1)), dim3(EW), 0, s, f.start,
                           nc, stride_at(q), f.near_tpb, q > 0 ? f.refined[q - 1] : nullptr,
                           q < R ? f.refined[q] : nullptr, f.chunks[q]);
        tb = f.temp_bytes;
        if ((e = hipcub::DeviceScan::ExclusiveSum(f.temp, tb, f.chunks[q], f.chunk_start[q],
                                                  (int)(nc + 1), s)) != hipSuccess)
            return e;
    }
    // multipole weights: zero (padding included), the deepest level, then upward
    Level lev[kFmmMaxDepth + 1];
    for (int l = 2; l <= F; ++l) {
        lev[l].side = int64_t(1) << l;
        lev[l].P = fmm_padded_side(l);
        lev[l].W = f.W[l];
        lev[l].L = f.L[l];
        lev[l].occ = f.occ[l];
        lev[l].tmask = l > D ? f.tmask[l - D] : f.occ[l];
        lev[l].tlist = nullptr;
        lev[l].tscan = nullptr;
        const int64_t nw = (int64_t)fmm_level_cells(l) * N3;
        hipLaunchKernelGGL(fill_kernel, dim3(ew_blocks(nw)), dim3(EW), 0, s, lev[l].W, nw);
        const int64_t no = (int64_t)fmm_level_cells(l);
        hipLaunchKernelGGL(fill_int_kernel, dim3(ew_blocks(no)), dim3(EW), 0, s, lev[l].occ, no);
        if (lev[l].tmask != lev[l].occ)
            hipLaunchKernelGGL(fill_int_kernel, dim3(ew_blocks(no)), dim3(EW), 0, s,
                               lev[l].tmask, no);
    }
    hipLaunchKernelGGL(transfer_kernel<N>, dim3(ew_blocks(8 * N3 * N3)), dim3(EW), 0, s, ch, f.Tm);
    using TS = TransShape<N>;
    const int64_t ntt = (int64_t)8 * TS::KP * TS::RP;
    hipLaunchKernelGGL(transfer_tables_kernel<N>, dim3(ew_blocks(ntt)), dim3(EW), 0, s, f.Tm, f.Tu,
                       f.Td);
    const int ntr_t = TS::RP / TM;
    auto trans_blocks = [&](int64_t ntc) {
        return (unsigned)((8 * ntc + kXcds - 1) / kXcds * kXcds * ntr_t);
    };
    hipLaunchKernelGGL((p2m_kernel<N, T>), dim3((unsigned)ncellsF), dim3(EW), 0, s, xs, ys, zs,
                       f.start, f.box, R, sD, lev[F], ch);
    for (int l = F - 1; l >= 2; --l) {
        const int64_t Q = lev[l].side / 2, ntc = (Q * Q * Q + TN - 1) / TN;
        hipLaunchKernelGGL(m2m_kernel<N>, dim3(trans_blocks(ntc)), dim3(kM2lThreads), 0, s, lev[l],
                           lev[l + 1], f.Tu, ntr_t, ntc);
    }
    // the refined levels' target cells, listed per class in sub-grid order
    for (int q = 1; q <= R; ++q) {
        const int l = D + q;
        const int64_t nc = ncells_at(q);
        hipLaunchKernelGGL(tmask_kernel, dim3(ew_blocks(nc)), dim3(EW), 0, s, lev[l],
                           f.refined[q - 1], q, sD);
        hipLaunchKernelGGL(tflag_kernel, dim3(ew_blocks(nc)), dim3(EW), 0, s, lev[l], f.tflag[q]);
        hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(EW), 0, s, f.tflag[q] + nc, (int64_t)1);
        tb = f.temp_bytes;
        if ((e = hipcub::DeviceScan::ExclusiveSum(f.temp, tb, f.tflag[q], f.tscan[q],
                                                  (int)(nc + 1), s)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(tlist_kernel, dim3(ew_blocks(nc)), dim3(EW), 0, s, lev[l], f.tflag[q],
                           f.tscan[q], f.tlist[q]);
        lev[l].tlist = f.tlist[q];
        lev[l].tscan = f.tscan[q];
    }
    // interactions (every level in one launch), then the downward pass
    const int64_t ntab = (int64_t)kOffsets * M2lShape<N>::KP * M2lShape<N>::RP;
    M2lPlan plan{};
    plan.nlev = F - 1;
    plan.ntr = M2lShape<N>::RP / TM;
    plan.ntiles = 0;
    int64_t npart = 0;
    for (int l = 2; l <= F; ++l) {
        double *At = f.A + (l - 2) * ntab;
        if (f.kernel == kKernelLog)
            hipLaunchKernelGGL((m2l_table_kernel<N, kKernelLog>), dim3(ew_blocks(ntab)), dim3(EW),
                               0, s, f.box, l, f.eps, ch, At);
        else
            hipLaunchKernelGGL((m2l_table_kernel<N, kKernelDistance>), dim3(ew_blocks(ntab)),
                               dim3(EW), 0, s, f.box, l, f.eps, ch, At);
        const int64_t Q = lev[l].side / 2, Q3 = Q * Q * Q;
        const int i = l - 2;
        plan.lev[i] = lev[l];
        plan.At[i] = At;
        plan.ntc[i] = (Q3 + TN - 1) / TN;
        plan.nsplit[i] = m2l_split(8 * plan.ntc[i] * plan.ntr);
        plan.first[i] = plan.ntiles;
        plan.ntiles += 8 * plan.ntc[i] * plan.nsplit[i];
        plan.pfirst[i] = npart;
        if (plan.nsplit[i] > 1)
            npart += 8 * plan.ntc[i] * plan.ntr * plan.nsplit[i];
    }
    plan.part = f.part;
    // near field (exact pair sums over the 27 cells around each target's cell
    // at its final level).  With the caller's second stream it runs there
    // beside the M2L (the near field on the vector ALUs, the M2L on the matrix
    // cores): the call's stream forks to it after the upward pass (which then
    // keeps the whole chip) and joins it before the L2P adds the far field.
    // Without one it runs on the call's stream.
    const bool fork = SPK_FMM_OVERLAP && f.side != nullptr && f.side != s;
    hipStream_t ns = fork ? f.side : s;
    struct Events {   // released on every path (a pending event may be destroyed)
        hipEvent_t fork = nullptr, join = nullptr;
        ~Events()
        {
            if (fork)
                (void)hipEventDestroy(fork);
            if (join)
                (void)hipEventDestroy(join);
        }
    } ev;
    if (fork) {
        if ((e = hipEventCreateWithFlags(&ev.fork, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&ev.join, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventRecord(ev.fork, s)) != hipSuccess ||
            (e = hipStreamWaitEvent(ns, ev.fork, 0)) != hipSuccess)
            return e;
    }
    NearLaunch nl;
    nl.precision = f.precision;
    nl.kernel = f.kernel;
    nl.energy = f.energy;
    nl.xs = xs;
    nl.ys = ys;
    nl.zs = zs;
    nl.order = f.vals_out;
    nl.start = f.start;
    nl.sD = sD;
    nl.t0 = f.t0;
    nl.nt = f.nt;
    nl.eps = f.eps;
    nl.acc = f.acc;
    nl.ld = f.ld;
    for (int q = 0; q <= R; ++q) {
        nl.sub = q;
        nl.stride = stride_at(q);
        nl.chunk_start = f.chunk_start[q];
        nl.ncells = ncells_at(q);
        nl.side = sD << q;
        nl.max_blocks = (p + f.near_tpb - 1) / f.near_tpb + ncells_at(q);
        if ((e = launch_near(nl, ns)) != hipSuccess)
            return e;
    }
    if (fork) {
        if ((e = hipEventRecord(ev.join, ns)) != hipSuccess)
            return e;
    }
    const int64_t nblocks = (plan.ntiles + kXcds - 1) / kXcds * kXcds * plan.ntr;
    hipLaunchKernelGGL(m2l_kernel<N>, dim3((unsigned)nblocks), dim3(kM2lThreads), 0, s, plan);
    for (int i = 0; i < plan.nlev; ++i)
        if (plan.nsplit[i] > 1)
            hipLaunchKernelGGL(m2l_reduce_kernel<N>,
                               dim3((unsigned)(8 * plan.ntc[i] * plan.ntr)), dim3(kM2lThreads),
                               0, s, plan, i);
    for (int l = 3; l <= F; ++l) {
        const int64_t Q = lev[l].side / 2, ntc = (4 * Q * Q * Q + TN - 1) / TN;
        hipLaunchKernelGGL(l2l_kernel<N>, dim3(trans_blocks(ntc)), dim3(kM2lThreads), 0, s,
                           lev[l - 1], lev[l], f.Td, ntr_t, ntc);
    }
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    // the near field's sums are in acc before the far field is added
    if (fork) {
        if ((e = hipStreamWaitEvent(s, ev.join, 0)) != hipSuccess)
            return e;
    }
    L2pLevels lv{};
    lv.R = R;
    lv.sD = sD;
    for (int q = 0; q <= R; ++q)
        lv.lev[q] = lev[D + q];
    for (int q = 0; q < R; ++q)
        lv.refined[q] = f.refined[q];
    hipLaunchKernelGGL((l2p_kernel<N, T>), dim3(ew_blocks(p)), dim3(EW), 0, s, xs, ys, zs,
                       f.keys_out, f.vals_out, p, f.box, lv, ch, f.t0, f.nt, f.energy, f.acc,
                       f.ld);
    return hipGetLastError();
}

template <int N>
hipError_t run_order(const FmmLaunch &f, hipStream_t s)
{
    return f.precision == SPK_PLAIN_FP64 ? run_typed<N, double>(f, s) : run_typed<N, float>(f, s);
}

}  // namespace

hipError_t launch_fmm_repulsion(const FmmLaunch &f, hipStream_t s)
{
    if (f.depth < 2 || f.adaptive < 0 || f.adaptive > kMaxRefine ||
        f.depth + f.adaptive > kFmmMaxDepth || f.p < 1)
        return hipErrorInvalidValue;
    switch (f.order) {
    case 3: return run_order<3>(f, s);
    case 4: return run_order<4>(f, s);
    case 5: return run_order<5>(f, s);
    case 6: return run_order<6>(f, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace spk
