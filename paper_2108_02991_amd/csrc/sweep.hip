// Pair sweeps of the SPARKLING gradient (gfx950).
//
// Repulsion (Sec. "Evaluating F^r and its gradient"): for target i and every
// sample j, d = K[i] - K[j], w = 1/sqrt(|d|^2 + g) with a guard g (eps^2, or
// the smallest normal when eps = 0, so d = 0 contributes w*0 = 0),
//   g_r[i] += w d,   u_r[i] += w |d|^2 (= H(d)).
// Attraction (Sec. "Evaluating F^a and its gradient", discretised density):
// the same with every grid cell v as a source weighted by rho_v,
//   g_a[i] += rho_v w d,   u_a[i] += rho_v w |d|^2.
//
// Layout and schedule.  Each lane owns R targets (register blocking), a block
// of 256 lanes owns 256*R consecutive targets (coalesced SoA loads), and the
// block's sources are staged tile by tile in LDS; every lane of a wave then
// reads the same LDS address (a broadcast) and runs R pairs per read.  There
// is no MFMA: the pair map is not a contraction, so the sweep is bound by the
// VALU issue rate (subtract, FMA, and one reciprocal square root per pair).
// The cell sweep walks the grid row by row: inside an x-row the y and z
// offsets are constant, so a pair costs one subtract, one FMA for |d|^2, the
// rsqrt, one multiply by rho_v, one add for the row weight and one FMA for
// the x force; the y and z forces are row weight times offset, once per row.
//
// Kernels (template KERN): the distance kernel H(d) = sqrt(|d|^2 + eps^2)
// above, or the logarithmic kernel H(d) = log(|d|^2 + eps^2) / 2 (the
// alternative the "3D SPARKLING formulation" mentions; eps > 0), whose pair
// is w = 1/(|d|^2 + eps^2) (one reciprocal) with the force w d, and the
// potential log2(|d|^2 + eps^2) accumulated as is and scaled by ln(2)/2 once
// per slab total.
//
// Precision forms (template MODE):
//   kPlain64 : double coordinates, double math, double running sums;
//   kComp    : float pair math, float per-tile sums folded into a float
//              (sum, compensation) pair by an error-free two-sum;
//   kNaive   : float pair math, one float running sum per slab (diagnostic);
//   kAcc64   : float pair math, every pair term added into a double (diagnostic).
// Every form writes its slab sums as doubles; slabs are combined in a fixed
// order elsewhere, so results do not depend on the target chunking.

#include <cfloat>

#include "sweep.h"

namespace spk {
namespace {

enum : int { kPlain64 = SPK_PLAIN_FP64, kComp = SPK_FP32_COMP, kNaive = SPK_FP32_NAIVE,
             kAcc64 = SPK_FP32_ACC64 };
enum : int { kDist = kKernelDistance, kLog = kKernelLog };

constexpr int BLK = kSweepBlock;

template <int MODE> struct ModeT {
    using T = float;       // coordinate / pair-math type
    using A = float;       // accumulator type inside a tile
};
template <> struct ModeT<kPlain64> { using T = double; using A = double; };
template <> struct ModeT<kAcc64> { using T = float; using A = double; };

template <int MODE> constexpr int lanes_targets() { return MODE == kPlain64 ? kTargetsF64 : kTargetsF32; }
template <int MODE> constexpr int min_waves() { return MODE == kComp || MODE == kNaive ? SPK_SWEEP_WAVES_F32 : 1; }
// The FP32-compensated cell sweep reads its cells one group ahead (below);
// held at 8 waves per SIMD (64 VGPRs, a few per-tile values spilled) it ran
// 2% faster than the plain loop, and 9% slower when left at 77 VGPRs.
template <int MODE> constexpr int cell_waves() { return MODE == kComp ? 8 : min_waves<MODE>(); }

template <typename T> struct alignas(4 * sizeof(T)) P4 { T x, y, z, w; };
template <typename T> struct alignas(2 * sizeof(T)) P2 { T x, y; };

__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// Double reciprocal square root for the guarded |d|^2 (finite, >= the
// smallest normal): the hardware estimate y0 refined once with the
// second-order term of (1 - r)^(-1/2) = 1 + r/2 + 3r^2/8 + ..., where
// r = 1 - x*y0^2 is formed with an FMA; the estimate's relative error e
// leaves O(e^3), far below double rounding.
__device__ inline double rsq(double x)
{
    const double y0 = __builtin_amdgcn_rsq(x);
    const double r = __builtin_fma(-x * y0, y0, 1.0);
    const double c = __builtin_fma(r, 0.375, 0.5);
    return __builtin_fma(y0 * r, c, y0);
}

__device__ inline float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Double reciprocal: the hardware estimate y0 refined once with the
// third-order step y0 (1 + e + e^2), e = 1 - x y0 (an FMA), leaving O(e^3).
__device__ inline double rcp(double x)
{
    const double y0 = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, y0, 1.0);
    return __builtin_fma(y0, __builtin_fma(e, e, e), y0);
}
// log2 of a normal positive number.
__device__ inline float lg2(float x) { return __builtin_amdgcn_logf(x); }
__device__ inline double lg2(double x) { return log2(x); }

// Pair weight of the kernel from the guarded |d|^2.
template <int KERN, typename T> __device__ inline T pair_weight(T r2)
{
    if constexpr (KERN == kLog)
        return rcp(r2);
    else
        return rsq(r2);
}

// Factor turning the accumulated potential sum into H: 1, or ln(2)/2 for the
// log kernel, which accumulates log2(|d|^2 + eps^2).
template <int KERN> __device__ inline double potential_scale()
{
    return KERN == kLog ? 0.34657359027997264 : 1.0;
}

__device__ inline float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Cell centre -L + (i + 1/2) * (2L / G), evaluated exactly in this order in double.
__device__ inline double cell_centre(int64_t i, int64_t G, double L)
{
#pragma clang fp contract(off)
    return -L + ((double)i + 0.5) * (2.0 * L / (double)G);
}

template <typename T> __device__ inline T guard_value(double eps);
template <> __device__ inline float guard_value<float>(double eps)
{
    float e2 = (float)(eps * eps);
    return e2 > FLT_MIN ? e2 : FLT_MIN;
}
template <> __device__ inline double guard_value<double>(double eps)
{
    double e2 = eps * eps;
    return e2 > DBL_MIN ? e2 : DBL_MIN;
}

// Running sums of one target component across tiles.
template <int MODE> struct Acc {
    typename ModeT<MODE>::A t = 0;    // inside the current tile (or whole slab)
    float s = 0.f, c = 0.f;           // kComp: compensated total
    __device__ inline void end_tile()
    {
        if constexpr (MODE == kComp) {
            float x = t;
            float sum = s + x;
            float bp = sum - s;
            float err = (s - (sum - bp)) + (x - bp);
            s = sum;
            c += err;
            t = 0.f;
        }
    }
    __device__ inline double total() const
    {
        if constexpr (MODE == kComp)
            return (double)s + (double)c;
        else
            return (double)t;
    }
};

// gx += w * d for the accumulator of this mode.
template <int MODE, typename T>
__device__ inline void acc_fma(Acc<MODE> &a, T w, T d)
{
    if constexpr (MODE == kAcc64)
        a.t += (double)(w * d);
    else
        a.t = fmaT(w, d, a.t);
}

template <int MODE, typename T>
__device__ inline void acc_add(Acc<MODE> &a, T x)
{
    if constexpr (MODE == kAcc64)
        a.t += (double)x;
    else
        a.t += x;
}

template <int MODE, int R, bool ENERGY, int KERN>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(min_waves<MODE>())))
void sweep_samples_kernel(SweepLaunch l)
{
    using T = typename ModeT<MODE>::T;
    __shared__ P4<T> tile[kSampleTile];

    const T *tx = static_cast<const T *>(l.tx), *ty = static_cast<const T *>(l.ty),
            *tz = static_cast<const T *>(l.tz);
    const T *sx = static_cast<const T *>(l.sx), *sy = static_cast<const T *>(l.sy),
            *sz = static_cast<const T *>(l.sz);

    const int64_t tlast = l.t0 + l.nt - 1;
    const int64_t tbase = l.t0 + (int64_t)blockIdx.x * (BLK * R) + threadIdx.x;
    T xi[R], yi[R], zi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t t = tbase + r * BLK;
        t = t < tlast ? t : tlast;
        xi[r] = tx[t];
        yi[r] = ty[t];
        zi[r] = tz[t];
    }
    Acc<MODE> gx[R], gy[R], gz[R], ee[R];
    const T guard = guard_value<T>(l.eps);

    const int64_t lo = l.src_begin + (int64_t)blockIdx.y * l.slab;
    int64_t hi = lo + l.slab;
    hi = hi < l.src_end ? hi : l.src_end;

    for (int64_t base = lo; base < hi; base += kSampleTile) {
        const int n = (int)((hi - base) < kSampleTile ? (hi - base) : kSampleTile);
        for (int j = threadIdx.x; j < n; j += BLK)
            tile[j] = P4<T>{sx[base + j], sy[base + j], sz[base + j], T(0)};
        __syncthreads();

        auto pair = [&](const P4<T> s) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                T dx = xi[r] - s.x, dy = yi[r] - s.y, dz = zi[r] - s.z;
                T r2 = fmaT(dz, dz, fmaT(dy, dy, fmaT(dx, dx, guard)));
                T w = pair_weight<KERN>(r2);
                acc_fma(gx[r], w, dx);
                acc_fma(gy[r], w, dy);
                acc_fma(gz[r], w, dz);
                if constexpr (ENERGY) {
                    if constexpr (KERN == kLog)
                        acc_add(ee[r], lg2(r2));
                    else
                        acc_fma(ee[r], w, r2);
                }
            }
        };
        if (n == kSampleTile) {
            // Full tile: LDS reads run one group of U sources ahead of the
            // pair arithmetic, so the broadcast latency hides behind the
            // previous group's VALU work.
            constexpr int U = SPK_SOURCE_UNROLL;
            static_assert(kSampleTile % U == 0 && (kSampleTile & (kSampleTile - 1)) == 0, "");
            P4<T> cur[U], nxt[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                cur[u] = tile[u];
            for (int j = 0; j < kSampleTile; j += U) {
                const int jn = (j + U) & (kSampleTile - 1);   // the last group re-reads group 0
#pragma unroll
                for (int u = 0; u < U; ++u)
                    nxt[u] = tile[jn + u];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    pair(cur[u]);
#pragma unroll
                for (int u = 0; u < U; ++u)
                    cur[u] = nxt[u];
            }
        } else {
            for (int j = 0; j < n; ++j)
                pair(tile[j]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            gx[r].end_tile();
            gy[r].end_tile();
            gz[r].end_tile();
            if constexpr (ENERGY)
                ee[r].end_tile();
        }
        __syncthreads();
    }

    double *out = l.part + (int64_t)blockIdx.y * 4 * l.ld;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t t = tbase + r * BLK;
        if (t <= tlast) {
            const int64_t o = t - l.t0;
            out[o] = gx[r].total();
            out[l.ld + o] = gy[r].total();
            out[2 * l.ld + o] = gz[r].total();
            if constexpr (KERN == kLog)
                out[3 * l.ld + o] = ENERGY ? potential_scale<KERN>() * ee[r].total() : 0.0;
            else
                out[3 * l.ld + o] = ENERGY ? ee[r].total() : 0.0;
        }
    }
}

template <int MODE, int R, bool ENERGY, int KERN>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(cell_waves<MODE>())))
void sweep_cells_kernel(SweepLaunch l)
{
    using T = typename ModeT<MODE>::T;
    constexpr int TILE = MODE == kPlain64 ? kCellTileF64 : kCellTileF32;
    __shared__ P2<T> cell[TILE];     // (x_v, rho_v) of the tile's cells, row after row

    const T *tx = static_cast<const T *>(l.tx), *ty = static_cast<const T *>(l.ty),
            *tz = static_cast<const T *>(l.tz);
    const T *rho = static_cast<const T *>(l.rho);
    const int64_t G = l.grid;
    const int g = (int)G;
    const double L = l.half_width;

    const int64_t tlast = l.t0 + l.nt - 1;
    const int64_t tbase = l.t0 + (int64_t)blockIdx.x * (BLK * R) + threadIdx.x;
    T xi[R], yi[R], zi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t t = tbase + r * BLK;
        t = t < tlast ? t : tlast;
        xi[r] = tx[t];
        yi[r] = ty[t];
        zi[r] = tz[t];
    }
    Acc<MODE> gx[R], gy[R], gz[R], ee[R];
    const T guard = guard_value<T>(l.eps);

    const int rows_per_tile = TILE / g;
    const int64_t lo = l.src_begin + (int64_t)blockIdx.y * l.slab;
    int64_t hi = lo + l.slab;
    hi = hi < l.src_end ? hi : l.src_end;
    // row = iy + G*iz; the (iy, iz) counters advance with the rows (wave-uniform)
    int64_t iy = lo % G, iz = lo / G;

    for (int64_t base = lo; base < hi; base += rows_per_tile) {
        const int nr = (int)((hi - base) < rows_per_tile ? (hi - base) : rows_per_tile);
        const int nv = nr * g;
        for (int j = threadIdx.x; j < nv; j += BLK) {
            const int ix = j % g;
            cell[j] = P2<T>{(T)cell_centre(ix, G, L), rho[base * G + j]};
        }
        __syncthreads();

        for (int rr = 0; rr < nr; ++rr) {
            const P2<T> yz{(T)cell_centre(iy, G, L), (T)cell_centre(iz, G, L)};
            if (++iy == G) {
                iy = 0;
                ++iz;
            }
            T dy[R], dz[R], c[R];
            typename ModeT<MODE>::A wrow[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                dy[r] = yi[r] - yz.x;
                dz[r] = zi[r] - yz.y;
                c[r] = fmaT(dz[r], dz[r], fmaT(dy[r], dy[r], guard));
                wrow[r] = 0;
            }
            const P2<T> *rowp = cell + rr * g;
            auto pair = [&](const P2<T> v) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    T dx = xi[r] - v.x;
                    T r2 = fmaT(dx, dx, c[r]);
                    T w = v.y * pair_weight<KERN>(r2);
                    wrow[r] += w;
                    acc_fma(gx[r], w, dx);
                    if constexpr (ENERGY) {
                        if constexpr (KERN == kLog)
                            acc_fma(ee[r], v.y, lg2(r2));
                        else
                            acc_fma(ee[r], w, r2);
                    }
                }
            };
            int ix = 0;
            if constexpr (MODE == kComp) {
                // Cells in row order, read one group of 4 ahead of the pair
                // arithmetic into two alternating register groups (a read
                // past the row's last group re-reads its group 0).
                const int g4 = g & ~3;
                if (g4 > 0) {
                    P2<T> a[4], b[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        a[u] = rowp[u];
                    for (; ix < g4; ix += 8) {
                        const int j1 = ix + 4 < g4 ? ix + 4 : 0;
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            b[u] = rowp[j1 + u];
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            pair(a[u]);
                        if (ix + 4 >= g4) {
                            ix += 4;
                            break;
                        }
                        const int j2 = ix + 8 < g4 ? ix + 8 : 0;
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            a[u] = rowp[j2 + u];
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            pair(b[u]);
                    }
                }
            } else {
#pragma unroll 4
                for (; ix + 4 <= g; ix += 4) {
                    pair(rowp[ix]);
                    pair(rowp[ix + 1]);
                    pair(rowp[ix + 2]);
                    pair(rowp[ix + 3]);
                }
            }
            for (; ix < g; ++ix)
                pair(rowp[ix]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if constexpr (MODE == kAcc64) {
                    gy[r].t += wrow[r] * (double)dy[r];
                    gz[r].t += wrow[r] * (double)dz[r];
                } else {
                    gy[r].t = fmaT(wrow[r], dy[r], gy[r].t);
                    gz[r].t = fmaT(wrow[r], dz[r], gz[r].t);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            gx[r].end_tile();
            gy[r].end_tile();
            gz[r].end_tile();
            if constexpr (ENERGY)
                ee[r].end_tile();
        }
        __syncthreads();
    }

    double *out = l.part + (int64_t)blockIdx.y * 4 * l.ld;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t t = tbase + r * BLK;
        if (t <= tlast) {
            const int64_t o = t - l.t0;
            out[o] = gx[r].total();
            out[l.ld + o] = gy[r].total();
            out[2 * l.ld + o] = gz[r].total();
            if constexpr (KERN == kLog)
                out[3 * l.ld + o] = ENERGY ? potential_scale<KERN>() * ee[r].total() : 0.0;
            else
                out[3 * l.ld + o] = ENERGY ? ee[r].total() : 0.0;
        }
    }
}

// Near field of the far-field repulsion: every sample of a cell against the
// samples of the 27 cells around it (itself included).  Those are runs of the
// cell-sorted samples: nine runs of three leaves along x at the leaves' level,
// 27 single cells below it.  The block streams the runs as one
// sequence, in run order, through LDS tiles of kSampleTile sources, so tiles
// fill across run boundaries.  Blocks are one wave (kNearBlock threads), each
// with kNearBlock * R targets.  Block b takes chunk b - chunk_start[cell] of
// the cell with chunk_start[cell] <= b < chunk_start[cell + 1]; the pair
// arithmetic and the accumulation are those of the sample sweep, and the sums
// are written (not added) to the rows of targets in [t0, t0 + nt).
template <int MODE, int R, bool ENERGY, int KERN>
__global__ __launch_bounds__(kNearBlock) __attribute__((amdgpu_waves_per_eu(min_waves<MODE>())))
void near_kernel(NearLaunch l)
{
    using T = typename ModeT<MODE>::T;
    __shared__ P4<T> tile[kSampleTile];
    __shared__ int64_t run_lo[27], run_pre[28];
    const int64_t b = blockIdx.x;
    if (b >= (int64_t)l.chunk_start[l.ncells])
        return;
    int64_t lo = 0, hi = l.ncells;           // chunk_start[lo] <= b < chunk_start[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)l.chunk_start[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    const int64_t cell = lo, side = l.side;
    int64_t ix, iy, iz;
    comp_coords(cell, l.sub, l.sD, ix, iy, iz);
    const int64_t t_lo = l.start[l.stride * cell], t_hi = l.start[l.stride * (cell + 1)];
    // the source runs, in a fixed order (z, y, then x)
    if (threadIdx.x < 27) {
        const int o = (int)threadIdx.x;
        const int64_t x = ix + o % 3 - 1, y = iy + (o / 3) % 3 - 1, z = iz + o / 9 - 1;
        int64_t s0 = 0, s1 = 0;
        const bool in_y = y >= 0 && y < side && z >= 0 && z < side;
        if (l.sub > 0) {
            if (in_y && x >= 0 && x < side) {
                const int64_t k = comp_index(x, y, z, l.sub, l.sD);
                s0 = l.start[l.stride * k];
                s1 = l.start[l.stride * (k + 1)];
            }
        } else if (in_y && o % 3 == 0) {     // one run of up to three leaves along x
            const int64_t x0 = ix > 0 ? ix - 1 : 0, x1 = ix + 1 < side ? ix + 1 : side - 1;
            const int64_t row = side * (y + side * z);
            s0 = l.start[l.stride * (x0 + row)];
            s1 = l.start[l.stride * (x1 + row + 1)];
        }
        run_lo[o] = s0;
        run_pre[o + 1] = s1 - s0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        run_pre[0] = 0;
        for (int o = 0; o < 27; ++o)
            run_pre[o + 1] += run_pre[o];
    }
    __syncthreads();
    const int64_t total = run_pre[27];
    const int64_t first = t_lo + (b - l.chunk_start[cell]) * (int64_t)(kNearBlock * R);
    const int64_t last = t_hi - 1;
    const T *xs = static_cast<const T *>(l.xs), *ys = static_cast<const T *>(l.ys),
            *zs = static_cast<const T *>(l.zs);
    T xi[R], yi[R], zi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        int64_t j = first + threadIdx.x + r * kNearBlock;
        j = j < last ? j : last;
        xi[r] = xs[j];
        yi[r] = ys[j];
        zi[r] = zs[j];
    }
    Acc<MODE> gx[R], gy[R], gz[R], ee[R];
    const T guard = guard_value<T>(l.eps);
    int run = 0;  // run of this thread's next source (sources are read in increasing order)
    for (int64_t base = 0; base < total; base += kSampleTile) {
        const int n = (int)((total - base) < kSampleTile ? (total - base) : kSampleTile);
        for (int j = threadIdx.x; j < n; j += kNearBlock) {
            const int64_t v = base + j;
            while (run_pre[run + 1] <= v)
                ++run;
            const int64_t src = run_lo[run] + (v - run_pre[run]);
            tile[j] = P4<T>{xs[src], ys[src], zs[src], T(0)};
        }
        __syncthreads();
        auto pair = [&](const P4<T> sv) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                T dx = xi[r] - sv.x, dy = yi[r] - sv.y, dz = zi[r] - sv.z;
                T r2 = fmaT(dz, dz, fmaT(dy, dy, fmaT(dx, dx, guard)));
                T w = pair_weight<KERN>(r2);
                acc_fma(gx[r], w, dx);
                acc_fma(gy[r], w, dy);
                acc_fma(gz[r], w, dz);
                if constexpr (ENERGY) {
                    if constexpr (KERN == kLog)
                        acc_add(ee[r], lg2(r2));
                    else
                        acc_fma(ee[r], w, r2);
                }
            }
        };
        if (n == kSampleTile) {
            // full tile: LDS reads one group of U sources ahead, as in the sweep
            constexpr int U = SPK_SOURCE_UNROLL;
            P4<T> cur[U], nxt[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                cur[u] = tile[u];
            for (int j = 0; j < kSampleTile; j += U) {
                const int jn = (j + U) & (kSampleTile - 1);
#pragma unroll
                for (int u = 0; u < U; ++u)
                    nxt[u] = tile[jn + u];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    pair(cur[u]);
#pragma unroll
                for (int u = 0; u < U; ++u)
                    cur[u] = nxt[u];
            }
        } else {
            for (int j = 0; j < n; ++j)
                pair(tile[j]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            gx[r].end_tile();
            gy[r].end_tile();
            gz[r].end_tile();
            if constexpr (ENERGY)
                ee[r].end_tile();
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j = first + threadIdx.x + r * kNearBlock;
        if (j > last)
            continue;
        const int64_t i = (int64_t)l.order[j] - l.t0;
        if (i < 0 || i >= l.nt)
            continue;
        l.acc[i] = gx[r].total();
        l.acc[l.ld + i] = gy[r].total();
        l.acc[2 * l.ld + i] = gz[r].total();
        if constexpr (KERN == kLog)
            l.acc[3 * l.ld + i] = ENERGY ? potential_scale<KERN>() * ee[r].total() : 0.0;
        else
            l.acc[3 * l.ld + i] = ENERGY ? ee[r].total() : 0.0;
    }
}

template <int MODE, bool ENERGY, int KERN>
hipError_t launch_near_mode(const NearLaunch &l, hipStream_t s)
{
    constexpr int R = lanes_targets<MODE>();
    hipLaunchKernelGGL((near_kernel<MODE, R, ENERGY, KERN>), dim3((unsigned)l.max_blocks),
                       dim3(kNearBlock), 0, s, l);
    return hipGetLastError();
}

template <int MODE, bool ENERGY, int KERN>
hipError_t launch_samples_mode(const SweepLaunch &l, hipStream_t s)
{
    constexpr int R = lanes_targets<MODE>();
    dim3 grid((unsigned)((l.nt + BLK * R - 1) / (BLK * R)), (unsigned)l.nslabs);
    hipLaunchKernelGGL((sweep_samples_kernel<MODE, R, ENERGY, KERN>), grid, dim3(BLK), 0, s, l);
    return hipGetLastError();
}

template <int MODE, bool ENERGY, int KERN>
hipError_t launch_cells_mode(const SweepLaunch &l, hipStream_t s)
{
    constexpr int R = lanes_targets<MODE>();
    dim3 grid((unsigned)((l.nt + BLK * R - 1) / (BLK * R)), (unsigned)l.nslabs);
    hipLaunchKernelGGL((sweep_cells_kernel<MODE, R, ENERGY, KERN>), grid, dim3(BLK), 0, s, l);
    return hipGetLastError();
}

template <bool CELLS, bool ENERGY, int MODE, int KERN>
hipError_t launch_one(const SweepLaunch &l, hipStream_t s)
{
    return CELLS ? launch_cells_mode<MODE, ENERGY, KERN>(l, s)
                 : launch_samples_mode<MODE, ENERGY, KERN>(l, s);
}

// The log kernel is built for the plain FP64 and compensated FP32 forms only.
template <bool CELLS, bool ENERGY>
hipError_t launch_any(const SweepLaunch &l, hipStream_t s)
{
    if (l.kernel == kLog) {
        switch (l.precision) {
        case kPlain64: return launch_one<CELLS, ENERGY, kPlain64, kLog>(l, s);
        case kComp: return launch_one<CELLS, ENERGY, kComp, kLog>(l, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (l.kernel != kDist)
        return hipErrorInvalidValue;
    switch (l.precision) {
    case kPlain64: return launch_one<CELLS, ENERGY, kPlain64, kDist>(l, s);
    case kComp: return launch_one<CELLS, ENERGY, kComp, kDist>(l, s);
    case kNaive: return launch_one<CELLS, ENERGY, kNaive, kDist>(l, s);
    case kAcc64: return launch_one<CELLS, ENERGY, kAcc64, kDist>(l, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_near(const NearLaunch &l, hipStream_t s)
{
    if (l.max_blocks <= 0)
        return hipSuccess;
    const bool e = l.energy;
    if (l.kernel == kLog) {
        if (l.precision == kPlain64)
            return e ? launch_near_mode<kPlain64, true, kLog>(l, s)
                     : launch_near_mode<kPlain64, false, kLog>(l, s);
        if (l.precision == kComp)
            return e ? launch_near_mode<kComp, true, kLog>(l, s)
                     : launch_near_mode<kComp, false, kLog>(l, s);
        return hipErrorInvalidValue;
    }
    if (l.precision == kPlain64)
        return e ? launch_near_mode<kPlain64, true, kDist>(l, s)
                 : launch_near_mode<kPlain64, false, kDist>(l, s);
    if (l.precision == kComp)
        return e ? launch_near_mode<kComp, true, kDist>(l, s)
                 : launch_near_mode<kComp, false, kDist>(l, s);
    return hipErrorInvalidValue;
}

int sweep_targets_per_block(int precision)
{
    return BLK * (precision == kPlain64 ? lanes_targets<kPlain64>() : lanes_targets<kComp>());
}

int near_targets_per_block(int precision)
{
    return kNearBlock *
           (precision == kPlain64 ? lanes_targets<kPlain64>() : lanes_targets<kComp>());
}

hipError_t launch_sweep_samples(const SweepLaunch &l, hipStream_t s)
{
    if (l.nt <= 0 || l.nslabs <= 0)
        return hipSuccess;
    return l.energy ? launch_any<false, true>(l, s) : launch_any<false, false>(l, s);
}

hipError_t launch_sweep_cells(const SweepLaunch &l, hipStream_t s)
{
    if (l.nt <= 0 || l.nslabs <= 0)
        return hipSuccess;
    return l.energy ? launch_any<true, true>(l, s) : launch_any<true, false>(l, s);
}

}  // namespace spk
