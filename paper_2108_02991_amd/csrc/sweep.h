// Interface of the pair sweeps (sweep.hip): tunables, the launch record and
// the launchers.  Everything that shapes the sweep kernels' code lives here
// and in sweep.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sparkling.h"

namespace spk {

// Build-time tunables of the pair sweeps (defaults are the tuned values).
#ifndef SPK_SWEEP_BLOCK
#define SPK_SWEEP_BLOCK 256
#endif
#ifndef SPK_SAMPLE_TILE
#define SPK_SAMPLE_TILE 512
#endif
#ifndef SPK_TARGETS_F32
#define SPK_TARGETS_F32 2
#endif
#ifndef SPK_TARGETS_F64
#define SPK_TARGETS_F64 2
#endif
#ifndef SPK_SOURCE_UNROLL
#define SPK_SOURCE_UNROLL 4
#endif
// Minimum waves per SIMD the FP32-accumulating sweeps are compiled for (caps
// VGPRs at 512/waves); 1 leaves the choice to the compiler.  Sweeps with FP64
// accumulators are not capped.
#ifndef SPK_SWEEP_WAVES_F32
#define SPK_SWEEP_WAVES_F32 1
#endif

// Threads per block of the pair sweeps.
constexpr int kSweepBlock = SPK_SWEEP_BLOCK;
// Sources staged in LDS per tile by the sample sweep.
constexpr int kSampleTile = SPK_SAMPLE_TILE;
// Targets per lane (register blocking) of the FP32 forms and of plain FP64.
constexpr int kTargetsF32 = SPK_TARGETS_F32;
constexpr int kTargetsF64 = SPK_TARGETS_F64;
// Density cells staged in LDS per tile by the cell sweep (rows of G cells).
constexpr int kCellTileF32 = 2048;
constexpr int kCellTileF64 = 1024;
// Largest grid side supported (one row must fit a tile).
constexpr int64_t kMaxGrid = 1024;

// Targets handled by one block of a sweep (blockDim * targets per lane).
int sweep_targets_per_block(int precision);
// The near-field kernel runs one wave per block, so that cells with few
// targets leave few lanes idle; near_targets_per_block() targets per block.
constexpr int kNearBlock = 64;
int near_targets_per_block(int precision);

// Pair kernels H of the sweeps.
constexpr int kKernelDistance = 0;   // sqrt(|d|^2 + eps^2)
constexpr int kKernelLog = 1;        // log(|d|^2 + eps^2) / 2, eps > 0

// One launch of a pair sweep: a target range against `nslabs` consecutive
// source slabs.  Slab y covers sources [src_begin + y*slab, min(+slab, src_end))
// where a source is a sample (sample sweep) or a row of G cells (cell sweep).
// Block (x, y) writes its four sums (gx, gy, gz, potential) for target t into
// part[(y*4 + c)*ld + (t - t0)] as doubles.
struct SweepLaunch {
    int precision = 0;
    int kernel = kKernelDistance;
    bool energy = false;
    const void *tx = nullptr, *ty = nullptr, *tz = nullptr;
    int64_t t0 = 0, nt = 0;
    const void *sx = nullptr, *sy = nullptr, *sz = nullptr;  // sample sweep sources
    const void *rho = nullptr;                                 // cell sweep weights
    int64_t grid = 1;
    double half_width = 0.5;
    double eps = 0.0;
    int64_t src_begin = 0, slab = 0, src_end = 0;
    int nslabs = 1;
    double *part = nullptr;
    int64_t ld = 0;
};

hipError_t launch_sweep_samples(const SweepLaunch &l, hipStream_t s);
hipError_t launch_sweep_cells(const SweepLaunch &l, hipStream_t s);

// Near field of the far-field repulsion (plain FP64 and compensated FP32
// forms): targets of each leaf against the samples of the 27 leaves around
// it, from samples sorted by leaf.  Writes the four sums of every target in
// [t0, t0 + nt) to acc[c*ld + i - t0].  Blocks of sweep_targets_per_block()
// targets; chunk_start[k] is the first block of leaf k (an exclusive prefix
// sum of the per-leaf block counts, nleaves + 1 entries); the grid has
// max_blocks >= chunk_start[nleaves] blocks and the extra ones return.
// Composite cell index at level D + q (q >= 0 levels below the leaves of
// level D, sD leaves per axis): the x-fastest index of the level-D ancestor,
// then q octal digits, the child positions cx + 2 cy + 4 cz from the coarsest
// down.  Samples sorted by this index at the deepest level keep every cell of
// every level between contiguous.
__host__ __device__ inline int64_t comp_index(int64_t x, int64_t y, int64_t z, int q, int64_t sD)
{
    int64_t k = (x >> q) + sD * ((y >> q) + sD * (z >> q));
    for (int r = q - 1; r >= 0; --r)
        k = 8 * k + (((x >> r) & 1) | (((y >> r) & 1) << 1) | (((z >> r) & 1) << 2));
    return k;
}

__host__ __device__ inline void comp_coords(int64_t k, int q, int64_t sD, int64_t &x, int64_t &y,
                                            int64_t &z)
{
    int64_t dx = 0, dy = 0, dz = 0;
    for (int r = 0; r < q; ++r) {
        const int64_t c = k & 7;
        dx |= (c & 1) << r;
        dy |= ((c >> 1) & 1) << r;
        dz |= (c >> 2) << r;
        k >>= 3;
    }
    x = ((k % sD) << q) | dx;
    y = (((k / sD) % sD) << q) | dy;
    z = ((k / (sD * sD)) << q) | dz;
}

// Near-field cells are those of level D + sub in composite numbering; cell k
// owns sorted samples [start[stride k], start[stride (k+1)]) (stride = 8^(R -
// sub) with samples sorted R levels below the leaves).
struct NearLaunch {
    int precision = 0;
    int kernel = kKernelDistance;
    bool energy = false;
    int sub = 0;                       // levels below the leaves
    int64_t sD = 0;                    // leaves per axis
    const void *xs = nullptr, *ys = nullptr, *zs = nullptr;   // cell-sorted samples
    const uint32_t *order = nullptr;   // sorted position -> sample index
    const int32_t *start = nullptr;    // first sorted sample of each deepest cell
    int64_t stride = 1;                // start index of cell k is stride k
    const int32_t *chunk_start = nullptr;  // [ncells + 1] target chunks before each cell
    int64_t ncells = 0, side = 0;      // cells, and cells per axis
    int64_t t0 = 0, nt = 0;
    double eps = 0.0;
    double *acc = nullptr;
    int64_t ld = 0;
    int64_t max_blocks = 0;
};

hipError_t launch_near(const NearLaunch &l, hipStream_t s);

}  // namespace spk
