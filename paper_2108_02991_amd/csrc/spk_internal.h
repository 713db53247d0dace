// Internal interfaces between the translation units of libsparkling.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sparkling.h"
#include "sweep.h"

namespace spk {

// Largest shot length the projection kernel supports.
constexpr int64_t kMaxProjectSamples = 4096;

// Far field of the repulsion (fmm.hip): a Chebyshev fast multipole method on a
// uniform octree of `depth` levels below the root cube, interpolation order
// `order` per axis, with the near field summed exactly (launch_near).  Writes
// the four repulsion sums of targets [t0, t0 + nt) to acc[c*ld + i - t0].
constexpr int kFmmMaxDepth = 7;
constexpr int kFmmMinOrder = 3;
constexpr int kFmmMaxOrder = 6;
constexpr int kFmmBoxBlocks = 1024;
constexpr int kMaxRefine = 2;        // refinement levels of the adaptive tree
struct FmmLaunch {
    int precision = 0, kernel = kKernelDistance;
    bool energy = false;
    int depth = 0, order = 0;             // base depth D, interpolation order
    int adaptive = 0;                     // refinement levels R below the leaves (0..2)
    const void *x = nullptr, *y = nullptr, *z = nullptr;
    int64_t p = 0, t0 = 0, nt = 0;
    double eps = 0.0;
    double *acc = nullptr;
    int64_t ld = 0;
    int near_tpb = 0;                     // targets per near-field block
    hipStream_t side = nullptr;           // caller's second stream for the near field, or null
    // workspace
    double *box_part = nullptr;           // [kFmmBoxBlocks][6]
    double *box = nullptr;                // centre[3], half-width
    uint32_t *keys_in = nullptr, *keys_out = nullptr, *vals_in = nullptr, *vals_out = nullptr;
    void *xs = nullptr, *ys = nullptr, *zs = nullptr;
    // F = D + R: cell starts [8^F + 1]; per level D + q (q = 0..R) the
    // near-field chunks and their scan [8^(D+q) + 1]
    int32_t *start = nullptr;
    int32_t *chunks[kMaxRefine + 1] = {}, *chunk_start[kMaxRefine + 1] = {};
    int32_t *refined[kMaxRefine] = {};    // refine flags of level D + q, [8^(D+q)]
    // refined levels D + q (q = 1..R): target masks [8][P^3], their flags,
    // scans [8^(D+q) + 1] and lists [8^(D+q)]
    int32_t *tmask[kMaxRefine + 1] = {}, *tflag[kMaxRefine + 1] = {};
    int32_t *tscan[kMaxRefine + 1] = {}, *tlist[kMaxRefine + 1] = {};
    void *temp = nullptr;
    size_t temp_bytes = 0;
    double *W[kFmmMaxDepth + 1] = {};     // level l: [8][P^3][order^3]
    int32_t *occ[kFmmMaxDepth + 1] = {};  // level l: [8][P^3]
    double *L[kFmmMaxDepth + 1] = {};     // level l: [8][P^3][4 order^3]
    double *A = nullptr;                  // [F-1][343][k padded][rows padded]
    double *Tm = nullptr;                 // [8][order^3][order^3]
    double *Tu = nullptr, *Td = nullptr;  // M2M and L2L tables, [8][k padded][rows padded]
    double *part = nullptr;               // M2L partial tiles of split levels
};
// Padded class side P and cell slots 8 P^3 of level l.
int64_t fmm_padded_side(int level);
size_t fmm_level_cells(int level);
size_t fmm_table_doubles(int order);  // M2L table of one level, padded
size_t fmm_trans_doubles(int order);  // one M2M or L2L table, padded
size_t fmm_split_doubles(int order, int deepest);  // M2L partial tiles
// Temporary bytes of the cell sort (3 * depth key bits) and of the chunk scans.
size_t fmm_sort_temp_bytes(int64_t p, int depth);
// Price of refining one leaf, in direct pairs (adaptive tree).
int64_t fmm_refine_threshold(int order);
hipError_t launch_fmm_repulsion(const FmmLaunch &f, hipStream_t s);

// acc[c*ld + t] = (init ? 0 : acc[c*ld + t]) + part[0][c][t] + ... + part[n-1][c][t],
// with part[y][c][t] at part[(y*4 + c)*part_ld + t].
hipError_t launch_combine(double *acc, int64_t ld, const double *part, int64_t part_ld,
                          int nslabs, int64_t nt, bool init, hipStream_t s);

// g[c][t] = acc_a[c][t] * inv_p - acc_r[c][t] * inv_p2 (cast to the precision's type);
// pot_a/pot_r (nullable) receive row 3 of acc_a/acc_r.
hipError_t launch_finalize_grad(int precision, const double *acc_a, const double *acc_r,
                                int64_t ld, int64_t nt, double inv_p, double inv_p2,
                                void *gx, void *gy, void *gz, double *pot_a, double *pot_r,
                                hipStream_t s);

// Deterministic double sums of n values at x (stride 1), two series at once:
// out[0] = sum x0, out[1] = sum x1.  Uses `partials` (reduce_partials_size(n) doubles).
int64_t reduce_partials_size(int64_t n);
hipError_t launch_sum2(const double *x0, const double *x1, int64_t n, double *partials,
                       double *out, hipStream_t s);
// out[0] = sum_u w[u]*x[u]
hipError_t launch_wsum(const void *w, int precision, const double *x, int64_t n,
                       double *partials, double *out, hipStream_t s);

// Voxel-centre coordinates of cells v0 .. v0+n-1 of the G^3 grid (x fastest)
// into cx, cy, cz[0 .. n-1] (precision type).
hipError_t launch_cell_centres(int precision, int64_t G, double L, int64_t v0, int64_t n,
                               void *cx, void *cy, void *cz, hipStream_t s);

// Grid attraction: node coordinates (G+2 per axis), packing of node sums into
// the [n][4] field, and the trilinear interpolant writing the four attraction
// sums of targets [t0, t0+nt) into acc rows (like a cell sweep would).
// Node coordinates of nodes n0 .. n0+n-1 into nx, ny, nz[0 .. n-1]; packing of
// acc rows 0 .. n-1 into field nodes n0 .. n0+n-1.
// Node field by FP64 FFT convolution (fftfield.hip): workspace bytes, 0 when
// the grid is too large for it (2G + 1 > 512).
size_t field_fft_bytes(int64_t G);
hipError_t launch_field_fft(int precision, int kern, int64_t G, double L, double eps,
                            const void *rho, void *field, void *ws, hipStream_t s);
hipError_t launch_node_coords(int precision, int64_t G, double L, int64_t n0, int64_t n, void *nx,
                              void *ny, void *nz, hipStream_t s);
hipError_t launch_field_pack(int precision, const double *acc, int64_t ld, int64_t n0, int64_t n,
                             void *field, hipStream_t s);
hipError_t launch_interpolate(int precision, const void *kx, const void *ky, const void *kz,
                              int64_t t0, int64_t nt, int64_t G, double L, const void *field,
                              double *acc, int64_t ld, hipStream_t s);

// Step helpers.  K = {kx, ky, kz} (p each), k_prev/g_prev/g laid out [3][p].
// out[0] = sum (K - k_prev)^2, out[1] = sum (K - k_prev) (g - g_prev).
hipError_t launch_bb_dots(int precision, const void *kx, const void *ky, const void *kz,
                          const void *k_prev, const void *g, const void *g_prev, int64_t p,
                          double *partials, double *out, hipStream_t s);
// k_prev = K; g_prev = g; K = K - eta * g (computed in double).
hipError_t launch_axpy_save(int precision, void *kx, void *ky, void *kz, void *k_prev,
                            const void *g, void *g_prev, int64_t p, double eta,
                            const double *eta_dev, hipStream_t s);
// info[0] = eta, info[1..3] = F, F^a, F^r, info[8] = BB used, info[9] = 0, from the
// energy sums scal[0..1] and (bb) the dots scal[2..3]; eta is NaN when F is not finite.
hipError_t launch_step_policy(const double *scal, int64_t p, double eta_fixed, bool bb,
                              double *info, hipStream_t s);

// Dyadic linear up-sampling: coarse shots of N samples -> fine shots of 2N.
hipError_t launch_upsample(int precision, const void *kx, const void *ky, const void *kz, void *fx,
                           void *fy, void *fz, int64_t Nc, int64_t N, hipStream_t s);

// Projection and constraint check (one block per shot).  per_axis selects the
// per-axis maximum instead of the Euclidean norm in the speed and slew bounds.
// gate (nullable, device): a NaN there skips the projection (a step not taken).
// duals (nullable, device): [n_shots][6][n_samples] warm-start state, in/out.
hipError_t launch_project(int precision, void *kx, void *ky, void *kz, int64_t n_shots,
                          int64_t n_samples, double L, double a, double b, int64_t te,
                          int n_pit, bool per_axis, const double *gate, double *duals,
                          hipStream_t s);
// per_shot: n_shots*4 doubles; out: 4 doubles.
hipError_t launch_constraint_check(int precision, const void *kx, const void *ky, const void *kz,
                                   int64_t n_shots, int64_t n_samples, double L, double a,
                                   double b, int64_t te, bool per_axis, double *per_shot,
                                   double *out, hipStream_t s);

// Issue-rate probe of the repulsion pair's instruction mix (probe.hip).
// variant 0: the pair's 10 FP32 instructions + v_rsq_f32; 1: without the
// reciprocal square root; 2: reciprocal square roots (and one add each) alone.
// out: probe_out_elements(blocks) floats; each launch runs probe_pairs() pairs.
int64_t probe_out_elements(int64_t blocks);
int64_t probe_pairs(int64_t blocks, int iters);
hipError_t launch_pair_mix_probe(int variant, float *out, int64_t blocks, int iters,
                                 hipStream_t s);

// Repulsion potential rows from the forces: acc[3*ld + t] = 2 K[t0+t] . acc[0..2][t]
// for t in [0, nt) (in double; their sum over all targets is the pair sum of
// |K[i] - K[j]| when H = |d|).
hipError_t launch_force_potential(int precision, const void *kx, const void *ky, const void *kz,
                                  int64_t t0, int64_t nt, double *acc, int64_t ld,
                                  hipStream_t s);

}  // namespace spk
