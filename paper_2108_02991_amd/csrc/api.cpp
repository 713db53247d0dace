// Host side of libsparkling.so: argument validation, sweep planning,
// workspace layout, launch sequencing, kernel timing and the C entry points
// declared in sparkling.h.

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "spk_internal.h"

namespace {

using namespace spk;

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int device_fail(hipError_t e, const char *where)
{
    return fail(SPK_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define SPK_HIP(expr, where)                     \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess)                    \
            return device_fail(e_, where);       \
    } while (0)

// ------------------------------------------------------------------------
// Kernel timing (process-global, mutex-guarded).
// ------------------------------------------------------------------------
struct TimedLaunch {
    hipEvent_t a, b;
    int kind;
    double pairs;
};

std::mutex g_tmu;
bool g_timing = false;
// Set for the duration of an allocation-free call: its launches are not timed
// (timing creates events).
thread_local bool t_untimed = false;
std::vector<TimedLaunch> g_pending;
constexpr int kKinds = 5;
double g_ms[kKinds] = {};
int64_t g_launches[kKinds] = {};
double g_pairs[kKinds] = {};

// A roctx range around one entry point (seen by rocprofv3 --marker-trace; a
// no-op without a profiler).  None inside an allocation-free call.
class Range {
  public:
    explicit Range(const char *name) : on_(!t_untimed)
    {
        if (on_)
            roctxRangePushA(name);
    }
    ~Range()
    {
        if (on_)
            roctxRangePop();
    }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;

  private:
    bool on_;
};

// Brackets one launch with events when timing is on.
class Timed {
  public:
    Timed(int kind, double pairs, hipStream_t s) : kind_(kind), pairs_(pairs), s_(s)
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        if (!g_timing || t_untimed)
            return;
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s_, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
            return;
        if (hipEventCreate(&a_) != hipSuccess)
            return;
        if (hipEventCreate(&b_) != hipSuccess) {
            hipEventDestroy(a_);
            return;
        }
        on_ = hipEventRecord(a_, s_) == hipSuccess;
        if (!on_) {
            hipEventDestroy(a_);
            hipEventDestroy(b_);
        }
    }
    ~Timed()
    {
        if (!on_)
            return;
        std::lock_guard<std::mutex> lk(g_tmu);
        if (hipEventRecord(b_, s_) == hipSuccess) {
            g_pending.push_back({a_, b_, kind_, pairs_});
        } else {
            hipEventDestroy(a_);
            hipEventDestroy(b_);
        }
    }
    Timed(const Timed &) = delete;
    Timed &operator=(const Timed &) = delete;

  private:
    int kind_;
    double pairs_;
    hipStream_t s_;
    hipEvent_t a_{}, b_{};
    bool on_ = false;
};

// ------------------------------------------------------------------------
// Parameters and planning.
// ------------------------------------------------------------------------
size_t elt_size(int precision) { return precision == SPK_PLAIN_FP64 ? 8 : 4; }

int check_params(const spk_params *prm, bool need_projection)
{
    if (!prm)
        return fail(SPK_EINVAL, "params is NULL");
    if (prm->n_shots < 1)
        return fail(SPK_EINVAL, "n_shots must be >= 1 (got %lld)", (long long)prm->n_shots);
    if (prm->n_samples < 1)
        return fail(SPK_EINVAL, "n_samples must be >= 1 (got %lld)", (long long)prm->n_samples);
    if (prm->n_shots > ((int64_t(1) << 31) - 1) / prm->n_samples)
        return fail(SPK_EINVAL, "p = n_shots * n_samples must stay below 2^31");
    if (prm->grid < 1 || prm->grid > kMaxGrid)
        return fail(SPK_EINVAL, "grid must be in [1, %lld] (got %lld)", (long long)kMaxGrid,
                    (long long)prm->grid);
    if (prm->precision < SPK_PLAIN_FP64 || prm->precision > SPK_FP32_ACC64)
        return fail(SPK_EINVAL, "unknown precision %d", prm->precision);
    if (!(prm->half_width > 0.0) || !std::isfinite(prm->half_width))
        return fail(SPK_EINVAL, "half_width must be finite and > 0");
    if (!(prm->eps >= 0.0) || !std::isfinite(prm->eps))
        return fail(SPK_EINVAL, "eps must be finite and >= 0");
    if (!(prm->eps * prm->eps <= (prm->precision == SPK_PLAIN_FP64 ? DBL_MAX : FLT_MAX) / 4))
        return fail(SPK_EINVAL, "eps^2 must stay finite in the form's type");
    if (prm->te_index < -1 || prm->te_index >= prm->n_samples)
        return fail(SPK_EINVAL, "te_index must be -1 or in [0, n_samples)");
    if (prm->flags & ~(SPK_FLAG_DISCREPANCY | SPK_FLAG_ROTATION_VARIANT | SPK_FLAG_LOG_KERNEL |
                       SPK_FLAG_FIELD_DIRECT | SPK_FLAG_ENERGY_FROM_FORCE))
        return fail(SPK_EINVAL, "unknown flags 0x%x", prm->flags);
    if ((prm->flags & SPK_FLAG_ENERGY_FROM_FORCE) &&
        (prm->eps != 0.0 || (prm->flags & SPK_FLAG_LOG_KERNEL) || prm->far_field_depth != 0))
        return fail(SPK_EINVAL, "the energy from the forces needs the distance kernel with "
                                "eps = 0 and the exact repulsion");
    if (prm->flags & SPK_FLAG_LOG_KERNEL) {
        if (prm->precision != SPK_PLAIN_FP64 && prm->precision != SPK_FP32_COMP)
            return fail(SPK_EUNSUPPORTED, "the log kernel runs in the plain_fp64 and fp32_comp "
                                          "forms only");
        const double tiny = prm->precision == SPK_PLAIN_FP64 ? DBL_MIN : FLT_MIN;
        if (!(prm->eps * prm->eps >= tiny))
            return fail(SPK_EINVAL, "the log kernel needs eps > 0 with eps^2 >= %g", tiny);
    }
    if (prm->far_field_depth != 0) {
        if (prm->far_field_depth < 2 || prm->far_field_depth > kFmmMaxDepth)
            return fail(SPK_EINVAL, "far_field_depth must be 0 or in [2, %d]", kFmmMaxDepth);
        if (prm->far_field_order < kFmmMinOrder || prm->far_field_order > kFmmMaxOrder)
            return fail(SPK_EINVAL, "far_field_order must be in [%d, %d]", kFmmMinOrder,
                        kFmmMaxOrder);
        if (prm->precision != SPK_PLAIN_FP64 && prm->precision != SPK_FP32_COMP)
            return fail(SPK_EUNSUPPORTED, "the far field runs in the plain_fp64 and fp32_comp "
                                          "forms only");
        if (prm->far_field_adaptive < 0 || prm->far_field_adaptive > kMaxRefine)
            return fail(SPK_EINVAL, "far_field_adaptive must be in [0, %d]", kMaxRefine);
        if (prm->far_field_depth + prm->far_field_adaptive > kFmmMaxDepth)
            return fail(SPK_EINVAL, "far_field_depth + far_field_adaptive must be <= %d",
                        kFmmMaxDepth);
    } else if (prm->far_field_adaptive != 0) {
        return fail(SPK_EINVAL, "far_field_adaptive needs far_field_depth > 0");
    }
    if (prm->attraction_field &&
        reinterpret_cast<uintptr_t>(prm->attraction_field) % (4 * elt_size(prm->precision)))
        return fail(SPK_EINVAL, "attraction_field is not %zu-byte aligned",
                    4 * elt_size(prm->precision));
    if (need_projection) {
        if (prm->n_samples < 2)
            return fail(SPK_EINVAL, "projection needs n_samples >= 2");
        if (prm->n_samples > kMaxProjectSamples)
            return fail(SPK_EUNSUPPORTED, "projection supports n_samples <= %lld",
                        (long long)kMaxProjectSamples);
        if (!(prm->a_max > 0.0) || !(prm->b_max > 0.0) || !std::isfinite(prm->a_max) ||
            !std::isfinite(prm->b_max))
            return fail(SPK_EINVAL, "a_max and b_max must be finite and > 0");
        if (prm->n_pit < 0)
            return fail(SPK_EINVAL, "n_pit must be >= 0");
        if (reinterpret_cast<uintptr_t>(prm->proj_duals) % 8)
            return fail(SPK_EINVAL, "proj_duals is not 8-byte aligned");
    }
    return SPK_OK;
}

int check_ptr(const void *ptr, const char *name, size_t align)
{
    if (!ptr)
        return fail(SPK_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(ptr) % align)
        return fail(SPK_EINVAL, "%s is not %zu-byte aligned", name, align);
    return SPK_OK;
}

// Slab decomposition of one sweep.  Depends only on the total target count
// p_total, the source count and the precision, never on the target range of a
// call, which is what makes every chunking produce bit-identical rows.
struct Plan {
    int64_t slab = 1;        // sources (samples or cell rows) per slab
    int64_t nslab = 1;
    int64_t per_launch = 1;  // slabs per launch
    int64_t unit = 1;        // pair interactions per source and target
};

// Pair interactions of one slab at most (~0.25-0.5 s at full rate), and of one
// launch, whose grid's y extent holds several slabs: each launch ends with a
// few milliseconds in which its last blocks drain, so four slabs per launch
// save most of that against one (the partials then hold four slabs).
constexpr double kMaxPairsPerSlab = 1099511627776.0;   // 2^40
constexpr double kMaxPairsPerLaunch = 4.0 * kMaxPairsPerSlab;
// Slabs are grouped only while one launch's partials (32 B per target and
// slab) stay within this, so that very large problems keep one slab per
// launch and a workspace of about 100 B per sample.
constexpr double kMaxGroupedPartialBytes = 1073741824.0;   // 2^30
// Blocks a launch should have to fill 256 CUs several times over.
constexpr int64_t kWantBlocks = 2048;
// Slabs one launch may carry (the grid's y extent).
constexpr int64_t kMaxSlabsPerLaunch = 65535;

Plan make_plan(int precision, bool cells, int64_t p_total, int64_t n_src, int64_t G)
{
    Plan pl;
    pl.unit = cells ? G : 1;
    const int64_t tpb = sweep_targets_per_block(precision);
    const int64_t tb = (p_total + tpb - 1) / tpb;
    const int64_t gran = cells ? std::max<int64_t>(1, (precision == SPK_PLAIN_FP64 ? kCellTileF64
                                                                                  : kCellTileF32) / G)
                               : kSampleTile;
    const double max_pairs = precision == SPK_PLAIN_FP64 ? kMaxPairsPerSlab / 2 : kMaxPairsPerSlab;
    const double max_launch =
        precision == SPK_PLAIN_FP64 ? kMaxPairsPerLaunch / 2 : kMaxPairsPerLaunch;
    const int64_t nslab_par = std::max<int64_t>(1, (kWantBlocks + tb - 1) / tb);
    int64_t slab = (n_src + nslab_par - 1) / nslab_par;
    const double per_src = (double)p_total * (double)pl.unit;
    const int64_t slab_time = std::max<int64_t>(1, (int64_t)(max_pairs / per_src));
    slab = std::min(slab, slab_time);
    slab = (slab + gran - 1) / gran * gran;
    slab = std::max<int64_t>(slab, gran);
    pl.slab = slab;
    pl.nslab = (n_src + slab - 1) / slab;
    const int64_t fit = (int64_t)(max_launch / (per_src * (double)slab));
    const int64_t room = (int64_t)(kMaxGroupedPartialBytes / (32.0 * (double)p_total));
    pl.per_launch = std::max<int64_t>(1, std::min({pl.nslab, fit, room, kMaxSlabsPerLaunch}));
    return pl;
}

// Workspace layout (offsets from a 256-byte aligned base).
struct Layout {
    size_t acc_a = 0, acc_r = 0, part = 0, red = 0, scal = 0, grad = 0, viol = 0, cells = 0;
    size_t chunk_sums = 0, info = 0;
    // far field (only with far_field_depth > 0)
    size_t fmm_box_part = 0, fmm_box = 0, fmm_keys_in = 0, fmm_keys_out = 0, fmm_vals_in = 0,
           fmm_vals_out = 0, fmm_xs = 0, fmm_start = 0,
           fmm_temp = 0, fmm_temp_bytes = 0, fmm_A = 0, fmm_Tm = 0, fmm_Tu = 0, fmm_Td = 0,
           fmm_part = 0;
    size_t fmm_chunks_q[kMaxRefine + 1] = {}, fmm_chunk_start_q[kMaxRefine + 1] = {},
           fmm_refined[kMaxRefine] = {}, fmm_tmask[kMaxRefine + 1] = {},
           fmm_tflag[kMaxRefine + 1] = {}, fmm_tscan[kMaxRefine + 1] = {},
           fmm_tlist[kMaxRefine + 1] = {};
    size_t fmm_W[kFmmMaxDepth + 1] = {}, fmm_L[kFmmMaxDepth + 1] = {},
           fmm_occ[kFmmMaxDepth + 1] = {};
    size_t total = 0;
    int64_t ld = 0;
    int64_t part_rows = 0;   // capacity of the slab partials, in rows of 4 doubles
};

// Targets per pass of the sweeps whose targets are grid points (the node
// field, the cell centres of the self-energy), so that the accumulators
// stay at max(p, this) rows however large the grid is.
constexpr int64_t kGridTargetChunk = int64_t(1) << 21;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int64_t field_nodes(int64_t G) { return (G + 2) * (G + 2) * (G + 2); }

Layout make_layout(const spk_params *prm)
{
    Layout L;
    const int64_t p = prm->n_shots * prm->n_samples;
    const int64_t G = prm->grid, M = G * G * G, Mn = field_nodes(G);
    const bool disc = prm->flags & SPK_FLAG_DISCREPANCY;
    // targets of one sweep call: the samples, or one pass of field nodes
    // (which also covers a pass of cell centres of the self-energy, M < Mn)
    const int64_t cn = std::min(Mn, kGridTargetChunk), cm = std::min(M, kGridTargetChunk);
    const int64_t nt = std::max(p, cn);
    // slab partials: targets of a call times the slabs of one launch, per sweep kind
    const Plan pr = make_plan(prm->precision, false, p, p, G);
    const Plan pa = make_plan(prm->precision, true, p, G * G, G);
    int64_t part_rows = p * std::max(pr.per_launch, pa.per_launch);
    part_rows = std::max(part_rows, cn * make_plan(prm->precision, true, Mn, G * G, G).per_launch);
    if (disc)
        part_rows = std::max(part_rows,
                             cm * make_plan(prm->precision, true, M, G * G, G).per_launch);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.ld = nt;
    L.acc_a = take(sizeof(double) * 4 * nt);
    L.acc_r = take(sizeof(double) * 4 * nt);
    L.part = take(sizeof(double) * 4 * part_rows);
    L.part_rows = part_rows;
    L.red = take(sizeof(double) * reduce_partials_size(std::max(nt, 3 * p)));
    L.scal = take(sizeof(double) * 16);
    L.info = take(sizeof(double) * 16);
    L.grad = take(elt_size(prm->precision) * 3 * p);
    L.viol = take(sizeof(double) * 4 * prm->n_shots);
    L.cells = take(elt_size(prm->precision) * 3 * cn);
    L.chunk_sums = take(sizeof(double) * ((M + kGridTargetChunk - 1) / kGridTargetChunk));
    if (prm->far_field_depth > 0) {
        const int D = prm->far_field_depth, n = prm->far_field_order;
        const int R = prm->far_field_adaptive, F = D + R;   // deepest level
        const size_t n3 = (size_t)n * n * n;
        const int64_t ncells = int64_t(1) << (3 * F);
        auto cells_at = [&](int q) { return int64_t(1) << (3 * (D + q)); };
        L.fmm_box_part = take(sizeof(double) * 6 * kFmmBoxBlocks);
        L.fmm_box = take(sizeof(double) * 4);
        L.fmm_keys_in = take(sizeof(uint32_t) * p);
        L.fmm_keys_out = take(sizeof(uint32_t) * p);
        L.fmm_vals_in = take(sizeof(uint32_t) * p);
        L.fmm_vals_out = take(sizeof(uint32_t) * p);
        L.fmm_xs = take(elt_size(prm->precision) * 3 * p);
        L.fmm_start = take(sizeof(int32_t) * (ncells + 1));
        for (int q = 0; q <= R; ++q) {
            L.fmm_chunks_q[q] = take(sizeof(int32_t) * (cells_at(q) + 1));
            L.fmm_chunk_start_q[q] = take(sizeof(int32_t) * (cells_at(q) + 1));
        }
        for (int q = 0; q < R; ++q)
            L.fmm_refined[q] = take(sizeof(int32_t) * cells_at(q));
        for (int q = 1; q <= R; ++q) {
            L.fmm_tmask[q] = take(sizeof(int32_t) * fmm_level_cells(D + q));
            L.fmm_tflag[q] = take(sizeof(int32_t) * (cells_at(q) + 1));
            L.fmm_tscan[q] = take(sizeof(int32_t) * (cells_at(q) + 1));
            L.fmm_tlist[q] = take(sizeof(int32_t) * cells_at(q));
        }
        L.fmm_temp_bytes = fmm_sort_temp_bytes(p, F);
        L.fmm_temp = take(L.fmm_temp_bytes);
        for (int l = 2; l <= F; ++l) {
            L.fmm_W[l] = take(sizeof(double) * fmm_level_cells(l) * n3);
            L.fmm_L[l] = take(sizeof(double) * fmm_level_cells(l) * 4 * n3);
            L.fmm_occ[l] = take(sizeof(int32_t) * fmm_level_cells(l));
        }
        L.fmm_A = take(sizeof(double) * fmm_table_doubles(prm->far_field_order) * (F - 1));
        L.fmm_Tm = take(sizeof(double) * 8 * n3 * n3);
        L.fmm_Tu = take(sizeof(double) * fmm_trans_doubles(n));
        L.fmm_Td = take(sizeof(double) * fmm_trans_doubles(n));
        L.fmm_part = take(sizeof(double) * fmm_split_doubles(n, F));
    }
    L.total = off + 256;   // slack for aligning the caller's base pointer
    return L;
}

struct Ws {
    char *base;
    Layout L;
    double *acc_a() const { return reinterpret_cast<double *>(base + L.acc_a); }
    double *acc_r() const { return reinterpret_cast<double *>(base + L.acc_r); }
    double *part() const { return reinterpret_cast<double *>(base + L.part); }
    double *red() const { return reinterpret_cast<double *>(base + L.red); }
    double *chunk_sums() const { return reinterpret_cast<double *>(base + L.chunk_sums); }
    double *scal() const { return reinterpret_cast<double *>(base + L.scal); }
    double *info() const { return reinterpret_cast<double *>(base + L.info); }
    template <typename P> P *at(size_t off) const { return reinterpret_cast<P *>(base + off); }
    void *grad() const { return base + L.grad; }
    double *viol() const { return reinterpret_cast<double *>(base + L.viol); }
    void *cells() const { return base + L.cells; }
};

int bind_ws(const spk_params *prm, void *ws, size_t ws_bytes, Ws *out)
{
    out->L = make_layout(prm);
    if (!ws || ws_bytes < out->L.total)
        return fail(SPK_EWORKSPACE, "workspace needs %zu bytes (got %zu%s)", out->L.total,
                    ws_bytes, ws ? "" : ", NULL");
    uintptr_t b = reinterpret_cast<uintptr_t>(ws);
    out->base = reinterpret_cast<char *>((b + 255) / 256 * 256);
    return SPK_OK;
}

// Sweeps every target in [t0, t0 + nt) against one source set, accumulating
// the four sums into acc (rows of length ld).  p_total fixes the plan.
int run_sweep(const spk_params *prm, bool cells, const void *tx, const void *ty, const void *tz,
              int64_t t0, int64_t nt, int64_t p_total, const void *sx, const void *sy,
              const void *sz, const void *rho, bool energy, const Ws &w, double *acc,
              hipStream_t s)
{
    const int64_t G = prm->grid;
    const int64_t n_src = cells ? G * G : prm->n_shots * prm->n_samples;
    const Plan pl = make_plan(prm->precision, cells, p_total, n_src, G);
    SweepLaunch l;
    l.precision = prm->precision;
    l.kernel = (prm->flags & SPK_FLAG_LOG_KERNEL) ? kKernelLog : kKernelDistance;
    l.energy = energy;
    l.tx = tx;
    l.ty = ty;
    l.tz = tz;
    l.t0 = t0;
    l.nt = nt;
    l.sx = sx;
    l.sy = sy;
    l.sz = sz;
    l.rho = rho;
    l.grid = G;
    l.half_width = prm->half_width;
    l.eps = prm->eps;
    l.slab = pl.slab;
    l.src_end = n_src;
    l.part = w.part();
    l.ld = nt;   // the slab partials of this call: [slab][4][nt]
    const int kind = cells ? SPK_KIND_ATTRACTION : SPK_KIND_REPULSION;
    // Slab boundaries depend on p_total only.  A call with few targets groups
    // more slabs per launch (bounded by the partial buffer, the pairs of one
    // launch and the grid's y extent); the combine still adds every target's
    // slabs in slab order, so the grouping does not change any result bit.
    int64_t per_launch = pl.per_launch;
    if (nt > 0) {
        const double max_pairs =
            prm->precision == SPK_PLAIN_FP64 ? kMaxPairsPerLaunch / 2 : kMaxPairsPerLaunch;
        int64_t more = std::min<int64_t>(pl.nslab, w.L.part_rows / nt);
        more = std::min<int64_t>(
            more, std::max<int64_t>(1, (int64_t)(max_pairs / ((double)nt * (double)pl.slab *
                                                              (double)pl.unit))));
        more = std::min<int64_t>(more, kMaxSlabsPerLaunch);
        per_launch = std::max(per_launch, more);
    }
    bool first = true;
    for (int64_t s0 = 0; s0 < pl.nslab; s0 += per_launch) {
        l.src_begin = s0 * pl.slab;
        l.nslabs = (int)std::min<int64_t>(per_launch, pl.nslab - s0);
        const int64_t src_hi = std::min<int64_t>(n_src, (s0 + l.nslabs) * pl.slab);
        const double pairs = (double)nt * (double)(src_hi - l.src_begin) * (double)pl.unit;
        {
            Timed tm(kind, pairs, s);
            hipError_t e = cells ? launch_sweep_cells(l, s) : launch_sweep_samples(l, s);
            if (e != hipSuccess)
                return device_fail(e, cells ? "cell sweep launch" : "sample sweep launch");
        }
        {
            Timed tm(SPK_KIND_OTHER, 0.0, s);
            SPK_HIP(launch_combine(acc, w.L.ld, w.part(), nt, l.nslabs, nt, first, s), "combine");
        }
        first = false;
    }
    return SPK_OK;
}

// The repulsion sums of targets [t0, t0+nt) by the far-field method.
int run_far_field(const spk_params *prm, const void *kx, const void *ky, const void *kz,
                  int64_t t0, int64_t nt, bool energy, const Ws &w, hipStream_t s)
{
    const Layout &L = w.L;
    const int64_t p = prm->n_shots * prm->n_samples;
    FmmLaunch f;
    f.precision = prm->precision;
    f.kernel = (prm->flags & SPK_FLAG_LOG_KERNEL) ? kKernelLog : kKernelDistance;
    f.energy = energy;
    f.depth = prm->far_field_depth;
    f.order = prm->far_field_order;
    f.adaptive = prm->far_field_adaptive;
    f.x = kx;
    f.y = ky;
    f.z = kz;
    f.p = p;
    f.t0 = t0;
    f.nt = nt;
    f.eps = prm->eps;
    f.acc = w.acc_r();
    f.ld = L.ld;
    f.near_tpb = near_targets_per_block(prm->precision);
    f.side = static_cast<hipStream_t>(prm->far_field_stream);
    f.box_part = w.at<double>(L.fmm_box_part);
    f.box = w.at<double>(L.fmm_box);
    f.keys_in = w.at<uint32_t>(L.fmm_keys_in);
    f.keys_out = w.at<uint32_t>(L.fmm_keys_out);
    f.vals_in = w.at<uint32_t>(L.fmm_vals_in);
    f.vals_out = w.at<uint32_t>(L.fmm_vals_out);
    char *xs = w.at<char>(L.fmm_xs);
    const size_t al = elt_size(prm->precision);
    f.xs = xs;
    f.ys = xs + al * p;
    f.zs = xs + 2 * al * p;
    f.start = w.at<int32_t>(L.fmm_start);
    for (int q = 0; q <= f.adaptive; ++q) {
        f.chunks[q] = w.at<int32_t>(L.fmm_chunks_q[q]);
        f.chunk_start[q] = w.at<int32_t>(L.fmm_chunk_start_q[q]);
    }
    for (int q = 0; q < f.adaptive; ++q)
        f.refined[q] = w.at<int32_t>(L.fmm_refined[q]);
    for (int q = 1; q <= f.adaptive; ++q) {
        f.tmask[q] = w.at<int32_t>(L.fmm_tmask[q]);
        f.tflag[q] = w.at<int32_t>(L.fmm_tflag[q]);
        f.tscan[q] = w.at<int32_t>(L.fmm_tscan[q]);
        f.tlist[q] = w.at<int32_t>(L.fmm_tlist[q]);
    }
    f.temp = w.at<char>(L.fmm_temp);
    f.temp_bytes = L.fmm_temp_bytes;
    for (int l = 2; l <= f.depth + f.adaptive; ++l) {
        f.W[l] = w.at<double>(L.fmm_W[l]);
        f.L[l] = w.at<double>(L.fmm_L[l]);
        f.occ[l] = w.at<int32_t>(L.fmm_occ[l]);
    }
    f.A = w.at<double>(L.fmm_A);
    f.Tm = w.at<double>(L.fmm_Tm);
    f.Tu = w.at<double>(L.fmm_Tu);
    f.Td = w.at<double>(L.fmm_Td);
    f.part = w.at<double>(L.fmm_part);
    Timed tm(SPK_KIND_REPULSION, 0.0, s);
    SPK_HIP(launch_fmm_repulsion(f, s), "far-field repulsion");
    return SPK_OK;
}

// Both sweeps for targets [t0, t0+nt) of K; results in w.acc_a() / w.acc_r().
int run_gradient_sums(const spk_params *prm, const void *kx, const void *ky, const void *kz,
                      const void *rho, int64_t t0, int64_t nt, bool energy, const Ws &w,
                      hipStream_t s)
{
    const int64_t p = prm->n_shots * prm->n_samples;
    // with the energy from the forces the sweep skips its per-pair distances,
    // and each target's repulsion potential row holds 2 K[i] . G[i], whose sum
    // over all targets is the sum over all pairs of |K[i] - K[j]|
    const bool from_force = energy && (prm->flags & SPK_FLAG_ENERGY_FROM_FORCE);
    int rc = prm->far_field_depth > 0
                 ? run_far_field(prm, kx, ky, kz, t0, nt, energy, w, s)
                 : run_sweep(prm, false, kx, ky, kz, t0, nt, p, kx, ky, kz, nullptr,
                             energy && !from_force, w, w.acc_r(), s);
    if (rc)
        return rc;
    if (from_force) {
        Timed tm(SPK_KIND_OTHER, 0.0, s);
        SPK_HIP(launch_force_potential(prm->precision, kx, ky, kz, t0, nt, w.acc_r(), w.L.ld, s),
                "energy from the forces");
    }
    if (prm->attraction_field) {
        Timed tm(SPK_KIND_INTERPOLATION, (double)nt, s);
        SPK_HIP(launch_interpolate(prm->precision, kx, ky, kz, t0, nt, prm->grid, prm->half_width,
                                   prm->attraction_field, w.acc_a(), w.L.ld, s),
                "field interpolation");
        return SPK_OK;
    }
    return run_sweep(prm, true, kx, ky, kz, t0, nt, p, nullptr, nullptr, nullptr, rho, energy, w,
                     w.acc_a(), s);
}

// Energy sums of the potentials in acc rows 3 into scal[0] (attraction) and scal[1].
int reduce_energy(const Ws &w, int64_t nt, hipStream_t s)
{
    Timed tm(SPK_KIND_OTHER, 0.0, s);
    SPK_HIP(launch_sum2(w.acc_a() + 3 * w.L.ld, w.acc_r() + 3 * w.L.ld, nt, w.red(), w.scal(), s),
            "energy reduction");
    return SPK_OK;
}

void energies_from_sums(int64_t p, const double sums[2], double out[3])
{
    const double fa = sums[0] / (double)p;
    const double fr = sums[1] / (2.0 * (double)p * (double)p);
    out[0] = fa - fr;
    out[1] = fa;
    out[2] = fr;
}

int check_k(const spk_params *prm, const void *kx, const void *ky, const void *kz)
{
    const size_t al = elt_size(prm->precision);
    int rc;
    if ((rc = check_ptr(kx, "kx", al)) || (rc = check_ptr(ky, "ky", al)) ||
        (rc = check_ptr(kz, "kz", al)))
        return rc;
    return SPK_OK;
}

int constraint_check_into(const spk_params *prm, const void *kx, const void *ky, const void *kz,
                          const Ws &w, double *dev_out, hipStream_t s)
{
    Timed tm(SPK_KIND_OTHER, 0.0, s);
    SPK_HIP(launch_constraint_check(prm->precision, kx, ky, kz, prm->n_shots, prm->n_samples,
                                    prm->half_width, prm->a_max, prm->b_max, prm->te_index,
                                    (prm->flags & SPK_FLAG_ROTATION_VARIANT) != 0, w.viol(),
                                    dev_out, s),
            "constraint check");
    return SPK_OK;
}

int project_in_place(const spk_params *prm, void *kx, void *ky, void *kz, hipStream_t s,
                     const double *gate = nullptr)
{
    Timed tm(SPK_KIND_PROJECTION, 0.0, s);
    SPK_HIP(launch_project(prm->precision, kx, ky, kz, prm->n_shots, prm->n_samples,
                           prm->half_width, prm->a_max, prm->b_max, prm->te_index, prm->n_pit,
                           (prm->flags & SPK_FLAG_ROTATION_VARIANT) != 0, gate,
                           static_cast<double *>(prm->proj_duals), s),
            "projection");
    return SPK_OK;
}

int copy_to_host(double *dst, const double *src, size_t n, hipStream_t s)
{
    SPK_HIP(hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToHost, s), "copy to host");
    SPK_HIP(hipStreamSynchronize(s), "stream synchronize");
    return SPK_OK;
}

// Argument checks shared by the two step entry points.
int check_step(const spk_params *prm, void *kx, void *ky, void *kz, const void *rho,
               void *k_prev, void *g_prev, int64_t iter, double eta_fixed, void *ws,
               size_t ws_bytes, Ws *w)
{
    int rc = check_params(prm, true);
    if (rc)
        return rc;
    const size_t al = elt_size(prm->precision);
    if ((rc = check_k(prm, kx, ky, kz)) || (rc = check_ptr(rho, "rho", al)) ||
        (rc = check_ptr(k_prev, "k_prev", al)) || (rc = check_ptr(g_prev, "g_prev", al)))
        return rc;
    if (iter < 0 || !(eta_fixed > 0.0) || !std::isfinite(eta_fixed))
        return fail(SPK_EINVAL, "iter must be >= 0 and eta_fixed finite and > 0");
    return bind_ws(prm, ws, ws_bytes, w);
}

// First half of a step: gradient into the workspace, energy sums, the
// Barzilai-Borwein dots (iter >= 20) and the step-size rule, all on the
// device; info_dev[0..3] = eta, F, F^a, F^r and info_dev[8] = BB used.
int enqueue_step_front(const spk_params *prm, void *kx, void *ky, void *kz, const void *rho,
                       void *k_prev, void *g_prev, int64_t iter, double eta_fixed,
                       double *info_dev, const Ws &w, hipStream_t s)
{
    const int64_t p = prm->n_shots * prm->n_samples;
    const size_t al = elt_size(prm->precision);
    char *g = static_cast<char *>(w.grad());
    int rc = run_gradient_sums(prm, kx, ky, kz, rho, 0, p, true, w, s);
    if (rc)
        return rc;
    Timed tm(SPK_KIND_OTHER, 0.0, s);
    const double inv_p = 1.0 / (double)p, inv_p2 = 1.0 / ((double)p * (double)p);
    SPK_HIP(launch_finalize_grad(prm->precision, w.acc_a(), w.acc_r(), w.L.ld, p, inv_p, inv_p2,
                                 g, g + al * p, g + 2 * al * p, nullptr, nullptr, s),
            "finalize gradient");
    if ((rc = reduce_energy(w, p, s)))
        return rc;
    const bool bb = iter >= 20;
    if (bb)
        SPK_HIP(launch_bb_dots(prm->precision, kx, ky, kz, k_prev, g, g_prev, p, w.red(),
                               w.scal() + 2, s),
                "step dots");
    SPK_HIP(launch_step_policy(w.scal(), p, eta_fixed, bb, info_dev, s), "step size");
    return SPK_OK;
}

// Second half: K <- Pi_Q(K - eta g) with the state saved, both skipped when
// info_dev[0] (eta) is NaN, then the constraint check into info_dev[4..7].
int enqueue_step_back(const spk_params *prm, void *kx, void *ky, void *kz, void *k_prev,
                      void *g_prev, double *info_dev, const Ws &w, hipStream_t s)
{
    const int64_t p = prm->n_shots * prm->n_samples;
    {
        Timed tm(SPK_KIND_OTHER, 0.0, s);
        SPK_HIP(launch_axpy_save(prm->precision, kx, ky, kz, k_prev, w.grad(), g_prev, p, 0.0,
                                 info_dev, s),
                "step update");
    }
    int rc = project_in_place(prm, kx, ky, kz, s, info_dev);
    if (rc)
        return rc;
    return constraint_check_into(prm, kx, ky, kz, w, info_dev + 4, s);
}

}  // namespace

extern "C" {

const char *spk_status_string(int status)
{
    switch (status) {
    case SPK_OK: return "ok";
    case SPK_EINVAL: return "invalid argument";
    case SPK_EWORKSPACE: return "workspace too small";
    case SPK_EDEVICE: return "HIP device error";
    case SPK_EUNSUPPORTED: return "unsupported parameters";
    case SPK_ENONFINITE: return "non-finite energy";
    default: return "unknown status";
    }
}

const char *spk_last_error(void) { return g_err.c_str(); }

int spk_alpha_beta(double gmax, double smax, double raster_dt, double dwell_dt, double fov,
                   double kmax, double gamma_bar, double half_width, double *a_max, double *b_max)
{
    g_err.clear();
    const double in[] = {gmax, smax, raster_dt, dwell_dt, fov, kmax, gamma_bar, half_width};
    for (double v : in)
        if (!(v > 0.0) || !std::isfinite(v))
            return fail(SPK_EINVAL, "spk_alpha_beta: every input must be finite and > 0");
    if (!a_max || !b_max)
        return fail(SPK_EINVAL, "spk_alpha_beta: NULL output");
    const double amplitude_rate = gamma_bar * gmax;       // 1/(m s) reachable by the gradient
    const double nyquist_rate = 1.0 / (fov * dwell_dt);   // 1/(m s) allowed by the ADC
    const double speed = std::min(amplitude_rate, nyquist_rate) / kmax;
    const double slew = gamma_bar * smax / kmax;
    *a_max = speed * raster_dt * half_width;
    *b_max = slew * raster_dt * raster_dt * half_width;
    return SPK_OK;
}

int spk_lipschitz_bound(int64_t p, double eps, double rho_mass, int32_t flags,
                        double *lipschitz)
{
    if (!lipschitz)
        return fail(SPK_EINVAL, "lipschitz is NULL");
    if (p < 1)
        return fail(SPK_EINVAL, "p must be >= 1");
    if (!(eps > 0.0) || !std::isfinite(eps))
        return fail(SPK_EINVAL, "eps must be finite and > 0 (grad F is not Lipschitz at 0)");
    if (!(rho_mass >= 0.0) || !std::isfinite(rho_mass))
        return fail(SPK_EINVAL, "rho_mass must be finite and >= 0");
    const double pd = (double)p;
    if (flags & SPK_FLAG_LOG_KERNEL)
        *lipschitz = std::max(1.0 + rho_mass / 8.0, rho_mass + 1.0 / 8.0) / (pd * eps * eps);
    else
        *lipschitz = std::max(1.0, rho_mass) / (pd * eps);
    return SPK_OK;
}

int spk_workspace_size(const spk_params *prm, size_t *bytes)
{
    g_err.clear();
    int rc = check_params(prm, false);
    if (rc)
        return rc;
    if (!bytes)
        return fail(SPK_EINVAL, "bytes is NULL");
    *bytes = make_layout(prm).total;
    return SPK_OK;
}

int spk_field_workspace_size(const spk_params *prm, size_t *bytes)
{
    g_err.clear();
    int rc = check_params(prm, false);
    if (rc)
        return rc;
    if (!bytes)
        return fail(SPK_EINVAL, "bytes is NULL");
    const size_t fb = (prm->flags & SPK_FLAG_FIELD_DIRECT) ? 0 : field_fft_bytes(prm->grid);
    *bytes = fb ? fb : make_layout(prm).total;
    return SPK_OK;
}

int sparkling_grad(const spk_params *prm, const void *kx, const void *ky, const void *kz,
                   const void *rho, void *gx, void *gy, void *gz, int64_t tgt_begin,
                   int64_t tgt_end, double *pot_a, double *pot_r, double *energy, void *ws,
                   size_t ws_bytes, void *stream)
{
    Range range("sparkling_grad");
    g_err.clear();
    int rc = check_params(prm, false);
    if (rc)
        return rc;
    const int64_t p = prm->n_shots * prm->n_samples;
    const size_t al = elt_size(prm->precision);
    if (tgt_begin < 0 || tgt_end < tgt_begin || tgt_end > p)
        return fail(SPK_EINVAL, "target range [%lld, %lld) outside [0, %lld)",
                    (long long)tgt_begin, (long long)tgt_end, (long long)p);
    if ((rc = check_k(prm, kx, ky, kz)) || (rc = check_ptr(rho, "rho", al)))
        return rc;
    // outputs of an empty range are never touched and may be NULL
    if (tgt_end > tgt_begin &&
        ((rc = check_ptr(gx, "gx", al)) || (rc = check_ptr(gy, "gy", al)) ||
         (rc = check_ptr(gz, "gz", al))))
        return rc;
    if ((pot_a && (rc = check_ptr(pot_a, "pot_a", 8))) || (pot_r && (rc = check_ptr(pot_r, "pot_r", 8))))
        return rc;
    if (pot_r && (prm->flags & SPK_FLAG_ENERGY_FROM_FORCE))
        return fail(SPK_EINVAL, "per-target repulsion potentials are not available with the "
                                "energy from the forces");
    if (energy && (tgt_begin != 0 || tgt_end != p))
        return fail(SPK_EINVAL, "energy needs the full target range [0, p)");
    Ws w;
    if ((rc = bind_ws(prm, ws, ws_bytes, &w)))
        return rc;
    const int64_t nt = tgt_end - tgt_begin;
    if (nt == 0)
        return SPK_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool want_pot = energy || pot_a || pot_r;
    if ((rc = run_gradient_sums(prm, kx, ky, kz, rho, tgt_begin, nt, want_pot, w, s)))
        return rc;
    {
        Timed tm(SPK_KIND_OTHER, 0.0, s);
        const double inv_p = 1.0 / (double)p, inv_p2 = 1.0 / ((double)p * (double)p);
        SPK_HIP(launch_finalize_grad(prm->precision, w.acc_a(), w.acc_r(), w.L.ld, nt, inv_p,
                                     inv_p2, gx, gy, gz, pot_a, pot_r, s),
                "finalize gradient");
    }
    if (energy) {
        if ((rc = reduce_energy(w, nt, s)))
            return rc;
        double sums[2];
        if ((rc = copy_to_host(sums, w.scal(), 2, s)))
            return rc;
        energies_from_sums(p, sums, energy);
    }
    return SPK_OK;
}

int sparkling_field(const spk_params *prm, const void *rho, void *field, void *ws,
                    size_t ws_bytes, void *stream)
{
    Range range("sparkling_field");
    g_err.clear();
    int rc = check_params(prm, false);
    if (rc)
        return rc;
    const size_t al = elt_size(prm->precision);
    if ((rc = check_ptr(rho, "rho", al)) || (rc = check_ptr(field, "field", 4 * al)))
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t G = prm->grid, Mn = field_nodes(G);
    const size_t fb = (prm->flags & SPK_FLAG_FIELD_DIRECT) ? 0 : field_fft_bytes(G);
    if (fb) {
        // FFT convolution in FP64 (its own workspace, spk_field_workspace_size)
        if (!ws)
            return fail(SPK_EINVAL, "workspace is NULL");
        if (ws_bytes < fb)
            return fail(SPK_EWORKSPACE, "workspace of %zu bytes, the FFT field needs %zu", ws_bytes,
                        fb);
        const int kern = (prm->flags & SPK_FLAG_LOG_KERNEL) ? kKernelLog : kKernelDistance;
        Timed tm(SPK_KIND_OTHER, 0.0, s);
        SPK_HIP(launch_field_fft(prm->precision, kern, G, prm->half_width, prm->eps, rho, field,
                                 ws, s),
                "FFT node field");
        return SPK_OK;
    }
    Ws w;
    if ((rc = bind_ws(prm, ws, ws_bytes, &w)))
        return rc;
    const int64_t cap = std::min(Mn, kGridTargetChunk);
    char *pts = static_cast<char *>(w.cells());
    void *nx = pts, *ny = pts + al * cap, *nz = pts + 2 * al * cap;
    spk_params direct = *prm;
    direct.attraction_field = nullptr;
    // passes of at most `cap` nodes; the sweep plan depends on Mn only
    for (int64_t n0 = 0; n0 < Mn; n0 += cap) {
        const int64_t n = std::min(cap, Mn - n0);
        {
            Timed tm(SPK_KIND_OTHER, 0.0, s);
            SPK_HIP(launch_node_coords(prm->precision, G, prm->half_width, n0, n, nx, ny, nz, s),
                    "node coordinates");
        }
        if ((rc = run_sweep(&direct, true, nx, ny, nz, 0, n, Mn, nullptr, nullptr, nullptr, rho,
                            true, w, w.acc_a(), s)))
            return rc;
        Timed tm(SPK_KIND_OTHER, 0.0, s);
        SPK_HIP(launch_field_pack(prm->precision, w.acc_a(), w.L.ld, n0, n, field, s),
                "field pack");
    }
    return SPK_OK;
}

int sparkling_energy(const spk_params *prm, const void *kx, const void *ky, const void *kz,
                     const void *rho, double out[4], void *ws, size_t ws_bytes, void *stream)
{
    Range range("sparkling_energy");
    g_err.clear();
    int rc = check_params(prm, false);
    if (rc)
        return rc;
    const size_t al = elt_size(prm->precision);
    if ((rc = check_k(prm, kx, ky, kz)) || (rc = check_ptr(rho, "rho", al)))
        return rc;
    if (!out)
        return fail(SPK_EINVAL, "out is NULL");
    Ws w;
    if ((rc = bind_ws(prm, ws, ws_bytes, &w)))
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t p = prm->n_shots * prm->n_samples;
    if ((rc = run_gradient_sums(prm, kx, ky, kz, rho, 0, p, true, w, s)))
        return rc;
    if ((rc = reduce_energy(w, p, s)))
        return rc;
    const bool disc = prm->flags & SPK_FLAG_DISCREPANCY;
    double self_sum = 0.0;
    if (disc) {
        // E_rho = 1/2 sum_v rho_v sum_u rho_u H(x_v - x_u): cell sweeps whose
        // targets are the cell centres themselves, in passes of at most `cap`
        // cells; each pass's weighted sum lands in its own slot, and the
        // slots are added in pass order on the host.
        const int64_t G = prm->grid, M = G * G * G;
        const int64_t cap = std::min(M, kGridTargetChunk);
        const int64_t passes = (M + cap - 1) / cap;
        char *cells = static_cast<char *>(w.cells());
        void *cx = cells, *cy = cells + al * cap, *cz = cells + 2 * al * cap;
        spk_params direct = *prm;
        direct.attraction_field = nullptr;
        for (int64_t k = 0; k < passes; ++k) {
            const int64_t v0 = k * cap, n = std::min(cap, M - v0);
            {
                Timed tm(SPK_KIND_OTHER, 0.0, s);
                SPK_HIP(launch_cell_centres(prm->precision, G, prm->half_width, v0, n, cx, cy, cz,
                                            s),
                        "cell centres");
            }
            if ((rc = run_sweep(&direct, true, cx, cy, cz, 0, n, M, nullptr, nullptr, nullptr,
                                rho, true, w, w.acc_a(), s)))
                return rc;
            Timed tm(SPK_KIND_OTHER, 0.0, s);
            SPK_HIP(launch_wsum(static_cast<const char *>(rho) + al * v0, prm->precision,
                                w.acc_a() + 3 * w.L.ld, n, w.red(), w.chunk_sums() + k, s),
                    "self-energy reduction");
        }
        std::vector<double> part((size_t)passes);
        if ((rc = copy_to_host(part.data(), w.chunk_sums(), (size_t)passes, s)))
            return rc;
        for (double v : part)
            self_sum += v;
    }
    double sums[2];
    if ((rc = copy_to_host(sums, w.scal(), 2, s)))
        return rc;
    double e3[3];
    energies_from_sums(p, sums, e3);
    out[0] = e3[0];
    out[1] = e3[1];
    out[2] = e3[2];
    out[3] = disc ? e3[0] - 0.5 * self_sum : NAN;
    return SPK_OK;
}

int sparkling_constraint_check(const spk_params *prm, const void *kx, const void *ky,
                               const void *kz, double viol[4], void *ws, size_t ws_bytes,
                               void *stream)
{
    Range range("sparkling_constraint_check");
    g_err.clear();
    int rc = check_params(prm, true);
    if (rc)
        return rc;
    if ((rc = check_k(prm, kx, ky, kz)))
        return rc;
    if (!viol)
        return fail(SPK_EINVAL, "viol is NULL");
    Ws w;
    if ((rc = bind_ws(prm, ws, ws_bytes, &w)))
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = constraint_check_into(prm, kx, ky, kz, w, w.scal() + 8, s)))
        return rc;
    return copy_to_host(viol, w.scal() + 8, 4, s);
}

int sparkling_project(const spk_params *prm, void *kx, void *ky, void *kz, double *viol, void *ws,
                      size_t ws_bytes, void *stream)
{
    Range range("sparkling_project");
    g_err.clear();
    int rc = check_params(prm, true);
    if (rc)
        return rc;
    if ((rc = check_k(prm, kx, ky, kz)))
        return rc;
    Ws w;
    if ((rc = bind_ws(prm, ws, ws_bytes, &w)))
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = project_in_place(prm, kx, ky, kz, s)))
        return rc;
    if (!viol)
        return SPK_OK;
    if ((rc = constraint_check_into(prm, kx, ky, kz, w, w.scal() + 8, s)))
        return rc;
    return copy_to_host(viol, w.scal() + 8, 4, s);
}

int sparkling_step(const spk_params *prm, void *kx, void *ky, void *kz, const void *rho,
                   void *k_prev, void *g_prev, spk_step_info *info, void *ws, size_t ws_bytes,
                   void *stream)
{
    Range range("sparkling_step");
    g_err.clear();
    if (!info)
        return fail(SPK_EINVAL, "info is NULL");
    Ws w;
    int rc = check_step(prm, kx, ky, kz, rho, k_prev, g_prev, info->iter, info->eta_fixed, ws,
                        ws_bytes, &w);
    if (rc)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = enqueue_step_front(prm, kx, ky, kz, rho, k_prev, g_prev, info->iter,
                                 info->eta_fixed, w.info(), w, s)))
        return rc;
    double h[10];
    if ((rc = copy_to_host(h, w.info(), 4, s)))
        return rc;
    info->F = h[1];
    info->Fa = h[2];
    info->Fr = h[3];
    if (!std::isfinite(h[1])) {
        // nothing is updated: K and the caller's step state stay as they were
        info->eta = NAN;
        for (int c = 0; c < 4; ++c)
            info->viol[c] = NAN;
        info->bb_used = 0;
        info->bb_quotient = NAN;
        return fail(SPK_ENONFINITE, "energy is not finite (F = %g); K left unchanged", h[1]);
    }
    if ((rc = enqueue_step_back(prm, kx, ky, kz, k_prev, g_prev, w.info(), w, s)))
        return rc;
    if ((rc = copy_to_host(h, w.info(), 10, s)))
        return rc;
    info->eta = h[0];
    for (int c = 0; c < 4; ++c)
        info->viol[c] = h[4 + c];
    info->bb_used = h[8] != 0.0;
    info->bb_quotient = h[9];
    return SPK_OK;
}

int sparkling_step_async(const spk_params *prm, void *kx, void *ky, void *kz, const void *rho,
                         void *k_prev, void *g_prev, int64_t iter, double eta_fixed,
                         double *info_dev, void *ws, size_t ws_bytes, void *stream)
{
    Range range("sparkling_step_async");
    g_err.clear();
    Ws w;
    int rc = check_step(prm, kx, ky, kz, rho, k_prev, g_prev, iter, eta_fixed, ws, ws_bytes, &w);
    if (rc)
        return rc;
    if ((rc = check_ptr(info_dev, "info_dev", 8)))
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = enqueue_step_front(prm, kx, ky, kz, rho, k_prev, g_prev, iter, eta_fixed, info_dev,
                                 w, s)))
        return rc;
    return enqueue_step_back(prm, kx, ky, kz, k_prev, g_prev, info_dev, w, s);
}

}  // extern "C"

// ------------------------------------------------------------------------
// The allocation-free step: sparkling_step_async with its workspace in a
// static device array instead of a caller's buffer.
// ------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = SPK_SCRATCH_BYTES;
constexpr int kMaxScratchDevices = 64;

// One copy per device, held by the code object until the process ends.  In
// host code this name is a host-side stand-in, never a device address: host
// code uses the per-device address from hipGetSymbolAddress only.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int scratch_address(void **out)
{
    int dev = 0;
    SPK_HIP(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(SPK_EDEVICE, "device %d beyond the %d the static scratch tracks", dev,
                    kMaxScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *ptr = nullptr;
        SPK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "static scratch address");
        if (!ptr)
            return fail(SPK_EDEVICE, "static scratch address is NULL on device %d", dev);
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return SPK_OK;
}

struct Untimed {
    bool prev;
    Untimed() : prev(t_untimed) { t_untimed = true; }
    ~Untimed() { t_untimed = prev; }
};

}  // namespace

extern "C" {

size_t spk_noalloc_scratch_bytes(void) { return kScratchBytes; }

int sparkling_step_async_noalloc(const spk_params *prm, void *kx, void *ky, void *kz,
                                 const void *rho, void *k_prev, void *g_prev, int64_t iter,
                                 double eta_fixed, double *info_dev, void *stream)
{
    g_err.clear();
    int rc = check_params(prm, true);
    if (rc)
        return rc;
    // the arguments are checked before the scratch is looked up (no HIP call
    // for a rejected call), then again, identically, by the step itself
    const size_t al = elt_size(prm->precision);
    if ((rc = check_k(prm, kx, ky, kz)) || (rc = check_ptr(rho, "rho", al)) ||
        (rc = check_ptr(k_prev, "k_prev", al)) || (rc = check_ptr(g_prev, "g_prev", al)) ||
        (rc = check_ptr(info_dev, "info_dev", 8)))
        return rc;
    if (iter < 0 || !(eta_fixed > 0.0) || !std::isfinite(eta_fixed))
        return fail(SPK_EINVAL, "iter must be >= 0 and eta_fixed finite and > 0");
    if (prm->far_field_depth)
        return fail(SPK_EUNSUPPORTED, "the allocation-free step sums the repulsion exactly "
                                      "(far_field_depth must be 0)");
    const size_t need = make_layout(prm).total;
    if (need > kScratchBytes)
        return fail(SPK_EWORKSPACE, "the allocation-free step needs %zu bytes of scratch; its "
                                    "static scratch holds %zu",
                    need, kScratchBytes);
    void *ws = nullptr;
    if ((rc = scratch_address(&ws)))
        return rc;
    Untimed untimed;
    return sparkling_step_async(prm, kx, ky, kz, rho, k_prev, g_prev, iter, eta_fixed, info_dev,
                                ws, kScratchBytes, stream);
}

int sparkling_upsample(const spk_params *prm, const void *kx, const void *ky, const void *kz,
                       void *fx, void *fy, void *fz, void *stream)
{
    Range range("sparkling_upsample");
    g_err.clear();
    int rc = check_params(prm, false);
    if (rc)
        return rc;
    const int64_t p = prm->n_shots * prm->n_samples;
    if (2 * p > (int64_t(1) << 31) - 1)
        return fail(SPK_EINVAL, "the up-sampled trajectory must stay below 2^31 samples");
    const size_t al = elt_size(prm->precision);
    if ((rc = check_k(prm, kx, ky, kz)) || (rc = check_ptr(fx, "fx", al)) ||
        (rc = check_ptr(fy, "fy", al)) || (rc = check_ptr(fz, "fz", al)))
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Timed tm(SPK_KIND_OTHER, 0.0, s);
    SPK_HIP(launch_upsample(prm->precision, kx, ky, kz, fx, fy, fz, prm->n_shots, prm->n_samples, s),
            "up-sampling");
    return SPK_OK;
}

int spk_probe_pair_mix(int variant, int64_t blocks, int32_t iters, void *out,
                       size_t out_bytes, double *pairs, double *ms, void *stream)
{
    g_err.clear();
    if (variant < 0 || variant > 2)
        return fail(SPK_EINVAL, "probe variant must be 0, 1 or 2 (got %d)", variant);
    if (blocks < 1 || blocks > (int64_t(1) << 20) || iters < 1)
        return fail(SPK_EINVAL, "probe needs 1 <= blocks <= 2^20 and iters >= 1");
    if (!pairs || !ms)
        return fail(SPK_EINVAL, "pairs and ms must not be NULL");
    int rc;
    if ((rc = check_ptr(out, "out", 4)))
        return rc;
    const size_t need = sizeof(float) * (size_t)probe_out_elements(blocks);
    if (out_bytes < need)
        return fail(SPK_EWORKSPACE, "probe output needs %zu bytes (got %zu)", need,
                    out_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    struct Ev {
        hipEvent_t a = nullptr, b = nullptr;
        ~Ev()
        {
            if (a)
                (void)hipEventDestroy(a);
            if (b)
                (void)hipEventDestroy(b);
        }
    } ev;
    SPK_HIP(hipEventCreate(&ev.a), "probe event");
    SPK_HIP(hipEventCreate(&ev.b), "probe event");
    SPK_HIP(hipEventRecord(ev.a, s), "probe event record");
    SPK_HIP(launch_pair_mix_probe(variant, static_cast<float *>(out), blocks, iters, s),
            "probe launch");
    SPK_HIP(hipEventRecord(ev.b, s), "probe event record");
    SPK_HIP(hipEventSynchronize(ev.b), "probe synchronize");
    float t = 0.f;
    SPK_HIP(hipEventElapsedTime(&t, ev.a, ev.b), "probe elapsed time");
    *ms = t;
    *pairs = (double)probe_pairs(blocks, iters);
    return SPK_OK;
}

int spk_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    return SPK_OK;
}

int spk_timing_query(int kind, double *total_ms, int64_t *launches, double *pairs)
{
    if (kind < 0 || kind >= kKinds)
        return fail(SPK_EINVAL, "unknown timing kind %d", kind);
    std::lock_guard<std::mutex> lk(g_tmu);
    // Fold every pending launch into the totals; the events are released
    // whatever happens, so a failed query never counts a launch twice.
    bool ok = true;
    for (const TimedLaunch &t : g_pending) {
        float ms = 0.f;
        if (ok && (hipEventSynchronize(t.b) != hipSuccess ||
                   hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess))
            ok = false;
        if (ok) {
            g_ms[t.kind] += ms;
            g_launches[t.kind] += 1;
            g_pairs[t.kind] += t.pairs;
        }
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    g_pending.clear();
    if (!ok)
        return fail(SPK_EDEVICE, "timing event query failed; pending launches dropped");
    if (total_ms)
        *total_ms = g_ms[kind];
    if (launches)
        *launches = g_launches[kind];
    if (pairs)
        *pairs = g_pairs[kind];
    return SPK_OK;
}

int spk_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (const TimedLaunch &t : g_pending) {
        hipEventSynchronize(t.b);
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    g_pending.clear();
    for (int k = 0; k < kKinds; ++k) {
        g_ms[k] = 0;
        g_launches[k] = 0;
        g_pairs[k] = 0;
    }
    return SPK_OK;
}

}  // extern "C"
