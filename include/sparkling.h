/*
 * sparkling.h -- C ABI of libsparkling.so, the MI355X (gfx950) hot path of
 * full-3D SPARKLING trajectory optimisation (arXiv 2108.02991).
 *
 * The library evaluates the objective of the paper's "3D SPARKLING
 * formulation" section,
 *
 *     F(K) = F^a(K) - F^r(K),
 *     F^a  = (1/p)     sum_i sum_v rho_v H(K[i] - x_v)     (attraction),
 *     F^r  = 1/(2p^2)  sum_i sum_j H(K[i] - K[j])          (repulsion),
 *
 * with H(d) = |d|_2 (or the regularised sqrt(|d|^2 + eps^2) of Sec. "Choice
 * of step size"), its gradient (Secs. "Evaluating F^a and its gradient" and
 * "Evaluating F^r and its gradient"),
 *
 *     dF/dK[i] = (1/p) sum_v rho_v grad H(K[i] - x_v) - (1/p^2) sum_j grad H(K[i] - K[j]),
 *
 * the per-shot projection onto the hardware constraint set Q of Sec. "3D
 * K-space sampling" (supplement, "Multi-shot projection step"), and one
 * projected gradient step of the projected-gradient-descent equation with the
 * step-size policy of Sec. "Choice of step size".
 *
 * Conventions shared by every entry point
 *  - p = n_shots * n_samples samples in shot-lexicographic order: sample n of
 *    shot c is index i = c * n_samples + n.
 *  - K is passed as three device arrays kx, ky, kz of p elements each
 *    (structure of arrays).  Element type: double for SPK_PLAIN_FP64, float
 *    for every other precision.  rho and gradients use the same type.
 *  - rho holds G^3 weights of a cell-centred grid over [-L, L]^3, x fastest:
 *    weight v = ix + G*(iy + G*iz) sits at x_v = -L + (i + 1/2) * 2L/G per
 *    axis.  The library uses the weights as given (callers normalise them to
 *    sum 1, as the paper's density does).
 *  - grad H(0) = 0: coincident samples (every shot passes the k-space centre
 *    at the echo time) exert no force on each other.
 *  - All device pointers must be on the current HIP device, 4-byte aligned
 *    (8 for double), and must not alias each other except where an argument
 *    is documented as in/out.  The caller owns every buffer, including the
 *    workspace sized by spk_workspace_size(); the library allocates no device
 *    memory at run time and creates no stream (the static scratch of
 *    sparkling_step_async_noalloc is part of its code object).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *    their kernels on it and return without waiting, except that any call
 *    writing a host output (a double* documented as "host") synchronises the
 *    stream before returning.
 *  - Arguments are validated before anything is enqueued: SPK_EINVAL and
 *    SPK_EWORKSPACE mean nothing was launched and no output was written.
 *    SPK_EDEVICE means a HIP call failed; outputs are then undefined.
 *    spk_last_error() returns a text describing the last failure on the
 *    calling thread.
 *  - Results are deterministic: the same inputs give bit-identical outputs
 *    on every run, for every target chunking of sparkling_grad.
 */
#ifndef SPARKLING_H
#define SPARKLING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden visibility; these declarations are its
 * exported interface. */
#pragma GCC visibility push(default)

typedef enum {
    SPK_OK = 0,
    SPK_EINVAL = -1,        /* bad argument; nothing launched                     */
    SPK_EWORKSPACE = -2,    /* workspace NULL or smaller than spk_workspace_size  */
    SPK_EDEVICE = -3,       /* a HIP runtime call or launch failed                */
    SPK_EUNSUPPORTED = -4,  /* valid but outside what the library implements      */
    SPK_ENONFINITE = -5     /* the energy of a step was NaN or infinite           */
} spk_status;

typedef enum {
    SPK_PLAIN_FP64 = 0,     /* double coordinates, pair math and accumulation           */
    SPK_FP32_COMP = 1,      /* float pair math, per-tile float sums folded by two-sum   */
    SPK_FP32_NAIVE = 2,     /* float pair math and one float running sum (diagnostic)   */
    SPK_FP32_ACC64 = 3      /* float pair math, double accumulation per pair (diagn.)   */
} spk_precision;

enum {
    SPK_FLAG_DISCREPANCY = 1,        /* sparkling_energy also returns D = F - E_rho    */
    SPK_FLAG_ROTATION_VARIANT = 2,   /* constraint norms |.| are per-axis maxima (the
                                        l_inf bounds of Sec. "3D K-space sampling")
                                        instead of Euclidean norms                     */
    SPK_FLAG_LOG_KERNEL = 4,         /* H(d) = log(|d|^2 + eps^2) / 2, the logarithmic
                                        kernel the "3D SPARKLING formulation" names as
                                        an alternative, regularised; needs eps > 0
                                        with eps^2 a normal number of the form's type,
                                        and the plain_fp64 or fp32_comp form
                                        (SPK_EUNSUPPORTED otherwise)                   */
    SPK_FLAG_FIELD_DIRECT = 8,       /* sparkling_field sums the node field directly
                                        over the cells in the precision form instead
                                        of by FP64 FFT convolution                      */
    SPK_FLAG_ENERGY_FROM_FORCE = 16  /* F^r from the repulsion forces: with H = |d|,
                                        F^r is homogeneous of degree 1 in K (every
                                        distance scales with K), so by Euler's theorem
                                        F^r = sum_i K[i] . dF^r/dK[i]; the repulsion
                                        sweep then skips its per-pair distance term.
                                        Distance kernel with eps = 0 and the exact
                                        repulsion only (SPK_EINVAL with eps > 0, the log
                                        kernel or far_field_depth > 0); per-target
                                        repulsion potentials are then not available
                                        (sparkling_grad with pot_r: SPK_EINVAL)        */
};

typedef struct {
    int64_t n_shots;      /* N_c >= 1                                                   */
    int64_t n_samples;    /* N_s >= 1 (>= 2 for projection and step)                    */
    int64_t grid;         /* G in [1, 1024]: rho is G^3 cells                           */
    int32_t precision;    /* spk_precision                                              */
    int32_t te_index;     /* sample pinned to the origin in every shot; -1 = none       */
    double  half_width;   /* L > 0: sampling box [-L, L]^3 (the paper uses L = 1)       */
    double  eps;          /* >= 0: H(d) = sqrt(|d|^2 + eps^2); 0 gives H = |d|
                             (log kernel: H(d) = log(|d|^2 + eps^2) / 2, eps > 0)      */
    double  a_max;        /* per-raster-step speed bound (spk_alpha_beta), > 0          */
    double  b_max;        /* per-raster-step slew bound (spk_alpha_beta), > 0           */
    int32_t n_pit;        /* projection iterations, >= 0                                */
    int32_t flags;        /* SPK_FLAG_*                                                 */
    const void *attraction_field; /* NULL: attraction summed directly over the G^3
                                     cells; else the node field of sparkling_field(),
                                     evaluated by trilinear interpolation            */
    int32_t far_field_depth;  /* 0: repulsion summed over all p^2 pairs.  2..7: the
                                 samples' far field by a Chebyshev fast multipole
                                 method on a uniform octree of 8^depth leaves over
                                 the samples' bounding cube, the 27 leaves around
                                 each target summed exactly (plain_fp64 and
                                 fp32_comp forms; SPK_EUNSUPPORTED otherwise)    */
    int32_t far_field_order;  /* Chebyshev nodes per axis, 3..6, when depth > 0     */
    int32_t far_field_adaptive; /* refinement levels R, 0..2: 0 is the uniform
                                   octree.  Leaves whose near field is dense
                                   enough are refined one level, and (R = 2)
                                   their children again by the same rule; a
                                   target then sums exactly over the 27 cells
                                   around it at its deepest level only
                                   (depth + R <= 7)                               */
    void   *far_field_stream; /* hipStream_t, when depth > 0.  NULL: the far
                                 field's exact near-field sums run on the call's
                                 stream, after its translations.  Else a second
                                 stream of the caller's (same device, default
                                 priority, not the call's stream): the near-field
                                 sums run there beside the translations, forked
                                 from and joined back to the call's stream by
                                 events, so the call stays ordered on its
                                 stream.  The library creates no stream.      */
    void   *proj_duals;   /* NULL: every projection (sparkling_project, the
                             steps) starts its dual variables at 0, the cold
                             start.  Else device doubles [n_shots][6][n_samples],
                             caller-owned, in/out: per coordinate c, the speed
                             duals q at [c][n] (n < N_s-1) then the slew duals r
                             at [3+c][n] (n < N_s-2), other entries 0.  The
                             projection starts from them and leaves its last
                             dual iterate there (warm start across the steps;
                             the converged projection is the same).  Zero it
                             before the first call.  8-byte aligned; must not
                             alias any other argument.                      */
} spk_params;

/* Text of a status code (static storage). */
const char *spk_status_string(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *spk_last_error(void);

/*
 * Normalised speed and slew bounds (Sec. "3D K-space sampling"):
 *   alpha = min(gamma_bar * gmax, 1 / (fov * dwell_dt)) / kmax,
 *   beta  = gamma_bar * smax / kmax,
 * scaled to one raster step of a trajectory in [-L, L]^3:
 *   *a_max = alpha * raster_dt * L,  *b_max = beta * raster_dt^2 * L.
 * gamma_bar is the gyromagnetic ratio over 2 pi (42.576e6 Hz/T for 1H);
 * gmax in T/m, smax in T/m/s, times in s, fov in m, kmax in 1/m.
 * Host only.  SPK_EINVAL if any input is not strictly positive.
 */
int spk_alpha_beta(double gmax, double smax, double raster_dt, double dwell_dt, double fov,
                   double kmax, double gamma_bar, double half_width,
                   double *a_max, double *b_max);

/*
 * Bytes of device workspace that every entry point below needs for these
 * parameters (one size serves all of them).  Host only.
 */
int spk_workspace_size(const spk_params *prm, size_t *bytes);

/*
 * Energies of the objective ("3D SPARKLING formulation"): writes the host
 * array out[4] = {F, F^a, F^r, D}, where D = F - E_rho and
 * E_rho = 1/2 sum_{u,v} rho_u rho_v H(x_u - x_v) is the density's
 * self-energy (D >= 0).  D costs a G^6 pair sweep and is NaN unless
 * prm->flags has SPK_FLAG_DISCREPANCY.  Synchronises `stream`.
 */
int sparkling_energy(const spk_params *prm, const void *kx, const void *ky, const void *kz,
                     const void *rho, double out[4], void *ws, size_t ws_bytes, void *stream);

/*
 * Bound on the Lipschitz constant of grad F for the regularised kernels (Sec.
 * "Choice of step size": a fixed step inversely proportional to it gives the
 * convergence guarantee).  With p samples, regulariser eps > 0 and total
 * density mass rho_mass = sum_v rho_v (rho_v >= 0; 1 for a normalised
 * density), every eigenvalue of the Hessian of F lies in
 *   distance kernel: [-1, rho_mass] / (p eps),
 *   log kernel     : [-(1 + rho_mass/8), rho_mass + 1/8] / (p eps^2),
 * since the kernel's Hessian is bounded by [0, 1/eps] (distance) or
 * [-1/(8 eps^2), 1/eps^2] (log) and the repulsion's quadratic form sums
 * |v_i - v_j|^2 <= 2p |v|^2 over pairs.  *lipschitz receives the largest
 * magnitude; the step 1/(*lipschitz) then decreases F by at least
 * (*lipschitz/2) |K+ - K|^2 per step when the projection is exact (for
 * instance n_pit = 0 with unbounded speed and slew: box and echo time).
 * flags: only SPK_FLAG_LOG_KERNEL matters.  Host only.  SPK_EINVAL if p < 1,
 * eps <= 0, or rho_mass < 0 or not finite.
 */
int spk_lipschitz_bound(int64_t p, double eps, double rho_mass, int32_t flags,
                        double *lipschitz);

/*
 * Workspace bytes of sparkling_field for prm: the FFT buffers (two M^3
 * complex doubles, M the power of two >= 2G + 1, at least 8; 4.3 GB at
 * G = 192) when the field is taken by FFT, else spk_workspace_size(prm).
 * Host only.
 */
int spk_field_workspace_size(const spk_params *prm, size_t *bytes);

/*
 * Node field of the grid attraction (Sec. "Evaluating F^a and its gradient":
 * the discrete convolution of the sampled kernel with the sampled density,
 * computed once per density and evaluated off the grid by the trilinear
 * interpolant).  Nodes sit at X_k = -L + (k - 1/2) * 2L/G, k = 0..G+1, per
 * axis (the cell centres plus one node beyond each face), node
 * n = kx + (G+2)*(ky + (G+2)*kz).  field (device, K's type, 16-byte aligned
 * for float, 32 for double) receives 4*(G+2)^3 values laid out
 * [n][U, dU/dx, dU/dy, dU/dz] with U(x) = sum_v rho_v H(x - x_v) for the
 * kernel of prm (a field is valid only with the kernel and eps it was built
 * with).  When 2G + 1 <= 1024 the convolution runs as FP64 FFTs of size M^3
 * (exact up to FP64 rounding) and ws must hold spk_field_workspace_size(prm)
 * bytes; with SPK_FLAG_FIELD_DIRECT, or for larger grids, it is summed
 * directly over the cells in the precision form with the workspace of
 * spk_workspace_size(prm).  Setting
 * prm->attraction_field to this buffer makes energy, gradient and step use
 * the interpolant for the attraction (valid for samples inside
 * [-L - h/2, L + h/2]^3; outside, the nearest node layer is extrapolated
 * linearly).  prm->attraction_field is ignored by this call.
 */
int sparkling_field(const spk_params *prm, const void *rho, void *field, void *ws,
                    size_t ws_bytes, void *stream);

/*
 * Gradient of F (Secs. "Evaluating F^a and its gradient", "Evaluating F^r
 * and its gradient") for the targets i in [tgt_begin, tgt_end), 0 <= tgt_begin
 * <= tgt_end <= p, against all p samples and all G^3 cells.
 *   gx, gy, gz : device, element t - tgt_begin receives dF/dK[t] (K's type).
 *   pot_a, pot_r : device doubles or NULL; element t - tgt_begin receives
 *                  sum_v rho_v H(K[t] - x_v) and sum_j H(K[t] - K[j]).
 *   energy : host double[3] or NULL; receives {F, F^a, F^r} and requires the
 *            full range [0, p).  Synchronises `stream` when non-NULL.
 * An empty range is valid, launches nothing and accepts NULL outputs.  Every
 * chunking of [0, p) gives bit-identical rows.
 */
int sparkling_grad(const spk_params *prm, const void *kx, const void *ky, const void *kz,
                   const void *rho, void *gx, void *gy, void *gz,
                   int64_t tgt_begin, int64_t tgt_end, double *pot_a, double *pot_r,
                   double *energy, void *ws, size_t ws_bytes, void *stream);

/*
 * Per-shot projection onto Q (supplement, "Multi-shot projection step"), in
 * place on kx, ky, kz: each shot s becomes an approximation of
 * argmin_{s in Q} |s - k|^2 / 2 with Q = {|s|_inf <= L, s[te] = 0,
 * |s[n+1] - s[n]| <= a_max, |s[n+2] - 2 s[n+1] + s[n]| <= b_max}, computed
 * by prm->n_pit iterations of accelerated proximal gradient on the dual
 * (step 1/20, cold start), all in double precision.  |.| is the Euclidean
 * norm of a sample's 3 coordinates, or their largest magnitude when
 * prm->flags has SPK_FLAG_ROTATION_VARIANT (per-axis hardware bounds).  The box and the
 * echo-time point hold exactly; a shot already strictly inside Q is
 * returned unchanged.  viol: host double[4] or NULL, receives the
 * constraint check of the result (see sparkling_constraint_check) and then
 * synchronises `stream`.  n_samples must be in [2, 4096].
 */
int sparkling_project(const spk_params *prm, void *kx, void *ky, void *kz, double *viol,
                      void *ws, size_t ws_bytes, void *stream);

/*
 * Normalised constraint violations of K (Sec. "3D K-space sampling"),
 * host double[4]: {max |s[n+1]-s[n]| / a_max, max |s[n+2]-2s[n+1]+s[n]| / b_max,
 * max |s|_inf / L, max_shots |s[te]|_2}; values <= 1 (resp. 0) are feasible.
 * The first two use the norm that sparkling_project uses (per-axis maximum
 * with SPK_FLAG_ROTATION_VARIANT, else Euclidean).
 * Computed in double from the stored values; NaN propagates.  Synchronises.
 */
int sparkling_constraint_check(const spk_params *prm, const void *kx, const void *ky,
                               const void *kz, double viol[4], void *ws, size_t ws_bytes,
                               void *stream);

/*
 * Warm restart of the multi-resolution strategy (Sec. "Multi-resolution
 * strategy for faster convergence", Algorithm 1): every shot of the coarse
 * trajectory (prm->n_shots shots of prm->n_samples samples on a raster twice
 * as long) is up-sampled by linear interpolation to 2*n_samples samples.
 * Fine sample m sits at coarse position m/2: even m copy coarse sample m/2,
 * odd m average its two neighbours, and the last fine sample continues the
 * last coarse step (1.5 k[N-1] - 0.5 k[N-2]; a one-sample shot is repeated).
 * 2p must stay below 2^31.  kx, ky, kz: device, coarse,
 * p elements each; fx, fy, fz: device, 2p elements each, K's type, no
 * aliasing.  Asynchronous.
 */
int sparkling_upsample(const spk_params *prm, const void *kx, const void *ky, const void *kz,
                       void *fx, void *fy, void *fz, void *stream);

typedef struct {
    int64_t iter;         /* in: iteration index t (0-based)                              */
    double  eta_fixed;    /* in: fixed step size, used while t < 20 and as BB fallback    */
    double  eta;          /* out: step size used                                          */
    double  F, Fa, Fr;    /* out: energies at the input K                                 */
    double  viol[4];      /* out: constraint check of the new K                           */
    int32_t bb_used;      /* out: 1 if the Barzilai-Borwein step was taken                */
    int32_t reserved;
    double  bb_quotient;  /* out: s.s/s.y before the clamp (t >= 20; NaN for t < 20)       */
} spk_step_info;

/*
 * One projected gradient step (projected-gradient-descent equation,
 * step-size policy of Sec. "Choice of step size"):
 *   g = dF/dK at K;  eta = eta_fixed if iter < 20, else
 *   eta = (s.s)/(s.y), s = K - k_prev, y = g - g_prev (all 3p coordinates,
 *   double sums), clamped to [0.1, 10] * eta_fixed, or eta_fixed if s.y <= 0;
 *   k_prev = K; g_prev = g; K = Pi_Q(K - eta g).
 * kx, ky, kz: in/out.  k_prev, g_prev: device, 3p elements of K's type laid
 * out [3][p], caller-owned state carried between calls (contents ignored
 * while iter < 20).  info: host, in/out.  Synchronises `stream`.
 * Returns SPK_ENONFINITE if F at the input K is not finite; K, k_prev and
 * g_prev are then left unchanged and info holds F, F^a, F^r (eta and viol NaN).
 */
int sparkling_step(const spk_params *prm, void *kx, void *ky, void *kz, const void *rho,
                   void *k_prev, void *g_prev, spk_step_info *info,
                   void *ws, size_t ws_bytes, void *stream);

/*
 * The step of sparkling_step with no host synchronisation, for loops that run
 * many steps per host round trip or replay a captured HIP graph.  The same
 * kernels run in the same order; the step size is chosen on the device by the
 * same rule, so K, k_prev and g_prev evolve bit for bit as with
 * sparkling_step.  info_dev: device, 10 doubles, receives {eta, F, F^a, F^r,
 * viol[4], bb_used, bb_quotient}.  If F is not finite, eta is NaN and K, k_prev and
 * g_prev are left unchanged (the constraint check still reports on K).  The
 * launch sequence depends on iter only through iter >= 20, so one captured
 * graph serves every iteration of a phase.  Enqueues kernels only: no host
 * copy, no synchronisation, no allocation, no memset.
 */
int sparkling_step_async(const spk_params *prm, void *kx, void *ky, void *kz, const void *rho,
                         void *k_prev, void *g_prev, int64_t iter, double eta_fixed,
                         double *info_dev, void *ws, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the step of
 * sparkling_step_async, same kernels, same bits, with no workspace argument.
 * Its workspace is a static device array of SPK_SCRATCH_BYTES held by the
 * library on every device it runs on until the process ends; the call makes
 * no allocation of any kind (no hipMalloc, no event, no stream) and its
 * launches are not timed.  Every call on one device shares that device's
 * array: calls that overlap on one device (several streams or threads) race
 * and must be serialised by the caller.  No byte of the array needs to start
 * at any value: every call writes what it reads.  The first call on a device
 * looks up the array's device address (hipGetSymbolAddress, which may load
 * the code object): make it outside graph capture; later calls only enqueue
 * kernels and may be captured.
 * Errors: SPK_EWORKSPACE if spk_workspace_size(prm) exceeds SPK_SCRATCH_BYTES
 * (on a 32^3 density: p up to about 300,000 samples), SPK_EUNSUPPORTED for
 * far_field_depth > 0, otherwise as sparkling_step_async.
 */
#define SPK_SCRATCH_BYTES ((size_t)64 << 20)
int sparkling_step_async_noalloc(const spk_params *prm, void *kx, void *ky, void *kz,
                                 const void *rho, void *k_prev, void *g_prev, int64_t iter,
                                 double eta_fixed, double *info_dev, void *stream);
/* SPK_SCRATCH_BYTES, as built into the library. */
size_t spk_noalloc_scratch_bytes(void);

/*
 * Calibration, not an operation of the paper: issue rates of the repulsion
 * pair's instruction mix on the current device.  One launch of `blocks`
 * blocks of 256 threads runs, per thread and iteration, 4 sources against 2
 * targets with the sweep's per-pair instructions (variant 0: 3 subtractions,
 * 3 FMAs for |d|^2, v_rsq_f32, 4 FMAs, in one fixed order), the same without
 * the reciprocal square root (1), or the reciprocal square roots with one FMA
 * each (2), in registers only.  pairs (out) = blocks * 256 * iters * 8;
 * ms (out) = the launch's duration by HIP events.  out: device,
 * >= blocks * 256 * 4 bytes (one result per thread, so nothing is removed).
 * Synchronises `stream`.  SPK_EINVAL for a bad variant, blocks outside
 * [1, 2^20] or iters < 1; SPK_EWORKSPACE for a short output buffer.
 */
int spk_probe_pair_mix(int variant, int64_t blocks, int32_t iters, void *out,
                       size_t out_bytes, double *pairs, double *ms, void *stream);

/*
 * Kernel timing.  While enabled, every kernel launch of the kinds below is
 * bracketed by HIP events on the stream it runs on; spk_timing_query()
 * waits for those events and returns, for one kind, the summed duration in
 * ms, the launch count and the pair interactions processed.  Timing state is
 * process-global and guarded by a mutex.  Launches on a stream that is being
 * captured into a graph are not timed.
 */
enum {
    SPK_KIND_REPULSION = 0,   /* all-pairs sample sweep                   */
    SPK_KIND_ATTRACTION = 1,  /* sample x density-cell sweep              */
    SPK_KIND_PROJECTION = 2,  /* per-shot projection                      */
    SPK_KIND_OTHER = 3,       /* reductions, combine, step, check         */
    SPK_KIND_INTERPOLATION = 4 /* grid-attraction interpolant              */
};
int spk_timing_enable(int on);
int spk_timing_query(int kind, double *total_ms, int64_t *launches, double *pairs);
int spk_timing_reset(void);

#pragma GCC visibility pop

#ifdef __cplusplus
}
#endif

#endif /* SPARKLING_H */
