// Per-shot projection onto the hardware constraint set and the constraint
// check (Sec. "3D K-space sampling"; supplement, "Multi-shot projection step").
//
// One workgroup per shot; shots are independent, as the paper notes.  Thread j
// owns NPT consecutive samples m = j*NPT .. j*NPT+NPT-1 and keeps the dual
// variables q (speed, one per forward difference) and r (slew, one per second
// difference) and their extrapolations in registers, all in double.  Its
// input samples k stay in registers too (widened to double once), except at
// NPT = 8, where registers are short and k is re-read from memory each time.
// Stencils reach at most two samples across a thread boundary, so each
// iteration exchanges two values per thread through LDS: the last two dual
// entries to the right neighbour before the primal update, the first two
// primal entries to the left neighbour before the dual update.  Each exchange
// array has one slot more than there are threads, holding zeros, which the
// first thread reads as its left neighbour's tails and the last thread as its
// right neighbour's heads; so every thread reads unconditionally.
//
// The iteration (accelerated proximal gradient on the dual of
// min_{s in Q} |s - k|^2 / 2, step tau = 1/20 since |D1|^2 + |D2|^2 <= 20):
//   s  = P0(k - D1^T qh - D2^T rh)       P0: clamp to [-L, L], then s[te] = 0
//   q+ = shrink(qh + tau D1 s, tau a),  r+ = shrink(rh + tau D2 s, tau b)
//   t+ = (1 + sqrt(1 + 4 t^2)) / 2,     qh = q+ + ((t - 1)/t+)(q+ - q), same for r
// and the output is P0(k - D1^T q - D2^T r) of the last dual iterate.  The
// duals start at 0 (cold start), or from a caller's dual state, which then
// receives the last dual iterate (warm start across successive projections:
// the solution is the same, only the starting point of the iteration moves).
// With
// (D1 s)[n] = s[n+1] - s[n], (D2 s)[n] = s[n+2] - 2 s[n+1] + s[n] and
// shrink(z, th) = z * max(0, 1 - th/|z|) per sample (group soft threshold of
// the 3-vector), or per coordinate for per-axis bounds, where the dual prox
// acts on each axis on its own.  Floating-point contraction is off and every
// expression keeps one fixed evaluation order.

#include "spk_internal.h"

namespace spk {
namespace {

__device__ inline double clamp_box(double z, double L)
{
    return z < -L ? -L : (z > L ? L : z);   // NaN stays NaN
}

// A bound on |z|^2 below which |z| <= thr is certain: thr^2 (1 - 2^-40) while
// thr^2 is a normal number (rounding moves it by far less than the margin,
// and the rounded sqrt of anything below it stays <= thr), else -1, which
// sends every z to the exact test.
__device__ inline double shrink_floor(double thr)
{
#pragma clang fp contract(off)
    return (thr >= 1e-150 && thr <= 1e150) ? (thr * thr) * (1.0 - 0x1p-40) : -1.0;
}

// max(0, 1 - thr/|z|) with |z| = sqrt(z.z); below the floor the factor is 0
// without the square root (a NaN z gives 0 either way).
__device__ inline double shrink_factor(double z0, double z1, double z2, double thr, double floor2)
{
#pragma clang fp contract(off)
    const double n2 = (z0 * z0 + z1 * z1) + z2 * z2;
    if (!(n2 > floor2))
        return 0.0;
    const double nrm = sqrt(n2);
    return (nrm > thr) ? (1.0 - thr / nrm) : 0.0;
}

__device__ inline double shrink_one(double z, double thr)
{
#pragma clang fp contract(off)
    const double m = fabs(z);
    return z * ((m > thr) ? (1.0 - thr / m) : 0.0);
}

// Two samples per thread fit in 128 registers: four waves per SIMD, so two
// shots share a compute unit and one's barriers overlap the other's work.
template <int NPT> constexpr int project_waves() { return NPT == 2 ? 4 : 1; }

template <typename T, int NPT, bool PER_AXIS>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(project_waves<NPT>())))
void project_kernel(T *kx, T *ky, T *kz, int64_t Ns, double L, double a, double b, int64_t te,
                    int n_pit, const double *gate, double *duals)
{
#pragma clang fp contract(off)
    static_assert(NPT >= 2, "two-sample halo needs NPT >= 2");
    // a NaN gate (a step that was not taken) leaves every shot as it is; the
    // whole block leaves before its first barrier
    if (gate && !(*gate == *gate))
        return;
    extern __shared__ double xch[];
    const int nth = blockDim.x;
    const int j = threadIdx.x;
    const int ld = nth + 1;               // one zero slot per row
    // tails of thread j at slot j + 1 (slot 0: zeros); heads at slot j (slot nth: zeros)
    double *q_tail = xch;                 // [3][ld]  q[last]
    double *r_tail0 = q_tail + 3 * ld;    // [3][ld]  r[last-1]
    double *r_tail1 = r_tail0 + 3 * ld;   // [3][ld]  r[last]
    double *s_head0 = r_tail1 + 3 * ld;   // [3][ld]  s[first]
    double *s_head1 = s_head0 + 3 * ld;   // [3][ld]  s[first+1]
    if (j == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            q_tail[c * ld] = r_tail0[c * ld] = r_tail1[c * ld] = 0.0;
            s_head0[c * ld + nth] = s_head1[c * ld + nth] = 0.0;
        }
    }

    const int64_t m0 = (int64_t)j * NPT;
    // Samples of this wave (uniform across it): only the wave holding te
    // applies s[te] = 0, and only waves reaching past sample Ns-3 clear the
    // dual entries beyond their ranges; both overwrite values computed as
    // for any other sample, so the other waves skip them.
    const int64_t wm0 = (int64_t)(__builtin_amdgcn_readfirstlane(j) & ~63) * NPT;
    const int64_t wm1 = wm0 + 64 * NPT - 1;
    const bool wave_te = te >= wm0 && te <= wm1;
    const bool wave_tail = wm1 > Ns - 3;
    T *K[3] = {kx + (int64_t)blockIdx.x * Ns, ky + (int64_t)blockIdx.x * Ns,
               kz + (int64_t)blockIdx.x * Ns};

    // k widened to double (exact, the same value at every use)
    constexpr bool k_regs = NPT <= 4;
    double kr[3][k_regs ? NPT : 1];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < (k_regs ? NPT : 1); ++i)
            kr[c][i] = (k_regs && m0 + i < Ns) ? (double)K[c][m0 + i] : 0.0;
    // duals of this shot: q (speed, n < Ns-1) then r (slew, n < Ns-2), [c * Ns + n]
    double *D = duals ? duals + (int64_t)blockIdx.x * 6 * Ns : nullptr;
    double q[3][NPT], qh[3][NPT], r[3][NPT], rh[3][NPT];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int64_t m = m0 + i;
            const double q0 = (D && m <= Ns - 2) ? D[c * Ns + m] : 0.0;
            const double r0 = (D && m <= Ns - 3) ? D[(3 + c) * Ns + m] : 0.0;
            q[c][i] = qh[c][i] = q0;
            r[c][i] = rh[c][i] = r0;
        }
    auto kval = [&](int c, int i) -> double {
        if constexpr (k_regs)
            return kr[c][i];
        const int64_t m = m0 + i;
        return m < Ns ? (double)K[c][m] : 0.0;
    };

    // s[m] for the thread's samples from duals (dq, dr), halo values from the left.
    // The stencil needs no bounds tests: every dual entry outside its range
    // (q[n] for n > Ns-2, r[n] for n > Ns-3, and the padding threads') holds +0,
    // which the dual update below keeps, and the zero slots stand for q[-1],
    // r[-2] and r[-1]; so D1^T q and D2^T r read +0 exactly where the
    // definitions have no term.
    auto primal = [&](double (&s)[3][NPT + 2], const double (&dq)[3][NPT],
                      const double (&dr)[3][NPT]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double q_left = q_tail[c * ld + j];     // q[m0-1] (0 for j = 0)
            const double r_left0 = r_tail0[c * ld + j];   // r[m0-2]
            const double r_left1 = r_tail1[c * ld + j];   // r[m0-1]
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                const double qa = i >= 1 ? dq[c][i - 1] : q_left;                         // q[m-1]
                const double ra = i >= 2 ? dr[c][i - 2] : (i == 1 ? r_left1 : r_left0);  // r[m-2]
                const double rb = i >= 1 ? dr[c][i - 1] : r_left1;                        // r[m-1]
                const double d1t = qa - dq[c][i];
                const double d2t = (ra - 2.0 * rb) + dr[c][i];
                s[c][i] = clamp_box((kval(c, i) - d1t) - d2t, L);
            }
        }
        if (wave_te) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int i = 0; i < NPT; ++i)
                    s[c][i] = (m0 + i == te) ? 0.0 : s[c][i];
        }
    };
    auto publish_tails = [&](const double (&dq)[3][NPT], const double (&dr)[3][NPT]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            q_tail[c * ld + j + 1] = dq[c][NPT - 1];
            r_tail0[c * ld + j + 1] = dr[c][NPT - 2];
            r_tail1[c * ld + j + 1] = dr[c][NPT - 1];
        }
    };

    publish_tails(qh, rh);
    __syncthreads();

    const double tau = 1.0 / 20.0;
    const double thr_a = tau * a, thr_b = tau * b;
    const double floor_a = shrink_floor(thr_a), floor_b = shrink_floor(thr_b);
    // one dual step at every sample of the thread, given s and the momentum
    auto dual_update = [&](const double (&s)[3][NPT + 2], double mom) {
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            double zq[3], zr[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                zq[c] = qh[c][i] + tau * (s[c][i + 1] - s[c][i]);
                zr[c] = rh[c][i] + tau * ((s[c][i + 2] - 2.0 * s[c][i + 1]) + s[c][i]);
            }
            if constexpr (PER_AXIS) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    zq[c] = shrink_one(zq[c], thr_a);
                    zr[c] = shrink_one(zr[c], thr_b);
                }
            } else {
                const double fq = shrink_factor(zq[0], zq[1], zq[2], thr_a, floor_a);
                const double fr = shrink_factor(zr[0], zr[1], zr[2], thr_b, floor_b);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    zq[c] = zq[c] * fq;
                    zr[c] = zr[c] * fr;
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double qn = zq[c], rn = zr[c];
                qh[c][i] = qn + mom * (qn - q[c][i]);
                q[c][i] = qn;
                rh[c][i] = rn + mom * (rn - r[c][i]);
                r[c][i] = rn;
            }
        }
        // entries past the ranges back to +0 (their previous value was +0, so
        // this equals taking qn = rn = 0 there)
        if (wave_tail) {
#pragma unroll
            for (int i = 0; i < NPT; ++i) {
                const int64_t n = m0 + i;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    q[c][i] = (n <= Ns - 2) ? q[c][i] : 0.0;
                    qh[c][i] = (n <= Ns - 2) ? qh[c][i] : 0.0;
                    r[c][i] = (n <= Ns - 3) ? r[c][i] : 0.0;
                    rh[c][i] = (n <= Ns - 3) ? rh[c][i] : 0.0;
                }
            }
        }
    };
    double t = 1.0;
    for (int it = 0; it < n_pit; ++it) {
        double s[3][NPT + 2];
        primal(s, qh, rh);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s_head0[c * ld + j] = s[c][0];
            s_head1[c * ld + j] = s[c][1];
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s[c][NPT] = s_head0[c * ld + j + 1];       // 0 for the last thread
            s[c][NPT + 1] = s_head1[c * ld + j + 1];
        }
        const double tn = (1.0 + sqrt(1.0 + 4.0 * t * t)) / 2.0;
        const double mom = (t - 1.0) / tn;
        dual_update(s, mom);
        t = tn;
        publish_tails(qh, rh);
        __syncthreads();
    }

    publish_tails(q, r);
    __syncthreads();
    double s[3][NPT + 2];
    primal(s, q, r);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int64_t m = m0 + i;
            if (m < Ns) {
                K[c][m] = (T)s[c][i];
                if (D) {
                    D[c * Ns + m] = m <= Ns - 2 ? q[c][i] : 0.0;
                    D[(3 + c) * Ns + m] = m <= Ns - 3 ? r[c][i] : 0.0;
                }
            }
        }
}

// NaN-propagating maximum (order-independent: NaN is sticky, otherwise exact max).
__device__ inline double vmax(double m, double x)
{
    if (m != m)
        return m;
    return (x != x || x > m) ? x : m;
}

constexpr int CB = 256;

__device__ inline double norm3(double dx, double dy, double dz, int per_axis)
{
#pragma clang fp contract(off)
    if (per_axis)
        return vmax(vmax(fabs(dx), fabs(dy)), fabs(dz));
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

template <typename T>
__global__ __launch_bounds__(CB) void check_kernel(const T *kx, const T *ky, const T *kz,
                                                   int64_t Ns, double L, double a, double b,
                                                   int64_t te, int per_axis, double *per_shot)
{
#pragma clang fp contract(off)
    __shared__ double red[4][CB];
    const int64_t off = (int64_t)blockIdx.x * Ns;
    const T *x = kx + off, *y = ky + off, *z = kz + off;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t n = threadIdx.x; n < Ns; n += CB) {
        const double x0 = x[n], y0 = y[n], z0 = z[n];
        if (n + 1 < Ns) {
            const double dx = (double)x[n + 1] - x0, dy = (double)y[n + 1] - y0,
                         dz = (double)z[n + 1] - z0;
            m[0] = vmax(m[0], norm3(dx, dy, dz, per_axis) / a);
        }
        if (n + 2 < Ns) {
            const double dx = ((double)x[n + 2] - 2.0 * (double)x[n + 1]) + x0;
            const double dy = ((double)y[n + 2] - 2.0 * (double)y[n + 1]) + y0;
            const double dz = ((double)z[n + 2] - 2.0 * (double)z[n + 1]) + z0;
            m[1] = vmax(m[1], norm3(dx, dy, dz, per_axis) / b);
        }
        m[2] = vmax(m[2], fabs(x0) / L);
        m[2] = vmax(m[2], fabs(y0) / L);
        m[2] = vmax(m[2], fabs(z0) / L);
        if (n == te)
            m[3] = vmax(m[3], sqrt((x0 * x0 + y0 * y0) + z0 * z0));
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        red[c][threadIdx.x] = m[c];
    __syncthreads();
    for (int w = CB / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                red[c][threadIdx.x] = vmax(red[c][threadIdx.x], red[c][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 4)
        per_shot[(int64_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(CB) void check_final_kernel(const double *per_shot, int64_t n_shots,
                                                         double *out)
{
    __shared__ double red[4][CB];
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t s = threadIdx.x; s < n_shots; s += CB)
#pragma unroll
        for (int c = 0; c < 4; ++c)
            m[c] = vmax(m[c], per_shot[s * 4 + c]);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        red[c][threadIdx.x] = m[c];
    __syncthreads();
    for (int w = CB / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                red[c][threadIdx.x] = vmax(red[c][threadIdx.x], red[c][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 4)
        out[threadIdx.x] = red[threadIdx.x][0];
}

template <typename T, int NPT>
hipError_t launch_project_npt(T *kx, T *ky, T *kz, int64_t n_shots, int64_t Ns, double L,
                              double a, double b, int64_t te, int n_pit, int per_axis,
                              const double *gate, double *duals, hipStream_t s)
{
    int64_t nth = (Ns + NPT - 1) / NPT;
    nth = (nth + 63) / 64 * 64;
    const size_t lds = sizeof(double) * 15 * (size_t)(nth + 1);
    if (per_axis)
        hipLaunchKernelGGL((project_kernel<T, NPT, true>), dim3((unsigned)n_shots),
                           dim3((unsigned)nth), lds, s, kx, ky, kz, Ns, L, a, b, te, n_pit, gate,
                           duals);
    else
        hipLaunchKernelGGL((project_kernel<T, NPT, false>), dim3((unsigned)n_shots),
                           dim3((unsigned)nth), lds, s, kx, ky, kz, Ns, L, a, b, te, n_pit, gate,
                           duals);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_project_t(T *kx, T *ky, T *kz, int64_t n_shots, int64_t Ns, double L, double a,
                            double b, int64_t te, int n_pit, int per_axis, const double *gate,
                            double *duals, hipStream_t s)
{
    // at most 512 threads per shot: the halo buffers (15 doubles per thread
    // and 15 zero slots) stay under 64 KB of LDS
    if (Ns <= 2 * 512)
        return launch_project_npt<T, 2>(kx, ky, kz, n_shots, Ns, L, a, b, te, n_pit,
                                            per_axis, gate, duals, s);
    if (Ns <= 4 * 512)
        return launch_project_npt<T, 4>(kx, ky, kz, n_shots, Ns, L, a, b, te, n_pit,
                                            per_axis, gate, duals, s);
    return launch_project_npt<T, 8>(kx, ky, kz, n_shots, Ns, L, a, b, te, n_pit,
                                            per_axis, gate, duals, s);
}

}  // namespace

hipError_t launch_project(int precision, void *kx, void *ky, void *kz, int64_t n_shots,
                          int64_t n_samples, double L, double a, double b, int64_t te, int n_pit,
                          bool per_axis, const double *gate, double *duals, hipStream_t s)
{
    if (n_samples > kMaxProjectSamples)
        return hipErrorInvalidValue;
    if (precision == SPK_PLAIN_FP64)
        return launch_project_t((double *)kx, (double *)ky, (double *)kz, n_shots, n_samples, L,
                                a, b, te, n_pit, per_axis ? 1 : 0, gate, duals, s);
    return launch_project_t((float *)kx, (float *)ky, (float *)kz, n_shots, n_samples, L, a, b,
                            te, n_pit, per_axis ? 1 : 0, gate, duals, s);
}

hipError_t launch_constraint_check(int precision, const void *kx, const void *ky, const void *kz,
                                   int64_t n_shots, int64_t n_samples, double L, double a,
                                   double b, int64_t te, bool per_axis, double *per_shot,
                                   double *out, hipStream_t s)
{
    const int pa = per_axis ? 1 : 0;
    if (precision == SPK_PLAIN_FP64)
        hipLaunchKernelGGL(check_kernel<double>, dim3((unsigned)n_shots), dim3(CB), 0, s,
                           (const double *)kx, (const double *)ky, (const double *)kz, n_samples,
                           L, a, b, te, pa, per_shot);
    else
        hipLaunchKernelGGL(check_kernel<float>, dim3((unsigned)n_shots), dim3(CB), 0, s,
                           (const float *)kx, (const float *)ky, (const float *)kz, n_samples, L,
                           a, b, te, pa, per_shot);
    hipLaunchKernelGGL(check_final_kernel, dim3(1), dim3(CB), 0, s, per_shot, n_shots, out);
    return hipGetLastError();
}

}  // namespace spk
