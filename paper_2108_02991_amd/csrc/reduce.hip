// Combines, finalisation, deterministic reductions and the step's vector
// updates.  All HBM-bound; every sum runs in a fixed order that depends only
// on the element count, so results are bit-reproducible.

#include "spk_internal.h"

namespace spk {
namespace {

constexpr int RB = 256;        // threads per reduction block
constexpr int PER = 16;        // elements per thread per reduction block
constexpr int EW = 256;        // threads per elementwise block

inline unsigned ew_blocks(int64_t n) { return (unsigned)((n + EW - 1) / EW); }

__global__ __launch_bounds__(EW) void combine_kernel(double *acc, int64_t ld, const double *part,
                                                     int64_t part_ld, int nslabs, int64_t nt,
                                                     int init)
{
    const int64_t e = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (e >= 4 * nt)
        return;
    const int64_t c = e / nt, t = e - c * nt;
    const int64_t o = c * ld + t;
    double v = init ? 0.0 : acc[o];
    for (int y = 0; y < nslabs; ++y)
        v += part[((int64_t)y * 4 + c) * part_ld + t];
    acc[o] = v;
}

template <typename T>
__global__ __launch_bounds__(EW) void finalize_kernel(const double *acc_a, const double *acc_r,
                                                      int64_t ld, int64_t nt, double inv_p,
                                                      double inv_p2, T *gx, T *gy, T *gz,
                                                      double *pot_a, double *pot_r)
{
    const int64_t t = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (t >= nt)
        return;
    T *g[3] = {gx, gy, gz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double fa = acc_a[c * ld + t] * inv_p;
        const double fr = acc_r[c * ld + t] * inv_p2;
        g[c][t] = (T)(fa - fr);
    }
    if (pot_a)
        pot_a[t] = acc_a[3 * ld + t];
    if (pot_r)
        pot_r[t] = acc_r[3 * ld + t];
}

// Sum over the 64 lanes of a wave; every lane ends with the same value.
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Block sum in a fixed tree; the result is valid in thread 0.
__device__ inline double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        lds[w] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < RB / 64; ++k)
            tot += lds[k];
    __syncthreads();
    return tot;
}

// Stage 1 of a two-series sum: partial b covers elements [b*RB*PER, (b+1)*RB*PER).
// Series values come from a functor f(e, &v0, &v1).
template <class F>
__global__ __launch_bounds__(RB) void sum_stage1(F f, int64_t n, double *partials)
{
    __shared__ double lds[RB / 64];
    const int64_t base = (int64_t)blockIdx.x * RB * PER + threadIdx.x;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t e = base + (int64_t)k * RB;
        if (e < n) {
            double v0, v1;
            f(e, v0, v1);
            a0 += v0;
            a1 += v1;
        }
    }
    a0 = block_sum(a0, lds);
    a1 = block_sum(a1, lds);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = a0;
        partials[2 * blockIdx.x + 1] = a1;
    }
}

__global__ __launch_bounds__(RB) void sum_stage2(const double *partials, int64_t nb, double *out)
{
    __shared__ double lds[RB / 64];
    double a0 = 0.0, a1 = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += RB) {
        a0 += partials[2 * b];
        a1 += partials[2 * b + 1];
    }
    a0 = block_sum(a0, lds);
    a1 = block_sum(a1, lds);
    if (threadIdx.x == 0) {
        out[0] = a0;
        out[1] = a1;
    }
}

struct Pair2 {
    const double *x0, *x1;
    __device__ void operator()(int64_t e, double &v0, double &v1) const
    {
        v0 = x0[e];
        v1 = x1 ? x1[e] : 0.0;
    }
};

template <typename T> struct WeightedF {
    const T *w;
    const double *x;
    __device__ void operator()(int64_t e, double &v0, double &v1) const
    {
        v0 = (double)w[e] * x[e];
        v1 = 0.0;
    }
};

template <typename T> struct DotsF {
    const T *kx, *ky, *kz, *kp, *g, *gp;
    int64_t p;
    __device__ void operator()(int64_t e, double &ss, double &sy) const
    {
        const int64_t c = e / p, i = e - c * p;
        const T *k = c == 0 ? kx : (c == 1 ? ky : kz);
        const double s = (double)k[i] - (double)kp[e];
        const double y = (double)g[e] - (double)gp[e];
        ss = s * s;
        sy = s * y;
    }
};

template <class F>
hipError_t run_sum(F f, int64_t n, double *partials, double *out, hipStream_t s)
{
    const int64_t nb = n > 0 ? (n + RB * PER - 1) / (RB * PER) : 1;
    if (n > 0)
        hipLaunchKernelGGL(sum_stage1<F>, dim3((unsigned)nb), dim3(RB), 0, s, f, n, partials);
    else
        hipLaunchKernelGGL(sum_stage1<F>, dim3(1), dim3(RB), 0, s, f, (int64_t)0, partials);
    hipLaunchKernelGGL(sum_stage2, dim3(1), dim3(RB), 0, s, partials, nb, out);
    return hipGetLastError();
}

__device__ inline double cell_centre(int64_t i, int64_t G, double L)
{
#pragma clang fp contract(off)
    return -L + ((double)i + 0.5) * (2.0 * L / (double)G);
}

template <typename T>
__global__ __launch_bounds__(EW) void cell_centres_kernel(int64_t G, double L, int64_t v0,
                                                          int64_t cnt, T *cx, T *cy, T *cz)
{
    const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (i >= cnt)
        return;
    const int64_t v = v0 + i;
    cx[i] = (T)cell_centre(v % G, G, L);
    cy[i] = (T)cell_centre((v / G) % G, G, L);
    cz[i] = (T)cell_centre(v / (G * G), G, L);
}

template <typename T>
__global__ __launch_bounds__(EW) void axpy_save_kernel(T *kx, T *ky, T *kz, T *kp, const T *g,
                                                       T *gp, int64_t p, double eta,
                                                       const double *eta_dev)
{
    const int64_t e = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (e >= 3 * p)
        return;
    // a step size chosen on the device; NaN there means "no update"
    const double h = eta_dev ? *eta_dev : eta;
    if (!(h == h))
        return;
    const int64_t c = e / p, i = e - c * p;
    T *k = c == 0 ? kx : (c == 1 ? ky : kz);
    const T kv = k[i], gv = g[e];
    kp[e] = kv;
    gp[e] = gv;
    k[i] = (T)((double)kv - h * (double)gv);
}

// The step-size rule on the device, from the energy sums scal[0..1] and, in
// the Barzilai-Borwein phase, the dots scal[2] = s.s and scal[3] = s.y; the
// same operations, in the same order, as the host-side rule.  info[9] keeps
// the quotient s.s/s.y before the clamp (NaN in the fixed-step phase).
__global__ void step_policy_kernel(const double *scal, int64_t p, double eta_fixed, int bb,
                                   double *info)
{
#pragma clang fp contract(off)
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const double fa = scal[0] / (double)p;
    const double fr = scal[1] / (2.0 * (double)p * (double)p);
    const double F = fa - fr;
    double eta = eta_fixed;
    double used = 0.0;
    double quotient = __builtin_nan("");
    if (bb) {
        const double ss = scal[2], sy = scal[3];
        const double q = ss / sy;
        quotient = q;
        if (sy > 0.0 && q - q == 0.0) {
            eta = q;
            eta = fmin(fmax(eta, 0.1 * eta_fixed), 10.0 * eta_fixed);
            used = 1.0;
        }
    }
    if (!(F - F == 0.0)) {
        eta = __builtin_nan("");
        used = 0.0;
    }
    info[0] = eta;
    info[1] = F;
    info[2] = fa;
    info[3] = fr;
    info[8] = used;
    info[9] = quotient;
}

// Dyadic linear up-sampling of shots (fine sample m at coarse position m/2;
// the last one continues the last coarse step), in double, contraction off.
template <typename T>
__global__ __launch_bounds__(EW) void upsample_kernel(const T *kx, const T *ky, const T *kz, T *fx,
                                                      T *fy, T *fz, int64_t Nc, int64_t N)
{
#pragma clang fp contract(off)
    const int64_t pf = 2 * Nc * N;
    const int64_t e = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (e >= 3 * pf)
        return;
    const int64_t c = e / pf, i = e - c * pf;
    const int64_t shot = i / (2 * N), m = i - shot * (2 * N), n = m / 2;
    const T *k = (c == 0 ? kx : (c == 1 ? ky : kz)) + shot * N;
    T *f = (c == 0 ? fx : (c == 1 ? fy : fz)) + shot * 2 * N;
    double v;
    if (m % 2 == 0)
        v = (double)k[n];
    else if (n + 1 < N)
        v = ((double)k[n] + (double)k[n + 1]) * 0.5;
    else
        v = N > 1 ? 1.5 * (double)k[n] - 0.5 * (double)k[n - 1] : (double)k[n];
    f[m] = (T)v;
}

}  // namespace

hipError_t launch_upsample(int precision, const void *kx, const void *ky, const void *kz, void *fx,
                           void *fy, void *fz, int64_t Nc, int64_t N, hipStream_t s)
{
    const int64_t n = 3 * 2 * Nc * N;
    if (precision == SPK_PLAIN_FP64) {
        using T = double;
        hipLaunchKernelGGL(upsample_kernel<T>, dim3(ew_blocks(n)), dim3(EW), 0, s, (const T *)kx,
                           (const T *)ky, (const T *)kz, (T *)fx, (T *)fy, (T *)fz, Nc, N);
    } else {
        using T = float;
        hipLaunchKernelGGL(upsample_kernel<T>, dim3(ew_blocks(n)), dim3(EW), 0, s, (const T *)kx,
                           (const T *)ky, (const T *)kz, (T *)fx, (T *)fy, (T *)fz, Nc, N);
    }
    return hipGetLastError();
}

hipError_t launch_combine(double *acc, int64_t ld, const double *part, int64_t part_ld,
                          int nslabs, int64_t nt, bool init, hipStream_t s)
{
    if (nt <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(combine_kernel, dim3(ew_blocks(4 * nt)), dim3(EW), 0, s, acc, ld, part,
                       part_ld, nslabs, nt, init ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_finalize_grad(int precision, const double *acc_a, const double *acc_r,
                                int64_t ld, int64_t nt, double inv_p, double inv_p2, void *gx,
                                void *gy, void *gz, double *pot_a, double *pot_r, hipStream_t s)
{
    if (nt <= 0)
        return hipSuccess;
    if (precision == SPK_PLAIN_FP64)
        hipLaunchKernelGGL(finalize_kernel<double>, dim3(ew_blocks(nt)), dim3(EW), 0, s, acc_a,
                           acc_r, ld, nt, inv_p, inv_p2, (double *)gx, (double *)gy, (double *)gz,
                           pot_a, pot_r);
    else
        hipLaunchKernelGGL(finalize_kernel<float>, dim3(ew_blocks(nt)), dim3(EW), 0, s, acc_a,
                           acc_r, ld, nt, inv_p, inv_p2, (float *)gx, (float *)gy, (float *)gz,
                           pot_a, pot_r);
    return hipGetLastError();
}

int64_t reduce_partials_size(int64_t n)
{
    const int64_t nb = n > 0 ? (n + RB * PER - 1) / (RB * PER) : 1;
    return 2 * nb;
}

hipError_t launch_sum2(const double *x0, const double *x1, int64_t n, double *partials,
                       double *out, hipStream_t s)
{
    return run_sum(Pair2{x0, x1}, n, partials, out, s);
}

hipError_t launch_wsum(const void *w, int precision, const double *x, int64_t n,
                       double *partials, double *out, hipStream_t s)
{
    if (precision == SPK_PLAIN_FP64)
        return run_sum(WeightedF<double>{(const double *)w, x}, n, partials, out, s);
    return run_sum(WeightedF<float>{(const float *)w, x}, n, partials, out, s);
}

hipError_t launch_cell_centres(int precision, int64_t G, double L, int64_t v0, int64_t n,
                               void *cx, void *cy, void *cz, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    if (precision == SPK_PLAIN_FP64)
        hipLaunchKernelGGL(cell_centres_kernel<double>, dim3(ew_blocks(n)), dim3(EW), 0, s, G, L,
                           v0, n, (double *)cx, (double *)cy, (double *)cz);
    else
        hipLaunchKernelGGL(cell_centres_kernel<float>, dim3(ew_blocks(n)), dim3(EW), 0, s, G, L,
                           v0, n, (float *)cx, (float *)cy, (float *)cz);
    return hipGetLastError();
}

hipError_t launch_bb_dots(int precision, const void *kx, const void *ky, const void *kz,
                          const void *k_prev, const void *g, const void *g_prev, int64_t p,
                          double *partials, double *out, hipStream_t s)
{
    if (precision == SPK_PLAIN_FP64) {
        using T = double;
        return run_sum(DotsF<T>{(const T *)kx, (const T *)ky, (const T *)kz, (const T *)k_prev,
                                (const T *)g, (const T *)g_prev, p},
                       3 * p, partials, out, s);
    }
    using T = float;
    return run_sum(DotsF<T>{(const T *)kx, (const T *)ky, (const T *)kz, (const T *)k_prev,
                            (const T *)g, (const T *)g_prev, p},
                   3 * p, partials, out, s);
}

hipError_t launch_axpy_save(int precision, void *kx, void *ky, void *kz, void *k_prev,
                            const void *g, void *g_prev, int64_t p, double eta,
                            const double *eta_dev, hipStream_t s)
{
    if (precision == SPK_PLAIN_FP64) {
        using T = double;
        hipLaunchKernelGGL(axpy_save_kernel<T>, dim3(ew_blocks(3 * p)), dim3(EW), 0, s, (T *)kx,
                           (T *)ky, (T *)kz, (T *)k_prev, (const T *)g, (T *)g_prev, p, eta,
                           eta_dev);
    } else {
        using T = float;
        hipLaunchKernelGGL(axpy_save_kernel<T>, dim3(ew_blocks(3 * p)), dim3(EW), 0, s, (T *)kx,
                           (T *)ky, (T *)kz, (T *)k_prev, (const T *)g, (T *)g_prev, p, eta,
                           eta_dev);
    }
    return hipGetLastError();
}

hipError_t launch_step_policy(const double *scal, int64_t p, double eta_fixed, bool bb,
                              double *info, hipStream_t s)
{
    hipLaunchKernelGGL(step_policy_kernel, dim3(1), dim3(64), 0, s, scal, p, eta_fixed,
                       bb ? 1 : 0, info);
    return hipGetLastError();
}

namespace {
// 2 K[t] . G[t] per target, in double with contraction off (one fixed order).
template <typename T>
__global__ __launch_bounds__(EW) void force_potential_kernel(const T *kx, const T *ky,
                                                             const T *kz, int64_t t0, int64_t nt,
                                                             double *acc, int64_t ld)
{
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (t >= nt)
        return;
    const double x = (double)kx[t0 + t], y = (double)ky[t0 + t], z = (double)kz[t0 + t];
    acc[3 * ld + t] = 2.0 * ((x * acc[t] + y * acc[ld + t]) + z * acc[2 * ld + t]);
}
}  // namespace

hipError_t launch_force_potential(int precision, const void *kx, const void *ky, const void *kz,
                                  int64_t t0, int64_t nt, double *acc, int64_t ld, hipStream_t s)
{
    if (nt <= 0)
        return hipSuccess;
    if (precision == SPK_PLAIN_FP64)
        hipLaunchKernelGGL(force_potential_kernel<double>, dim3(ew_blocks(nt)), dim3(EW), 0, s,
                           (const double *)kx, (const double *)ky, (const double *)kz, t0, nt,
                           acc, ld);
    else
        hipLaunchKernelGGL(force_potential_kernel<float>, dim3(ew_blocks(nt)), dim3(EW), 0, s,
                           (const float *)kx, (const float *)ky, (const float *)kz, t0, nt,
                           acc, ld);
    return hipGetLastError();
}

}  // namespace spk
