// Grid attraction (Sec. "Evaluating F^a and its gradient"): node coordinates
// for the field precompute, packing of the node sums into the field layout,
// and the trilinear interpolant of the field at the samples.
//
// The field is an array of structures, one (U, dU/dx, dU/dy, dU/dz) quadruple
// per node, so each of the 8 corner reads of the interpolant is one 16-byte
// (float) or 32-byte (double) load.  The interpolant is a gather bound by
// HBM/L2 traffic: 8 corners x 16 B per sample in FP32, against 12 B of
// coordinates read and 32 B of FP64 sums written.

#include "spk_internal.h"

namespace spk {
namespace {

constexpr int EW = 256;

template <typename T> struct alignas(4 * sizeof(T)) Q4 { T u, x, y, z; };

// Node coordinate -L + (k - 1/2) * (2L/G), in this exact order.
__device__ inline double node_coord(int64_t k, int64_t G, double L)
{
#pragma clang fp contract(off)
    return -L + ((double)k - 0.5) * (2.0 * L / (double)G);
}

template <typename T>
__global__ __launch_bounds__(EW) void node_coords_kernel(int64_t G, double L, int64_t n0,
                                                         int64_t cnt, T *nx, T *ny, T *nz)
{
    const int64_t Gn = G + 2;
    const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (i >= cnt)
        return;
    const int64_t n = n0 + i;
    nx[i] = (T)node_coord(n % Gn, G, L);
    ny[i] = (T)node_coord((n / Gn) % Gn, G, L);
    nz[i] = (T)node_coord(n / (Gn * Gn), G, L);
}

template <typename T>
__global__ __launch_bounds__(EW) void field_pack_kernel(const double *acc, int64_t ld,
                                                        int64_t cnt, Q4<T> *field)
{
    const int64_t i = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (i >= cnt)
        return;
    field[i] = Q4<T>{(T)acc[3 * ld + i], (T)acc[i], (T)acc[ld + i], (T)acc[2 * ld + i]};
}

// Lower node and upper weight along one axis: t = (x - X_0)/h, k0 = floor(t)
// clamped to [0, G], f = t - k0 (all in double, contraction off).
__device__ inline void axis_weight(double x, int64_t G, double L, int64_t &k0, double &f)
{
#pragma clang fp contract(off)
    const double h = 2.0 * L / (double)G;
    const double t = (x - node_coord(0, G, L)) / h;
    double k = floor(t);
    // NaN and -inf go to node 0 (the weight then carries the NaN/inf), +inf to G
    k = !(k >= 0.0) ? 0.0 : (k > (double)G ? (double)G : k);
    k0 = (int64_t)k;
    f = t - k;
}

template <typename T>
__global__ __launch_bounds__(EW) void interp_kernel(const T *kx, const T *ky, const T *kz,
                                                    int64_t t0, int64_t nt, int64_t G, double L,
                                                    const Q4<T> *field, double *acc, int64_t ld)
{
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (t >= nt)
        return;
    const int64_t i = t0 + t;
    const int64_t Gn = G + 2;
    int64_t k[3];
    double f[3];
    axis_weight((double)kx[i], G, L, k[0], f[0]);
    axis_weight((double)ky[i], G, L, k[1], f[1]);
    axis_weight((double)kz[i], G, L, k[2], f[2]);
    double out[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                                 (dz ? f[2] : 1.0 - f[2]);
                const Q4<T> v = field[(k[0] + dx) + Gn * ((k[1] + dy) + Gn * (k[2] + dz))];
                out[0] += w * (double)v.u;
                out[1] += w * (double)v.x;
                out[2] += w * (double)v.y;
                out[3] += w * (double)v.z;
            }
    acc[t] = out[1];
    acc[ld + t] = out[2];
    acc[2 * ld + t] = out[3];
    acc[3 * ld + t] = out[0];
}

inline unsigned ew_blocks(int64_t n) { return (unsigned)((n + EW - 1) / EW); }

}  // namespace

hipError_t launch_node_coords(int precision, int64_t G, double L, int64_t n0, int64_t n, void *nx,
                              void *ny, void *nz, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    if (precision == SPK_PLAIN_FP64)
        hipLaunchKernelGGL(node_coords_kernel<double>, dim3(ew_blocks(n)), dim3(EW), 0, s, G, L,
                           n0, n, (double *)nx, (double *)ny, (double *)nz);
    else
        hipLaunchKernelGGL(node_coords_kernel<float>, dim3(ew_blocks(n)), dim3(EW), 0, s, G, L,
                           n0, n, (float *)nx, (float *)ny, (float *)nz);
    return hipGetLastError();
}

hipError_t launch_field_pack(int precision, const double *acc, int64_t ld, int64_t n0, int64_t n,
                             void *field, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    if (precision == SPK_PLAIN_FP64)
        hipLaunchKernelGGL(field_pack_kernel<double>, dim3(ew_blocks(n)), dim3(EW), 0, s, acc, ld,
                           n, (Q4<double> *)field + n0);
    else
        hipLaunchKernelGGL(field_pack_kernel<float>, dim3(ew_blocks(n)), dim3(EW), 0, s, acc, ld,
                           n, (Q4<float> *)field + n0);
    return hipGetLastError();
}

hipError_t launch_interpolate(int precision, const void *kx, const void *ky, const void *kz,
                              int64_t t0, int64_t nt, int64_t G, double L, const void *field,
                              double *acc, int64_t ld, hipStream_t s)
{
    if (nt <= 0)
        return hipSuccess;
    if (precision == SPK_PLAIN_FP64)
        hipLaunchKernelGGL(interp_kernel<double>, dim3(ew_blocks(nt)), dim3(EW), 0, s,
                           (const double *)kx, (const double *)ky, (const double *)kz, t0, nt, G,
                           L, (const Q4<double> *)field, acc, ld);
    else
        hipLaunchKernelGGL(interp_kernel<float>, dim3(ew_blocks(nt)), dim3(EW), 0, s,
                           (const float *)kx, (const float *)ky, (const float *)kz, t0, nt, G, L,
                           (const Q4<float> *)field, acc, ld);
    return hipGetLastError();
}

}  // namespace spk
