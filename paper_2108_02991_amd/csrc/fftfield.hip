// Node field of the grid attraction by FFT convolution (Sec. "Evaluating F^a
// and its gradient": the convolution of the sampled kernel with the sampled
// density, computed with the FFT).
//
// Nodes X_k = -L + (k - 1/2) h (k = 0..G+1) and cell centres x_v = -L + (v +
// 1/2) h (v = 0..G-1), h = 2L/G, differ by (k - v - 1) h, so per component
//   U_c(k) = sum_v rho_v K_c[k - v - 1],  K_c[d] = (H, dH/dx, dH/dy, dH/dz)(d h),
// a linear convolution in which d stays in [-G, G] per axis.  A circular
// convolution of length M >= 2G + 1 per axis keeps every such d apart
// (d -> d mod M), so it equals the linear one on the nodes:
//   U_c(k) = IFFT(FFT(rho) . FFT(K_c))[(k - 1) mod M].
// Everything runs in FP64 on M^3 complex arrays (M a power of two, 8..1024);
// two real kernels share one complex transform (K_a + i K_b): since rho is
// real, the real and imaginary parts of the inverse are the two convolutions.
//
// The 3-D transform is three passes of 1-D transforms of length M, 8 lines
// per block in LDS (4 at M = 1024; bit-reversed load, in-place radix-2
// butterflies taken two stages at a time).  Along x the lines are contiguous; along y and z a block takes
// neighbouring lines in x, so each step along the line reads 8 (4) consecutive
// complex values.

#include <cmath>

#include "spk_internal.h"

namespace spk {
namespace {

constexpr int EW = 256;
constexpr int kFftThreads = 256;
constexpr int kMaxLog2 = 10;  // M <= 1024
// lines per block: 8 (LDS of 64 KB at M = 512), 4 at M = 1024
template <int LOG2M> constexpr int lines_of() { return LOG2M <= 9 ? 8 : 4; }

struct alignas(16) Cx {
    double re, im;
};

inline unsigned ew_blocks(int64_t n) { return (unsigned)((n + EW - 1) / EW); }

// tw[k] = exp(-2 pi i k / M), k < M/2.
__global__ __launch_bounds__(EW) void twiddle_kernel(int64_t M, Cx *tw)
{
    const int64_t k = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (k >= M / 2)
        return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)M, &s, &c);
    tw[k] = Cx{c, s};
}

// a[j] = rho_v (zero padded), j = vx + M (vy + M vz).
template <typename T>
__global__ __launch_bounds__(EW) void rho_fill_kernel(const T *rho, int64_t G, int64_t M, Cx *a)
{
    const int64_t j = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (j >= M * M * M)
        return;
    const int64_t x = j % M, y = (j / M) % M, z = j / (M * M);
    a[j] = (x < G && y < G && z < G) ? Cx{(double)rho[x + G * (y + G * z)], 0.0} : Cx{0.0, 0.0};
}

// Signed offset of circular index j, or a value outside [-G, G] when j is
// none of them.
__device__ inline int64_t offset_of(int64_t j, int64_t G, int64_t M)
{
    if (j <= G)
        return j;
    if (j >= M - G)
        return j - M;
    return G + 1;
}

// b[j] = K_ca[d] + i K_cb[d] for the offset d of j (0 where j is no offset);
// pair 0 holds (H, dH/dx), pair 1 (dH/dy, dH/dz).
__global__ __launch_bounds__(EW) void kernel_fill_kernel(int64_t G, int64_t M, double h, double eps,
                                                         int kern, int pair, Cx *b)
{
    const int64_t j = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (j >= M * M * M)
        return;
    const int64_t ox = offset_of(j % M, G, M), oy = offset_of((j / M) % M, G, M),
                  oz = offset_of(j / (M * M), G, M);
    if (ox > G || oy > G || oz > G) {
        b[j] = Cx{0.0, 0.0};
        return;
    }
    const double d[3] = {(double)ox * h, (double)oy * h, (double)oz * h};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps * eps;
    double v[4];
    if (kern == kKernelLog) {
        v[0] = 0.5 * log(r2);
        for (int a = 0; a < 3; ++a)
            v[1 + a] = d[a] / r2;
    } else {
        const double r = sqrt(r2);
        v[0] = r;
        for (int a = 0; a < 3; ++a)
            v[1 + a] = r > 0.0 ? d[a] / r : 0.0;
    }
    b[j] = Cx{v[2 * pair], v[2 * pair + 1]};
}

// One pass of 1-D transforms of length M = 2^LOG2M along `axis` (0 = x),
// kLines lines per block.  inverse: conjugate twiddles (no scaling).
template <int LOG2M>
__global__ __launch_bounds__(kFftThreads) void fft_kernel(Cx *a, int axis, const Cx *tw,
                                                          int inverse)
{
    constexpr int M = 1 << LOG2M, kLines = lines_of<LOG2M>();
    __shared__ Cx s[kLines][M];
    const int64_t b = blockIdx.x;
    const int64_t g = b % (M / kLines), o = b / (M / kLines);
    const int64_t MM = (int64_t)M * M;
    // line i of the block, position j along the axis
    auto at = [&](int i, int j) -> int64_t {
        const int64_t l = g * kLines + i;
        if (axis == 0)
            return j + M * l + MM * o;
        if (axis == 1)
            return l + (int64_t)M * j + MM * o;
        return l + (int64_t)M * o + MM * j;
    };
    const int t = threadIdx.x;
    for (int e = t; e < kLines * M; e += kFftThreads) {
        const int i = axis == 0 ? e / M : e % kLines, j = axis == 0 ? e % M : e / kLines;
        const int rj = (int)(__brev((unsigned)j) >> (32 - LOG2M));
        s[i][rj] = a[at(i, j)];
    }
    __syncthreads();
    // u +- w v for stage st's twiddle index k (conjugate when inverse)
    auto bfly = [&](Cx &u, Cx &v, int k) {
        const Cx w = tw[k];
        const double wi = inverse ? -w.im : w.im;
        const Cx vw = Cx{v.re * w.re - v.im * wi, v.re * wi + v.im * w.re};
        const Cx a = u;
        u = Cx{a.re + vw.re, a.im + vw.im};
        v = Cx{a.re - vw.re, a.im - vw.im};
    };
    // stages st and st + 1 together: each group of 4 elements (distance
    // half = 2^(st-1)) does stage st's two butterflies, then stage st+1's two,
    // in registers; one barrier per pair of stages
    int st = 1;
#pragma unroll 1
    for (; st + 1 <= LOG2M; st += 2) {
        const int half = 1 << (st - 1);
        for (int q = t; q < kLines * (M / 4); q += kFftThreads) {
            const int i = q / (M / 4), r = q % (M / 4);
            const int pos = r & (half - 1), lo = 4 * (r - pos) + pos;
            Cx a0 = s[i][lo], a1 = s[i][lo + half], a2 = s[i][lo + 2 * half],
               a3 = s[i][lo + 3 * half];
            bfly(a0, a1, pos << (LOG2M - st));
            bfly(a2, a3, pos << (LOG2M - st));
            bfly(a0, a2, pos << (LOG2M - st - 1));
            bfly(a1, a3, (pos + half) << (LOG2M - st - 1));
            s[i][lo] = a0;
            s[i][lo + half] = a1;
            s[i][lo + 2 * half] = a2;
            s[i][lo + 3 * half] = a3;
        }
        __syncthreads();
    }
    if (st == LOG2M) {   // odd number of stages: the last one alone
        const int half = 1 << (st - 1);
        for (int q = t; q < kLines * (M / 2); q += kFftThreads) {
            const int i = q / (M / 2), r = q % (M / 2);
            const int pos = r & (half - 1), lo = 2 * (r - pos) + pos;
            Cx u = s[i][lo], v = s[i][lo + half];
            bfly(u, v, pos << (LOG2M - st));
            s[i][lo] = u;
            s[i][lo + half] = v;
        }
        __syncthreads();
    }
    for (int e = t; e < kLines * M; e += kFftThreads) {
        const int i = axis == 0 ? e / M : e % kLines, j = axis == 0 ? e % M : e / kLines;
        a[at(i, j)] = s[i][j];
    }
}

// b[j] = b[j] * a[j] * scale.
__global__ __launch_bounds__(EW) void mul_kernel(const Cx *a, Cx *b, int64_t n, double scale)
{
    const int64_t j = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (j >= n)
        return;
    const Cx x = a[j], y = b[j];
    b[j] = Cx{(x.re * y.re - x.im * y.im) * scale, (x.re * y.im + x.im * y.re) * scale};
}

// field[n][2 pair], field[n][2 pair + 1] = re, im of b at ((k - 1) mod M).
template <typename T>
__global__ __launch_bounds__(EW) void extract_kernel(const Cx *b, int64_t G, int64_t M, int pair,
                                                     T *field)
{
    const int64_t Gn = G + 2, n = (int64_t)blockIdx.x * EW + threadIdx.x;
    if (n >= Gn * Gn * Gn)
        return;
    const int64_t kx = n % Gn, ky = (n / Gn) % Gn, kz = n / (Gn * Gn);
    const int64_t jx = (kx + M - 1) % M, jy = (ky + M - 1) % M, jz = (kz + M - 1) % M;
    const Cx v = b[jx + M * (jy + M * jz)];
    field[4 * n + 2 * pair] = (T)v.re;
    field[4 * n + 2 * pair + 1] = (T)v.im;
}

template <int LOG2M>
hipError_t fft3(Cx *a, const Cx *tw, int inverse, hipStream_t s)
{
    constexpr int64_t M = int64_t(1) << LOG2M;
    for (int axis = 0; axis < 3; ++axis)
        hipLaunchKernelGGL(fft_kernel<LOG2M>, dim3((unsigned)(M * M / lines_of<LOG2M>())),
                           dim3(kFftThreads), 0, s, a, axis, tw, inverse);
    return hipGetLastError();
}

hipError_t fft3_any(int log2m, Cx *a, const Cx *tw, int inverse, hipStream_t s)
{
    switch (log2m) {
    case 3: return fft3<3>(a, tw, inverse, s);
    case 4: return fft3<4>(a, tw, inverse, s);
    case 5: return fft3<5>(a, tw, inverse, s);
    case 6: return fft3<6>(a, tw, inverse, s);
    case 7: return fft3<7>(a, tw, inverse, s);
    case 8: return fft3<8>(a, tw, inverse, s);
    case 9: return fft3<9>(a, tw, inverse, s);
    case 10: return fft3<10>(a, tw, inverse, s);
    default: return hipErrorInvalidValue;
    }
}

int fft_log2(int64_t G)
{
    int l = 3;
    while ((int64_t(1) << l) < 2 * G + 1)
        ++l;
    return l;
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

}  // namespace

size_t field_fft_bytes(int64_t G)
{
    if (G < 1 || 2 * G + 1 > (int64_t(1) << kMaxLog2))
        return 0;
    const int64_t M = int64_t(1) << fft_log2(G);
    return 2 * align256(sizeof(Cx) * M * M * M) + align256(sizeof(Cx) * (M / 2)) + 256;
}

template <typename T>
static hipError_t field_fft_typed(int kern, int64_t G, double L, double eps, const T *rho, T *field,
                                  void *ws, hipStream_t s)
{
    const int lg = fft_log2(G);
    const int64_t M = int64_t(1) << lg, n = M * M * M;
    char *base = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(ws) + 255) / 256 * 256);
    Cx *A = reinterpret_cast<Cx *>(base);
    Cx *B = reinterpret_cast<Cx *>(base + align256(sizeof(Cx) * n));
    Cx *tw = reinterpret_cast<Cx *>(base + 2 * align256(sizeof(Cx) * n));
    const double h = 2.0 * L / (double)G;
    hipError_t e;
    hipLaunchKernelGGL(twiddle_kernel, dim3(ew_blocks(M / 2)), dim3(EW), 0, s, M, tw);
    hipLaunchKernelGGL(rho_fill_kernel<T>, dim3(ew_blocks(n)), dim3(EW), 0, s, rho, G, M, A);
    if ((e = fft3_any(lg, A, tw, 0, s)) != hipSuccess)
        return e;
    for (int pair = 0; pair < 2; ++pair) {
        hipLaunchKernelGGL(kernel_fill_kernel, dim3(ew_blocks(n)), dim3(EW), 0, s, G, M, h, eps,
                           kern, pair, B);
        if ((e = fft3_any(lg, B, tw, 0, s)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(mul_kernel, dim3(ew_blocks(n)), dim3(EW), 0, s, A, B, n,
                           1.0 / (double)n);
        if ((e = fft3_any(lg, B, tw, 1, s)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(extract_kernel<T>, dim3(ew_blocks((G + 2) * (G + 2) * (G + 2))),
                           dim3(EW), 0, s, B, G, M, pair, field);
    }
    return hipGetLastError();
}

hipError_t launch_field_fft(int precision, int kern, int64_t G, double L, double eps,
                            const void *rho, void *field, void *ws, hipStream_t s)
{
    if (field_fft_bytes(G) == 0)
        return hipErrorInvalidValue;
    if (precision == SPK_PLAIN_FP64)
        return field_fft_typed<double>(kern, G, L, eps, static_cast<const double *>(rho),
                                       static_cast<double *>(field), ws, s);
    return field_fft_typed<float>(kern, G, L, eps, static_cast<const float *>(rho),
                                  static_cast<float *>(field), ws, s);
}

}  // namespace spk
