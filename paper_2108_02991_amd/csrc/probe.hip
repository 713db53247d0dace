// Issue-rate probes of the repulsion pair's instruction mix (gfx950).
//
// The repulsion sweep's inner loop issues, per pair, 3 subtractions, 3 FMAs
// for |d|^2 (the guard folded into the first), one v_rsq_f32 and 4 FMAs for
// the three force components and the energy: 10 FP32 instructions with all
// operands in VGPRs plus one quarter-rate transcendental.  These kernels issue
// parts of that mix from registers only (no memory traffic, no address
// arithmetic), 8 pairs (4 sources against 2 targets) per loop iteration, in
// volatile asm so that nothing is hoisted or removed; the accumulators carry
// a dependence from one iteration to the next as in the sweep.  Variants:
//   0  the whole mix in one fixed order (all subtractions, the |d|^2 FMAs,
//      the reciprocal square roots, the accumulations);
//   1  the same without the reciprocal square root (w = |d|^2): the rate of
//      the pair's 10 FP32 instructions as a stream;
//   2  the 8 reciprocal square roots with one FMA each: their cost.
// Variants 1 and 2 give the component rates from which the sweep's issue
// bound is estimated; variant 0 shows what one fixed order achieves (the
// compiled sweep, whose scheduler spreads the reciprocal square roots, runs
// faster than it).

#include <hip/hip_runtime.h>

#include <cstdint>

#include "spk_internal.h"

namespace spk {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeSources = 4;      // sources per iteration, against 2 targets

template <int VARIANT>
__global__ __launch_bounds__(kProbeThreads) void pair_mix_probe(float *out, int iters)
{
    const float base = 1e-3f * (float)(threadIdx.x + 1) + 1e-6f * (float)blockIdx.x;
    const float xi0 = base, yi0 = 0.5f * base, zi0 = -base;
    const float xi1 = -0.25f * base, yi1 = base, zi1 = 0.75f * base;
    float sx[kProbeSources], sy[kProbeSources], sz[kProbeSources];
#pragma unroll
    for (int u = 0; u < kProbeSources; ++u) {
        sx[u] = 0.1f * (float)(u + 1);
        sy[u] = 0.05f * (float)(u + 2);
        sz[u] = 0.02f * (float)(u + 3);
    }
    const float guard = 1.17549435e-38f;
    float gx0 = 0.f, gy0 = 0.f, gz0 = 0.f, e0 = 0.f, gx1 = 0.f, gy1 = 0.f, gz1 = 0.f, e1 = 0.f;
    float dx[kProbeSources][2], dy[kProbeSources][2], dz[kProbeSources][2];
    float r[kProbeSources][2], w[kProbeSources][2];
    for (int it = 0; it < iters; ++it) {
        if constexpr (VARIANT == 0) {
            asm volatile(
                "v_sub_f32 %[dx00], %[xi0], %[sx0]\n\t"
                "v_sub_f32 %[dx01], %[xi1], %[sx0]\n\t"
                "v_sub_f32 %[dx10], %[xi0], %[sx1]\n\t"
                "v_sub_f32 %[dx11], %[xi1], %[sx1]\n\t"
                "v_sub_f32 %[dx20], %[xi0], %[sx2]\n\t"
                "v_sub_f32 %[dx21], %[xi1], %[sx2]\n\t"
                "v_sub_f32 %[dx30], %[xi0], %[sx3]\n\t"
                "v_sub_f32 %[dx31], %[xi1], %[sx3]\n\t"
                "v_sub_f32 %[dy00], %[yi0], %[sy0]\n\t"
                "v_sub_f32 %[dy01], %[yi1], %[sy0]\n\t"
                "v_sub_f32 %[dy10], %[yi0], %[sy1]\n\t"
                "v_sub_f32 %[dy11], %[yi1], %[sy1]\n\t"
                "v_sub_f32 %[dy20], %[yi0], %[sy2]\n\t"
                "v_sub_f32 %[dy21], %[yi1], %[sy2]\n\t"
                "v_sub_f32 %[dy30], %[yi0], %[sy3]\n\t"
                "v_sub_f32 %[dy31], %[yi1], %[sy3]\n\t"
                "v_sub_f32 %[dz00], %[zi0], %[sz0]\n\t"
                "v_sub_f32 %[dz01], %[zi1], %[sz0]\n\t"
                "v_sub_f32 %[dz10], %[zi0], %[sz1]\n\t"
                "v_sub_f32 %[dz11], %[zi1], %[sz1]\n\t"
                "v_sub_f32 %[dz20], %[zi0], %[sz2]\n\t"
                "v_sub_f32 %[dz21], %[zi1], %[sz2]\n\t"
                "v_sub_f32 %[dz30], %[zi0], %[sz3]\n\t"
                "v_sub_f32 %[dz31], %[zi1], %[sz3]\n\t"
                "v_fma_f32 %[r00], %[dx00], %[dx00], %[gd]\n\t"
                "v_fma_f32 %[r01], %[dx01], %[dx01], %[gd]\n\t"
                "v_fma_f32 %[r10], %[dx10], %[dx10], %[gd]\n\t"
                "v_fma_f32 %[r11], %[dx11], %[dx11], %[gd]\n\t"
                "v_fma_f32 %[r20], %[dx20], %[dx20], %[gd]\n\t"
                "v_fma_f32 %[r21], %[dx21], %[dx21], %[gd]\n\t"
                "v_fma_f32 %[r30], %[dx30], %[dx30], %[gd]\n\t"
                "v_fma_f32 %[r31], %[dx31], %[dx31], %[gd]\n\t"
                "v_fmac_f32 %[r00], %[dy00], %[dy00]\n\t"
                "v_fmac_f32 %[r01], %[dy01], %[dy01]\n\t"
                "v_fmac_f32 %[r10], %[dy10], %[dy10]\n\t"
                "v_fmac_f32 %[r11], %[dy11], %[dy11]\n\t"
                "v_fmac_f32 %[r20], %[dy20], %[dy20]\n\t"
                "v_fmac_f32 %[r21], %[dy21], %[dy21]\n\t"
                "v_fmac_f32 %[r30], %[dy30], %[dy30]\n\t"
                "v_fmac_f32 %[r31], %[dy31], %[dy31]\n\t"
                "v_fmac_f32 %[r00], %[dz00], %[dz00]\n\t"
                "v_fmac_f32 %[r01], %[dz01], %[dz01]\n\t"
                "v_fmac_f32 %[r10], %[dz10], %[dz10]\n\t"
                "v_fmac_f32 %[r11], %[dz11], %[dz11]\n\t"
                "v_fmac_f32 %[r20], %[dz20], %[dz20]\n\t"
                "v_fmac_f32 %[r21], %[dz21], %[dz21]\n\t"
                "v_fmac_f32 %[r30], %[dz30], %[dz30]\n\t"
                "v_fmac_f32 %[r31], %[dz31], %[dz31]\n\t"
                "v_rsq_f32 %[w00], %[r00]\n\t"
                "v_rsq_f32 %[w01], %[r01]\n\t"
                "v_rsq_f32 %[w10], %[r10]\n\t"
                "v_rsq_f32 %[w11], %[r11]\n\t"
                "v_rsq_f32 %[w20], %[r20]\n\t"
                "v_rsq_f32 %[w21], %[r21]\n\t"
                "v_rsq_f32 %[w30], %[r30]\n\t"
                "v_rsq_f32 %[w31], %[r31]\n\t"
                "v_fmac_f32 %[gx0], %[w00], %[dx00]\n\t"
                "v_fmac_f32 %[gy0], %[w00], %[dy00]\n\t"
                "v_fmac_f32 %[gz0], %[w00], %[dz00]\n\t"
                "v_fmac_f32 %[e0], %[w00], %[r00]\n\t"
                "v_fmac_f32 %[gx1], %[w01], %[dx01]\n\t"
                "v_fmac_f32 %[gy1], %[w01], %[dy01]\n\t"
                "v_fmac_f32 %[gz1], %[w01], %[dz01]\n\t"
                "v_fmac_f32 %[e1], %[w01], %[r01]\n\t"
                "v_fmac_f32 %[gx0], %[w10], %[dx10]\n\t"
                "v_fmac_f32 %[gy0], %[w10], %[dy10]\n\t"
                "v_fmac_f32 %[gz0], %[w10], %[dz10]\n\t"
                "v_fmac_f32 %[e0], %[w10], %[r10]\n\t"
                "v_fmac_f32 %[gx1], %[w11], %[dx11]\n\t"
                "v_fmac_f32 %[gy1], %[w11], %[dy11]\n\t"
                "v_fmac_f32 %[gz1], %[w11], %[dz11]\n\t"
                "v_fmac_f32 %[e1], %[w11], %[r11]\n\t"
                "v_fmac_f32 %[gx0], %[w20], %[dx20]\n\t"
                "v_fmac_f32 %[gy0], %[w20], %[dy20]\n\t"
                "v_fmac_f32 %[gz0], %[w20], %[dz20]\n\t"
                "v_fmac_f32 %[e0], %[w20], %[r20]\n\t"
                "v_fmac_f32 %[gx1], %[w21], %[dx21]\n\t"
                "v_fmac_f32 %[gy1], %[w21], %[dy21]\n\t"
                "v_fmac_f32 %[gz1], %[w21], %[dz21]\n\t"
                "v_fmac_f32 %[e1], %[w21], %[r21]\n\t"
                "v_fmac_f32 %[gx0], %[w30], %[dx30]\n\t"
                "v_fmac_f32 %[gy0], %[w30], %[dy30]\n\t"
                "v_fmac_f32 %[gz0], %[w30], %[dz30]\n\t"
                "v_fmac_f32 %[e0], %[w30], %[r30]\n\t"
                "v_fmac_f32 %[gx1], %[w31], %[dx31]\n\t"
                "v_fmac_f32 %[gy1], %[w31], %[dy31]\n\t"
                "v_fmac_f32 %[gz1], %[w31], %[dz31]\n\t"
                "v_fmac_f32 %[e1], %[w31], %[r31]"
                : [dx00] "=&v"(dx[0][0]), [dy00] "=&v"(dy[0][0]), [dz00] "=&v"(dz[0][0]),
                  [r00] "=&v"(r[0][0]), [w00] "=&v"(w[0][0]), [dx01] "=&v"(dx[0][1]),
                  [dy01] "=&v"(dy[0][1]), [dz01] "=&v"(dz[0][1]), [r01] "=&v"(r[0][1]),
                  [w01] "=&v"(w[0][1]), [dx10] "=&v"(dx[1][0]), [dy10] "=&v"(dy[1][0]),
                  [dz10] "=&v"(dz[1][0]), [r10] "=&v"(r[1][0]), [w10] "=&v"(w[1][0]),
                  [dx11] "=&v"(dx[1][1]), [dy11] "=&v"(dy[1][1]), [dz11] "=&v"(dz[1][1]),
                  [r11] "=&v"(r[1][1]), [w11] "=&v"(w[1][1]), [dx20] "=&v"(dx[2][0]),
                  [dy20] "=&v"(dy[2][0]), [dz20] "=&v"(dz[2][0]), [r20] "=&v"(r[2][0]),
                  [w20] "=&v"(w[2][0]), [dx21] "=&v"(dx[2][1]), [dy21] "=&v"(dy[2][1]),
                  [dz21] "=&v"(dz[2][1]), [r21] "=&v"(r[2][1]), [w21] "=&v"(w[2][1]),
                  [dx30] "=&v"(dx[3][0]), [dy30] "=&v"(dy[3][0]), [dz30] "=&v"(dz[3][0]),
                  [r30] "=&v"(r[3][0]), [w30] "=&v"(w[3][0]), [dx31] "=&v"(dx[3][1]),
                  [dy31] "=&v"(dy[3][1]), [dz31] "=&v"(dz[3][1]), [r31] "=&v"(r[3][1]),
                  [w31] "=&v"(w[3][1]), [gx0] "+v"(gx0), [gy0] "+v"(gy0), [gz0] "+v"(gz0),
                  [gx1] "+v"(gx1), [gy1] "+v"(gy1), [gz1] "+v"(gz1), [e0] "+v"(e0),
                  [e1] "+v"(e1)
                : [xi0] "v"(xi0), [yi0] "v"(yi0), [zi0] "v"(zi0), [xi1] "v"(xi1),
                  [yi1] "v"(yi1), [zi1] "v"(zi1), [sx0] "v"(sx[0]), [sy0] "v"(sy[0]),
                  [sz0] "v"(sz[0]), [sx1] "v"(sx[1]), [sy1] "v"(sy[1]), [sz1] "v"(sz[1]),
                  [sx2] "v"(sx[2]), [sy2] "v"(sy[2]), [sz2] "v"(sz[2]), [sx3] "v"(sx[3]),
                  [sy3] "v"(sy[3]), [sz3] "v"(sz[3]), [gd] "v"(guard));
        } else if constexpr (VARIANT == 1) {
            asm volatile(
                "v_sub_f32 %[dx00], %[xi0], %[sx0]\n\t"
                "v_sub_f32 %[dx01], %[xi1], %[sx0]\n\t"
                "v_sub_f32 %[dx10], %[xi0], %[sx1]\n\t"
                "v_sub_f32 %[dx11], %[xi1], %[sx1]\n\t"
                "v_sub_f32 %[dx20], %[xi0], %[sx2]\n\t"
                "v_sub_f32 %[dx21], %[xi1], %[sx2]\n\t"
                "v_sub_f32 %[dx30], %[xi0], %[sx3]\n\t"
                "v_sub_f32 %[dx31], %[xi1], %[sx3]\n\t"
                "v_sub_f32 %[dy00], %[yi0], %[sy0]\n\t"
                "v_sub_f32 %[dy01], %[yi1], %[sy0]\n\t"
                "v_sub_f32 %[dy10], %[yi0], %[sy1]\n\t"
                "v_sub_f32 %[dy11], %[yi1], %[sy1]\n\t"
                "v_sub_f32 %[dy20], %[yi0], %[sy2]\n\t"
                "v_sub_f32 %[dy21], %[yi1], %[sy2]\n\t"
                "v_sub_f32 %[dy30], %[yi0], %[sy3]\n\t"
                "v_sub_f32 %[dy31], %[yi1], %[sy3]\n\t"
                "v_sub_f32 %[dz00], %[zi0], %[sz0]\n\t"
                "v_sub_f32 %[dz01], %[zi1], %[sz0]\n\t"
                "v_sub_f32 %[dz10], %[zi0], %[sz1]\n\t"
                "v_sub_f32 %[dz11], %[zi1], %[sz1]\n\t"
                "v_sub_f32 %[dz20], %[zi0], %[sz2]\n\t"
                "v_sub_f32 %[dz21], %[zi1], %[sz2]\n\t"
                "v_sub_f32 %[dz30], %[zi0], %[sz3]\n\t"
                "v_sub_f32 %[dz31], %[zi1], %[sz3]\n\t"
                "v_fma_f32 %[r00], %[dx00], %[dx00], %[gd]\n\t"
                "v_fma_f32 %[r01], %[dx01], %[dx01], %[gd]\n\t"
                "v_fma_f32 %[r10], %[dx10], %[dx10], %[gd]\n\t"
                "v_fma_f32 %[r11], %[dx11], %[dx11], %[gd]\n\t"
                "v_fma_f32 %[r20], %[dx20], %[dx20], %[gd]\n\t"
                "v_fma_f32 %[r21], %[dx21], %[dx21], %[gd]\n\t"
                "v_fma_f32 %[r30], %[dx30], %[dx30], %[gd]\n\t"
                "v_fma_f32 %[r31], %[dx31], %[dx31], %[gd]\n\t"
                "v_fmac_f32 %[r00], %[dy00], %[dy00]\n\t"
                "v_fmac_f32 %[r01], %[dy01], %[dy01]\n\t"
                "v_fmac_f32 %[r10], %[dy10], %[dy10]\n\t"
                "v_fmac_f32 %[r11], %[dy11], %[dy11]\n\t"
                "v_fmac_f32 %[r20], %[dy20], %[dy20]\n\t"
                "v_fmac_f32 %[r21], %[dy21], %[dy21]\n\t"
                "v_fmac_f32 %[r30], %[dy30], %[dy30]\n\t"
                "v_fmac_f32 %[r31], %[dy31], %[dy31]\n\t"
                "v_fmac_f32 %[r00], %[dz00], %[dz00]\n\t"
                "v_fmac_f32 %[r01], %[dz01], %[dz01]\n\t"
                "v_fmac_f32 %[r10], %[dz10], %[dz10]\n\t"
                "v_fmac_f32 %[r11], %[dz11], %[dz11]\n\t"
                "v_fmac_f32 %[r20], %[dz20], %[dz20]\n\t"
                "v_fmac_f32 %[r21], %[dz21], %[dz21]\n\t"
                "v_fmac_f32 %[r30], %[dz30], %[dz30]\n\t"
                "v_fmac_f32 %[r31], %[dz31], %[dz31]\n\t"
                "v_fmac_f32 %[gx0], %[r00], %[dx00]\n\t"
                "v_fmac_f32 %[gy0], %[r00], %[dy00]\n\t"
                "v_fmac_f32 %[gz0], %[r00], %[dz00]\n\t"
                "v_fmac_f32 %[e0], %[r00], %[r00]\n\t"
                "v_fmac_f32 %[gx1], %[r01], %[dx01]\n\t"
                "v_fmac_f32 %[gy1], %[r01], %[dy01]\n\t"
                "v_fmac_f32 %[gz1], %[r01], %[dz01]\n\t"
                "v_fmac_f32 %[e1], %[r01], %[r01]\n\t"
                "v_fmac_f32 %[gx0], %[r10], %[dx10]\n\t"
                "v_fmac_f32 %[gy0], %[r10], %[dy10]\n\t"
                "v_fmac_f32 %[gz0], %[r10], %[dz10]\n\t"
                "v_fmac_f32 %[e0], %[r10], %[r10]\n\t"
                "v_fmac_f32 %[gx1], %[r11], %[dx11]\n\t"
                "v_fmac_f32 %[gy1], %[r11], %[dy11]\n\t"
                "v_fmac_f32 %[gz1], %[r11], %[dz11]\n\t"
                "v_fmac_f32 %[e1], %[r11], %[r11]\n\t"
                "v_fmac_f32 %[gx0], %[r20], %[dx20]\n\t"
                "v_fmac_f32 %[gy0], %[r20], %[dy20]\n\t"
                "v_fmac_f32 %[gz0], %[r20], %[dz20]\n\t"
                "v_fmac_f32 %[e0], %[r20], %[r20]\n\t"
                "v_fmac_f32 %[gx1], %[r21], %[dx21]\n\t"
                "v_fmac_f32 %[gy1], %[r21], %[dy21]\n\t"
                "v_fmac_f32 %[gz1], %[r21], %[dz21]\n\t"
                "v_fmac_f32 %[e1], %[r21], %[r21]\n\t"
                "v_fmac_f32 %[gx0], %[r30], %[dx30]\n\t"
                "v_fmac_f32 %[gy0], %[r30], %[dy30]\n\t"
                "v_fmac_f32 %[gz0], %[r30], %[dz30]\n\t"
                "v_fmac_f32 %[e0], %[r30], %[r30]\n\t"
                "v_fmac_f32 %[gx1], %[r31], %[dx31]\n\t"
                "v_fmac_f32 %[gy1], %[r31], %[dy31]\n\t"
                "v_fmac_f32 %[gz1], %[r31], %[dz31]\n\t"
                "v_fmac_f32 %[e1], %[r31], %[r31]"
                : [dx00] "=&v"(dx[0][0]), [dy00] "=&v"(dy[0][0]), [dz00] "=&v"(dz[0][0]),
                  [r00] "=&v"(r[0][0]), [dx01] "=&v"(dx[0][1]), [dy01] "=&v"(dy[0][1]),
                  [dz01] "=&v"(dz[0][1]), [r01] "=&v"(r[0][1]), [dx10] "=&v"(dx[1][0]),
                  [dy10] "=&v"(dy[1][0]), [dz10] "=&v"(dz[1][0]), [r10] "=&v"(r[1][0]),
                  [dx11] "=&v"(dx[1][1]), [dy11] "=&v"(dy[1][1]), [dz11] "=&v"(dz[1][1]),
                  [r11] "=&v"(r[1][1]), [dx20] "=&v"(dx[2][0]), [dy20] "=&v"(dy[2][0]),
                  [dz20] "=&v"(dz[2][0]), [r20] "=&v"(r[2][0]), [dx21] "=&v"(dx[2][1]),
                  [dy21] "=&v"(dy[2][1]), [dz21] "=&v"(dz[2][1]), [r21] "=&v"(r[2][1]),
                  [dx30] "=&v"(dx[3][0]), [dy30] "=&v"(dy[3][0]), [dz30] "=&v"(dz[3][0]),
                  [r30] "=&v"(r[3][0]), [dx31] "=&v"(dx[3][1]), [dy31] "=&v"(dy[3][1]),
                  [dz31] "=&v"(dz[3][1]), [r31] "=&v"(r[3][1]), [gx0] "+v"(gx0),
                  [gy0] "+v"(gy0), [gz0] "+v"(gz0), [gx1] "+v"(gx1), [gy1] "+v"(gy1),
                  [gz1] "+v"(gz1), [e0] "+v"(e0), [e1] "+v"(e1)
                : [xi0] "v"(xi0), [yi0] "v"(yi0), [zi0] "v"(zi0), [xi1] "v"(xi1),
                  [yi1] "v"(yi1), [zi1] "v"(zi1), [sx0] "v"(sx[0]), [sy0] "v"(sy[0]),
                  [sz0] "v"(sz[0]), [sx1] "v"(sx[1]), [sy1] "v"(sy[1]), [sz1] "v"(sz[1]),
                  [sx2] "v"(sx[2]), [sy2] "v"(sy[2]), [sz2] "v"(sz[2]), [sx3] "v"(sx[3]),
                  [sy3] "v"(sy[3]), [sz3] "v"(sz[3]), [gd] "v"(guard));
        } else {
            asm volatile(
                "v_rsq_f32 %[w00], %[sx0]\n\t"
                "v_rsq_f32 %[w01], %[sy0]\n\t"
                "v_rsq_f32 %[w10], %[sx1]\n\t"
                "v_rsq_f32 %[w11], %[sy1]\n\t"
                "v_rsq_f32 %[w20], %[sx2]\n\t"
                "v_rsq_f32 %[w21], %[sy2]\n\t"
                "v_rsq_f32 %[w30], %[sx3]\n\t"
                "v_rsq_f32 %[w31], %[sy3]\n\t"
                "v_fmac_f32 %[e0], %[w00], %[sx0]\n\t"
                "v_fmac_f32 %[e1], %[w01], %[sy0]\n\t"
                "v_fmac_f32 %[e0], %[w10], %[sx1]\n\t"
                "v_fmac_f32 %[e1], %[w11], %[sy1]\n\t"
                "v_fmac_f32 %[e0], %[w20], %[sx2]\n\t"
                "v_fmac_f32 %[e1], %[w21], %[sy2]\n\t"
                "v_fmac_f32 %[e0], %[w30], %[sx3]\n\t"
                "v_fmac_f32 %[e1], %[w31], %[sy3]"
                : [w00] "=&v"(w[0][0]), [w01] "=&v"(w[0][1]), [w10] "=&v"(w[1][0]),
                  [w11] "=&v"(w[1][1]), [w20] "=&v"(w[2][0]), [w21] "=&v"(w[2][1]),
                  [w30] "=&v"(w[3][0]), [w31] "=&v"(w[3][1]), [e0] "+v"(e0), [e1] "+v"(e1)
                : [sx0] "v"(sx[0]), [sy0] "v"(sy[0]), [sx1] "v"(sx[1]), [sy1] "v"(sy[1]),
                  [sx2] "v"(sx[2]), [sy2] "v"(sy[2]), [sx3] "v"(sx[3]), [sy3] "v"(sy[3]));
        }
    }
    (void)xi0; (void)yi0; (void)zi0; (void)xi1; (void)yi1; (void)zi1; (void)guard;
    (void)dx; (void)dy; (void)dz; (void)r; (void)w;
    const int64_t t = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
    out[t] = ((gx0 + gy0) + (gz0 + e0)) + ((gx1 + gy1) + (gz1 + e1));
}

}  // namespace

int64_t probe_out_elements(int64_t blocks) { return blocks * kProbeThreads; }

int64_t probe_pairs(int64_t blocks, int iters)
{
    // two targets against kProbeSources sources per thread and iteration
    return blocks * kProbeThreads * (int64_t)iters * kProbeSources * 2;
}

hipError_t launch_pair_mix_probe(int variant, float *out, int64_t blocks, int iters,
                                 hipStream_t s)
{
    if (blocks < 1 || blocks > (int64_t(1) << 20) || iters < 1)
        return hipErrorInvalidValue;
    switch (variant) {
    case 0:
        hipLaunchKernelGGL(pair_mix_probe<0>, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s,
                           out, iters);
        break;
    case 1:
        hipLaunchKernelGGL(pair_mix_probe<1>, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s,
                           out, iters);
        break;
    case 2:
        hipLaunchKernelGGL(pair_mix_probe<2>, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s,
                           out, iters);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace spk
