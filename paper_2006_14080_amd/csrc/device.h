// Device-side helpers shared by the HIP kernels of libmriadmm (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mri {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr double kInv2Pi = 0.15915494309189533576888376337251436;  // 1 / (2 pi)

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
// c + a b, each part as two fused multiply-adds
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// exp(-2 pi i f r) for a sample frequency f in revolutions per pixel and an
// integer pixel offset r (eq. (1), Alg. 1).  The argument is reduced in FP64:
// t = f r - rint(f r) is exact up to one FP64 rounding of the product, which
// keeps |phase| errors near 1e-7 rad even where |omega r| reaches hundreds of
// radians; only sin/cos of 2 pi t in [-pi, pi] are evaluated in FP32.
__device__ __forceinline__ float2 expi_neg(double f, double r) {
    double t = f * r;
    t -= rint(t);
    float s, c;
    sincospif(2.0f * static_cast<float>(t), &s, &c);
    return make_float2(c, -s);
}
// exp(+2 pi i f r), the conjugate phase used by the adjoint.
__device__ __forceinline__ float2 expi_pos(double f, double r) {
    double t = f * r;
    t -= rint(t);
    float s, c;
    sincospif(2.0f * static_cast<float>(t), &s, &c);
    return make_float2(c, s);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide FP64 sum in a fixed order (wave shuffles, then waves in index
// order).  Every thread of the block must call it; thread 0 gets the total.
template <int NWAVES>
__device__ __forceinline__ double block_sum(double v, double* smem) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) smem[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NWAVES; ++i) t += smem[i];
    }
    __syncthreads();
    return t;
}

// Workgroup index remap so that consecutive tiles run on the same XCD.
// Workgroups are dispatched round-robin over the 8 XCDs (wg % 8); tiles that
// share operands (same slice and coil) are numbered consecutively, so this
// keeps their shared operands in one XCD's L2.
__device__ __forceinline__ int xcd_remap(int wg, int total) {
    const int per = total >> 3;
    if (wg < (per << 3)) return (wg & 7) * per + (wg >> 3);
    return wg;
}

}  // namespace mri
