// Phase factors exp(-/+ 2 pi i f r) of the non-uniform DFT (eq. (1), Alg. 1),
// generated on the fly from the trajectory.
//
// Range reduction is done in FP64: t = f r in revolutions (f = omega / 2 pi,
// r an integer pixel offset), u = 4 t, n = rint(u), v = u - n in [-1/2, 1/2];
// n mod 4 selects the quadrant and theta = v pi / 2 lies in [-pi/4, pi/4].
// Only sin/cos of theta are evaluated in FP32, by their Taylor polynomials
// (sin to theta^9, cos to theta^8; truncation below 3e-8 on the octant).
// Phase errors therefore stay near 1e-7 rad even where |omega r| reaches
// hundreds of radians, and both signs share the same reduction.
#pragma once

#include <hip/hip_runtime.h>

namespace mri {

struct SinCos {
    float s, c;
};

// The evaluation in three steps (so a kernel can spread them between other
// work): reduction, the two polynomials, the quadrant rotation.
struct QuarterTurn {
    float th;    // reduced angle in radians, [-pi/4, pi/4]
    int q;       // quadrant, 0..3
};
__device__ __forceinline__ QuarterTurn reduce_quarter_turns(double t4) {
    const double n = rint(t4);
    const float v = static_cast<float>(t4 - n);           // [-0.5, 0.5] quarter turns
    return {v * 1.57079632679489661923f, static_cast<int>(n) & 3};
}
// sin and cos of th on [-pi/4, pi/4].
__device__ __forceinline__ SinCos sincos_octant(float th) {
    const float t2 = th * th;
    // sin th = th (1 - t2/3! + t2^2/5! - t2^3/7! + t2^4/9!)
    float ps = fmaf(t2, 2.7557319224e-6f, -1.9841269841e-4f);
    ps = fmaf(t2, ps, 8.3333333333e-3f);
    ps = fmaf(t2, ps, -1.6666666667e-1f);
    const float sn = fmaf(th * t2, ps, th);
    // cos th = 1 - t2/2! + t2^2/4! - t2^3/6! + t2^4/8!
    float pc = fmaf(t2, 2.4801587302e-5f, -1.3888888889e-3f);
    pc = fmaf(t2, pc, 4.1666666667e-2f);
    pc = fmaf(t2, pc, -0.5f);
    const float cs = fmaf(t2, pc, 1.0f);
    return {sn, cs};
}
// Rotate by q quarter turns: (s, c) -> q=1: (c, -s), q=2: (-s, -c), q=3: (-c, s).
__device__ __forceinline__ SinCos rotate_quadrant(SinCos sc, int q) {
    SinCos r;
    const bool swap = q & 1;
    const float a = swap ? sc.c : sc.s;
    const float b = swap ? sc.s : sc.c;
    r.s = (q & 2) ? -a : a;
    r.c = ((q + 1) & 2) ? -b : b;
    return r;
}

// sin and cos of 2 pi * t4 / 4 (t4 = 4 f r, in quarter turns), FP64 reduction.
__device__ __forceinline__ SinCos sincos_quarter_turns(double t4) {
    const QuarterTurn r = reduce_quarter_turns(t4);
    return rotate_quadrant(sincos_octant(r.th), r.q);
}

// exp(-2 pi i f r) with f4 = 4 f precomputed per sample.
__device__ __forceinline__ float2 phase_neg(double f4, double r) {
    const SinCos sc = sincos_quarter_turns(f4 * r);
    return make_float2(sc.c, -sc.s);
}

// exp(+2 pi i f r).
__device__ __forceinline__ float2 phase_pos(double f4, double r) {
    const SinCos sc = sincos_quarter_turns(f4 * r);
    return make_float2(sc.c, sc.s);
}

// 4 / (2 pi): turns radians per pixel into quarter turns per pixel.
constexpr double kQuarterTurnsPerRad = 0.63661977236758134307553505349006;

}  // namespace mri
