// Forward and adjoint multi-coil non-uniform DFT as dense complex matrix
// products on MFMA (eq. (1)-(2), Alg. 1, Alg. 3), gfx950.
//
// Both operators use the separable phase of Alg. 1,
//   exp(-i (w0 x + w1 y)) = Ex[k][x] * Ey[k][y],
// and never store a phase matrix: every phase tile is formed in LDS one
// K-step ahead of the matrix cores, from the trajectory (forward, phase.h) or
// from the separable factor tables built from it once per trajectory
// (adjoint, k_adj_phases).
//
// Forward, per slice b and coil g:  T[y][k] = sum_x I[y][x] Ex[k][x] with
// I = s_g (.) x_b (formed by a pre-pass, k_coil_weight), then
// y[g][k] = sum_y T[y][k] Ey[k][y] in the epilogue.  GEMM M = y, N = k, K = x.
//
// Adjoint, per slice:  X_g[y][x] = sum_k W[(g,y)][k] conj(Ex[k][x]) with
// W = y[g][k] conj(Ey[k][y]) generated as the A operand; the epilogue forms
// sum_g conj(s_g[y][x]) X_g[y][x].  GEMM M = (coil, y), N = x, K = samples,
// split over sample ranges; partial images are summed in a fixed order
// afterwards.
//
// Complex products on real MFMA (v_mfma_f32_32x32x2_f32): the two K-slots of
// the instruction carry the real and imaginary parts, so with the A operand
// [Ar, Ai] in slots (0, 1):
//   C_re += [Ar, Ai] . [Br; -Bi],   C_im += [Ar, Ai] . [Bi; Br]
// and a complex multiply-add costs exactly its 8 real flops.  Operands sit in
// LDS as planes (Ar, Ai | Br, Bi, -Bi) with K contiguous, so every lane loads
// four K values with one 16-byte read and no per-product select.
//
// Pipeline: two LDS stages; while the matrix cores consume stage s, global
// loads for stage s+1 are in flight and its phase tiles are generated; one
// barrier per K-step.
#include "device.h"
#include "internal.h"
#include "phase.h"

namespace mri {
namespace {

constexpr int kThreads = 256;             // 4 waves: 2 (rows) x 2 (cols)
constexpr int kThreads8 = 512;            // split-form adjoint: 8 waves, 2 (rows) x 4 (cols)
constexpr int kAdjCols8 = kAdjCols;       // its x columns per tile (128)
constexpr int kNT = 4;                    // 32-row MFMA tiles per wave
constexpr int kRows = 2 * kNT * 32;       // GEMM rows per pass (256)
constexpr int KC = kKStep;                // complex K values per stage (8)
constexpr int RS = KC + 4;                // LDS row stride in floats: conflict-free 16-byte reads
constexpr int kXAnchor = 8;               // forward: K-steps per exactly generated step phase

__device__ __forceinline__ int find_item(const NudftTable& t, int tile) {
    int i = 0;
    while (i + 1 < t.nitems && tile >= t.it[i + 1].tile_begin) ++i;
    return i;
}

// ---------------------------------------------------------------------------
// Operand policies.  A stage holds kRows GEMM rows x KC complex K values of
// the A operand; B holds 64 columns of the B operand in the two forms
// (Br, -Bi) and (Bi, Br) that produce the real and imaginary accumulators.
//   store_a(stage, row, v[KC])        one row of A, K values 0..KC-1
//   store_b(stage, col, kp, e0, e1)   B column col, K values kp, kp+1
//   mma<NT>(a, b, arow0, bcol0, lane, ntile, acc_re, acc_im)  NT row tiles
//   from row arow0 (skipped as a whole when the wave has no live tile).
// ---------------------------------------------------------------------------

// FP32: v_mfma_f32_32x32x2_f32, K-slot 0 = real part, slot 1 = imaginary.
// LDS planes with K contiguous: A (Ar, Ai); B (Br, Bi, -Bi).  Lanes 0-31 read
// plane Ar / Br / Bi, lanes 32-63 read Ai / -Bi / Br, four K values per read.
struct PolF32 {
    static constexpr bool kPresplitA = false;        // forward A staged from the FP32 coil-weighted image
    static constexpr bool kScaled = false;
    static constexpr float kBScale = 1.0f;
    static constexpr int kABytes = 2 * kRows * RS * 4;
    static constexpr int kBBytes = 3 * 64 * RS * 4;

    __device__ __forceinline__ static void store_a(char* st, int row, const float2 (&v)[KC]) {
        float* re = reinterpret_cast<float*>(st) + row * RS;
        float* im = re + kRows * RS;
#pragma unroll
        for (int j = 0; j < KC; j += 4) {
            *reinterpret_cast<float4*>(re + j) = make_float4(v[j].x, v[j + 1].x, v[j + 2].x, v[j + 3].x);
            *reinterpret_cast<float4*>(im + j) = make_float4(v[j].y, v[j + 1].y, v[j + 2].y, v[j + 3].y);
        }
    }
    // A stage row, K values 4h..4h+3 only (re and im planes).
    __device__ __forceinline__ static void store_a_half(char* st, int row, int rows, int h, const float2* v) {
        float* re = reinterpret_cast<float*>(st) + row * RS + 4 * h;
        float* im = re + rows * RS;
        *reinterpret_cast<float4*>(re) = make_float4(v[0].x, v[1].x, v[2].x, v[3].x);
        *reinterpret_cast<float4*>(im) = make_float4(v[0].y, v[1].y, v[2].y, v[3].y);
    }
    // B stages of BC columns: planes Br, Bi, -Bi of [BC][RS] floats.
    template <int BC>
    static constexpr int bbytes() { return 3 * BC * RS * 4; }
    template <int BC = 64>
    __device__ __forceinline__ static void store_b(char* st, int col, int kp, float2 e0, float2 e1) {
        float* p = reinterpret_cast<float*>(st) + col * RS + kp;
        *reinterpret_cast<float2*>(p) = make_float2(e0.x, e1.x);
        *reinterpret_cast<float2*>(p + BC * RS) = make_float2(e0.y, e1.y);
        *reinterpret_cast<float2*>(p + 2 * BC * RS) = make_float2(-e0.y, -e1.y);
    }
    template <int NT, int BC = 64>
    __device__ __forceinline__ static void mma(const char* a, const char* b, int arow0, int bcol0, int lane,
                                               int ntile, floatx16 (&acc_re)[NT], floatx16 (&acc_im)[NT]) {
        const int h = lane >> 5, l32 = lane & 31;
        const float* ap = reinterpret_cast<const float*>(a) + (h * kRows + arow0 + l32) * RS;
        const float* bre = reinterpret_cast<const float*>(b) + ((h ? 2 : 0) * BC + bcol0 + l32) * RS;
        const float* bim = reinterpret_cast<const float*>(b) + ((h ? 0 : 1) * BC + bcol0 + l32) * RS;
        // A wave with no live row tile skips the stage; otherwise all NT tiles
        // run (rows past the valid range hold zeros) as one branch-free burst.
        if (__builtin_amdgcn_readfirstlane(ntile) == 0) return;
#pragma unroll
        for (int kq = 0; kq < KC; kq += 4) {
            const floatx4 br = *reinterpret_cast<const floatx4*>(bre + kq);
            const floatx4 bi = *reinterpret_cast<const floatx4*>(bim + kq);
            // Row tile outer: each tile's A operand is read just before its eight
            // MFMAs (re and im alternate, so dependent MFMAs are two apart).
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const floatx4 av = *reinterpret_cast<const floatx4*>(ap + t * 32 * RS + kq);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc_re[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[j], br[j], acc_re[t], 0, 0, 0);
                    acc_im[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[j], bi[j], acc_im[t], 0, 0, 0);
                }
            }
        }
    }
};

// Split products (Sec. II-A "decomposition and accumulation"): each FP32
// value a = hi + lo with hi = T(a), lo = T(a - hi) (round to nearest even) for
// a 16-bit type T; a real product a b is formed as hi_a hi_b + lo_a hi_b +
// hi_a lo_b with FP32 accumulation.  v_mfma_f32_32x32x16_{bf16,f16} take 8
// K-slots per lane half: lane half h holds complex K values 4h..4h+3 as four
// 32-bit words, each one converted (re, im) pair, so no word is repacked.
// A 16-byte chunk holds one part (hi or lo) of those four values:
//   A    : (ArH, AiH) x4   or  (ArL, AiL) x4
//   B_re : (BrH, -BiH) x4  or  (BrL, -BiL) x4   -> Ar Br - Ai Bi
//   B_im : (BiH, BrH) x4   or  (BiL, BrL) x4    -> Ar Bi + Ai Br
// and the three products of 8 complex K values are three MFMAs per
// accumulator: (A hi, B hi), (A lo, B hi), (A hi, B lo).  Each part is stored
// and read from LDS once (two chunks per lane half instead of three, so a
// third less LDS traffic than a slot order that repeats hi words within a
// K value); LDS holds A [h][part][row], B [var][h][part][col].
//
// T = bf16 (the paper's form): 8 significant bits per part, so hi + lo holds
// about 16 bits of each operand; it needs no scaling (bf16 has the FP32
// exponent range).
// T = fp16 (same MFMA rate on gfx950): 11 bits per part, about 22 bits per
// operand, but a narrow exponent range, so operands are scaled by powers of
// two (exact) into [2^14, 2^15) before the split and the results scaled back:
// phases by 2^14; the forward's coil-weighted image per row (pre-pass); the
// adjoint's data per coil over each workgroup's sample range.  Parts that
// fall below fp16's normal range then carry less than 2^-28 of an operand's
// magnitude.
template <class T, bool Scaled>
struct PolSplit {
    typedef T vec8 __attribute__((ext_vector_type(8)));
    typedef T vec2 __attribute__((ext_vector_type(2)));
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    static constexpr bool kPresplitA = true;         // forward A pre-split into operand chunks once per call
    static constexpr bool kScaled = Scaled;
    static constexpr float kBScale = Scaled ? 16384.0f : 1.0f;   // phases (|e| <= 1) -> [-2^14, 2^14]
    static constexpr int kChunks = 4;                // 16-byte chunks per row and K-step: (lane half, part)
    static constexpr int kABytes = kChunks * kRows * 16;
    static constexpr int kBBytes = 2 * kChunks * 64 * 16;
    static_assert(kChunks * 16 == kSplitUnitBytes, "pre-split unit size");

    // (hi, lo) words of the pair (a, b): hi = [T(a), T(b)], lo = [T(a - hi_a), T(b - hi_b)].
    struct Words {
        uint32_t hi, lo;
    };
    __device__ __forceinline__ static Words split2(float a, float b) {
        uint32_t hw, lw;
        float ha, hb;
        if constexpr (__is_same(T, __bf16)) {
            // A bf16 is the top half of an FP32: read both back from the packed
            // word.  The conversion is written as the instruction itself so the
            // compiler keeps the one packed result instead of converting each
            // half again.
            asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(hw) : "v"(a), "v"(b));
            ha = __builtin_bit_cast(float, hw << 16);
            hb = __builtin_bit_cast(float, hw & 0xffff0000u);
            const vec2 l = {static_cast<T>(a - ha), static_cast<T>(b - hb)};
            lw = __builtin_bit_cast(uint32_t, l);
        } else {
            // Both halves in one packed conversion (round to nearest even, as
            // the per-component conversion), for the high and the low parts.
            asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(hw) : "v"(a), "v"(b));
            const vec2 h = __builtin_bit_cast(vec2, hw);
            ha = static_cast<float>(h.x);
            hb = static_cast<float>(h.y);
            asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(lw) : "v"(a - ha), "v"(b - hb));
        }
        return {hw, lw};
    }
    // [x, y] -> [-y, x] on the two 16-bit halves (swap, then negate the low half).
    __device__ __forceinline__ static uint32_t rot(uint32_t w) {
        return ((w >> 16) | (w << 16)) ^ 0x8000u;
    }
    __device__ __forceinline__ static floatx16 mfma(vec8 a, vec8 b, floatx16 c);

    // One row of A (K values 0..KC-1) as four 16-byte chunks; chunk (h, part)
    // of row r sits at ((h*2+part)*rows + r)*16.
    __device__ __forceinline__ static void store_a_rows(char* st, int row, int rows, const float2 (&v)[KC]) {
        store_a_half(st, row, rows, 0, v);
        store_a_half(st, row, rows, 1, v + 4);
    }
    // Chunks (h, hi) and (h, lo) of one row: K values 4h..4h+3 from v[0..3].
    __device__ __forceinline__ static void store_a_half(char* st, int row, int rows, int h, const float2* v) {
        uint32_t hi[4], lo[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const Words p = split2(v[q].x, v[q].y);
            hi[q] = p.hi;
            lo[q] = p.lo;
        }
        *reinterpret_cast<u32x4*>(st + ((int64_t)(h * 2) * rows + row) * 16) = u32x4{hi[0], hi[1], hi[2], hi[3]};
        *reinterpret_cast<u32x4*>(st + ((int64_t)(h * 2 + 1) * rows + row) * 16) = u32x4{lo[0], lo[1], lo[2], lo[3]};
    }
    __device__ __forceinline__ static void store_a(char* st, int row, const float2 (&v)[KC]) {
        store_a_rows(st, row, kRows, v);
    }
    // B column col, complex K values kp and kp+1 (kp even): words kp&3 and
    // (kp&3)+1 of the hi and lo chunks of both variants.
    template <int BC>
    static constexpr int bbytes() { return 2 * kChunks * BC * 16; }
    template <int BC = 64>
    __device__ __forceinline__ static void store_b(char* st, int col, int kp, float2 e0, float2 e1) {
        store_b_words<BC>(st, col, kp, split_b(e0), split_b(e1));
    }
    // [Br, -Bi] words of one B value; the caller passes the phase already
    // multiplied by kBScale (folded into a mask or a per-thread factor).
    __device__ __forceinline__ static Words split_b(float2 e) { return split2(e.x, -e.y); }
    // All four B words of one value e = (x, y) converted directly: for the
    // real output [x, -y] (hi, lo), for the imaginary output [y, x] (hi, lo),
    // which are the real words with halves swapped and the low half negated
    // (round to nearest even is symmetric, so the bits equal rot() of the
    // real words); the sign flips are source modifiers of the packed
    // conversions.  Fewer vector instructions than split_b plus rot(), but
    // four words stay live instead of two (used by the forward, whose
    // producer pieces keep them for one piece only).
    struct BWords {
        uint32_t rh, rl, ih, il;
    };
    __device__ __forceinline__ static BWords split_b4(float2 e) {
        const float x = e.x, y = e.y;
        BWords w;
        float hx, hy;
        if constexpr (__is_same(T, __bf16)) {
            asm("v_cvt_pk_bf16_f32 %0, %1, -%2" : "=v"(w.rh) : "v"(x), "v"(y));
            asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(w.ih) : "v"(y), "v"(x));
            hx = __builtin_bit_cast(float, w.ih & 0xffff0000u);
            hy = __builtin_bit_cast(float, w.ih << 16);
        } else {
            asm("v_cvt_pk_f16_f32 %0, %1, -%2" : "=v"(w.rh) : "v"(x), "v"(y));
            asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(w.ih) : "v"(y), "v"(x));
            const vec2 h = __builtin_bit_cast(vec2, w.ih);
            hx = static_cast<float>(h.y);
            hy = static_cast<float>(h.x);
        }
        const float dx = x - hx;
        const float dyn = hy - y;             // the low part of -y, as (-y) - (-hy)
        if constexpr (__is_same(T, __bf16)) {
            asm("v_cvt_pk_bf16_f32 %0, %1, %2" : "=v"(w.rl) : "v"(dx), "v"(dyn));
            asm("v_cvt_pk_bf16_f32 %0, -%1, %2" : "=v"(w.il) : "v"(dyn), "v"(dx));
        } else {
            asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(w.rl) : "v"(dx), "v"(dyn));
            asm("v_cvt_pk_f16_f32 %0, -%1, %2" : "=v"(w.il) : "v"(dyn), "v"(dx));
        }
        return w;
    }
    template <int BC>
    __device__ __forceinline__ static void store_b_words4(char* st, int col, int kp, BWords r0, BWords r1) {
        const int h = kp >> 2;
        char* re = st + ((h * 2) * BC + col) * 16 + (kp & 3) * 4;
        char* im = re + 2 * 2 * BC * 16;
        *reinterpret_cast<u32x2*>(re) = u32x2{r0.rh, r1.rh};
        *reinterpret_cast<u32x2*>(re + BC * 16) = u32x2{r0.rl, r1.rl};
        *reinterpret_cast<u32x2*>(im) = u32x2{r0.ih, r1.ih};
        *reinterpret_cast<u32x2*>(im + BC * 16) = u32x2{r0.il, r1.il};
    }
    // B stages hold BC columns: [var][h][part][col], 16 bytes per chunk.
    template <int BC>
    __device__ __forceinline__ static void store_b_words(char* st, int col, int kp, Words r0, Words r1) {
        const int h = kp >> 2;
        char* re = st + ((h * 2) * BC + col) * 16 + (kp & 3) * 4;
        char* im = re + 2 * 2 * BC * 16;
        *reinterpret_cast<u32x2*>(re) = u32x2{r0.hi, r1.hi};
        *reinterpret_cast<u32x2*>(re + BC * 16) = u32x2{r0.lo, r1.lo};
        *reinterpret_cast<u32x2*>(im) = u32x2{rot(r0.hi), rot(r1.hi)};
        *reinterpret_cast<u32x2*>(im + BC * 16) = u32x2{rot(r0.lo), rot(r1.lo)};
    }
    template <int NT, int BC = 64>
    __device__ __forceinline__ static void mma(const char* a, const char* b, int arow0, int bcol0, int lane,
                                               int ntile, floatx16 (&acc_re)[NT], floatx16 (&acc_im)[NT]) {
        const int h = lane >> 5, l32 = lane & 31;
        const char* bre = b + ((h * 2) * BC + bcol0 + l32) * 16;
        const char* bim = bre + 2 * 2 * BC * 16;
        const char* ap = a + ((h * 2) * kRows + arow0 + l32) * 16;
        if (__builtin_amdgcn_readfirstlane(ntile) == 0) return;   // see PolF32::mma
        // (A hi, B hi), (A lo, B hi), (A hi, B lo); re and im alternate, so
        // dependent MFMAs are 2 NT apart.
        const vec8 brh = *reinterpret_cast<const vec8*>(bre);
        const vec8 bih = *reinterpret_cast<const vec8*>(bim);
        vec8 ah[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) ah[t] = *reinterpret_cast<const vec8*>(ap + t * 32 * 16);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc_re[t] = mfma(ah[t], brh, acc_re[t]);
            acc_im[t] = mfma(ah[t], bih, acc_im[t]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const vec8 al = *reinterpret_cast<const vec8*>(ap + (kRows + t * 32) * 16);
            acc_re[t] = mfma(al, brh, acc_re[t]);
            acc_im[t] = mfma(al, bih, acc_im[t]);
        }
        const vec8 brl = *reinterpret_cast<const vec8*>(bre + BC * 16);
        const vec8 bil = *reinterpret_cast<const vec8*>(bim + BC * 16);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc_re[t] = mfma(ah[t], brl, acc_re[t]);
            acc_im[t] = mfma(ah[t], bil, acc_im[t]);
        }
    }
    // The same products with a producer interleaved: prod(i), i = 0..5, runs
    // with each sixth of the MFMAs.  Scheduling fences keep each piece of
    // vector work within its group of matrix-core instructions, and group
    // barriers alternate one MFMA with a few ALU instructions, so the SIMD
    // executes both at once instead of one burst after the other.  Every wave
    // runs all its tiles (a wave without live rows works on rows the epilogue
    // never reads): a skip branch would make the compiler copy the
    // accumulators where the two paths meet.
    //   kByTile false: the groups are (part, half of the tiles) and all
    //     operands are read up front (the forward: fewer waits);
    //   kByTile true: the MFMAs go tile by tile, (hi, hi), (lo, hi), (hi, lo)
    //     with re and im alternating, and a tile's A operands are read one
    //     group ahead, so only B and about two tiles of A are live (the
    //     adjoint, whose producers hold more registers).
    template <int NT, int BC, bool kByTile, class Prod>
    __device__ __forceinline__ static void mma_with(const char* a, const char* b, int arow0, int bcol0, int lane,
                                                    floatx16 (&acc_re)[NT], floatx16 (&acc_im)[NT], Prod&& prod) {
        const int h = lane >> 5, l32 = lane & 31;
        const char* bre = b + ((h * 2) * BC + bcol0 + l32) * 16;
        const char* bim = bre + 2 * 2 * BC * 16;
        const char* ap = a + ((h * 2) * kRows + arow0 + l32) * 16;
        const vec8 bh[2] = {*reinterpret_cast<const vec8*>(bre), *reinterpret_cast<const vec8*>(bim)};
        const vec8 bl[2] = {*reinterpret_cast<const vec8*>(bre + BC * 16),
                            *reinterpret_cast<const vec8*>(bim + BC * 16)};
        vec8 ah[NT], al[NT];
        if constexpr (!kByTile) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                ah[t] = *reinterpret_cast<const vec8*>(ap + t * 32 * 16);
                al[t] = *reinterpret_cast<const vec8*>(ap + (kRows + t * 32) * 16);
            }
        }
#pragma unroll
        for (int g = 0; g < 6; ++g) {
            if constexpr (kByTile) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int gt = (6 * t) / NT;          // group of tile t's first MFMA
                    if ((g == 0 && gt <= 1) || (g > 0 && gt == g + 1)) {
                        ah[t] = *reinterpret_cast<const vec8*>(ap + t * 32 * 16);
                        al[t] = *reinterpret_cast<const vec8*>(ap + (kRows + t * 32) * 16);
                    }
                }
#pragma unroll
                for (int i = g * NT; i < (g + 1) * NT; ++i) {
                    const int t = i / 6, part = (i % 6) / 2;
                    const vec8 av = part == 1 ? al[t] : ah[t];
                    if ((i & 1) == 0)
                        acc_re[t] = mfma(av, part == 2 ? bl[0] : bh[0], acc_re[t]);
                    else
                        acc_im[t] = mfma(av, part == 2 ? bl[1] : bh[1], acc_im[t]);
                }
            } else {
                const int part = g >> 1;
                const int t0 = (g & 1) ? NT / 2 : 0, t1 = (g & 1) ? NT : NT / 2;
#pragma unroll
                for (int t = t0; t < t1; ++t) {
                    const vec8 av = part == 1 ? al[t] : ah[t];
                    acc_re[t] = mfma(av, part == 2 ? bl[0] : bh[0], acc_re[t]);
                    acc_im[t] = mfma(av, part == 2 ? bl[1] : bh[1], acc_im[t]);
                }
            }
            // The producer piece is scheduled among this group's matrix
            // instructions: one MFMA, then up to five vector or scalar ALU
            // instructions, so the SIMD issues them while the MFMAs run
            // (forward 6 % faster; adjoint 2-4 % faster once its pieces no
            // longer read LDS, the conj(Ey) values being read at the start of
            // the step).
            prod(g);
#pragma unroll
            for (int q = 0; q < NT; ++q) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
                __builtin_amdgcn_sched_group_barrier(0x006, 5, 0);   // five VALU / SALU
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
};

template <>
__device__ __forceinline__ floatx16 PolSplit<__bf16, false>::mfma(vec8 a, vec8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ floatx16 PolSplit<_Float16, true>::mfma(vec8 a, vec8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

typedef PolSplit<__bf16, false> PolBF16;
typedef PolSplit<_Float16, true> PolF16;

// Power-of-two scale exponent that maps magnitudes <= m into [2^14, 2^15)
// (kept within FP32's normal range; m = 0 or non-finite gives a finite scale).
__device__ __forceinline__ int split_scale_exp(float m) {
    int e = 0;
    frexpf(m, &e);                       // m = f 2^e, f in [0.5, 1)
    const int s = 15 - e;
    return s > 126 ? 126 : s < -126 ? -126 : s;
}

// ---------------------------------------------------------------------------
// Pre-pass of the forward: I[b][g][y][x] = s_g[y][x] x_b[y][x], rows padded to
// a multiple of KC with zeros so the GEMM loads whole K-steps unguarded.
// ---------------------------------------------------------------------------
// Each thread takes four consecutive pixels of one padded row of one slice
// (the pitch is a multiple of 8, so a group never crosses a row), reads the
// image once and writes the group for every coil (two 16-byte writes each).
__global__ __launch_bounds__(256) void k_coil_weight(const NudftTable tab) {
    // Each item starts on a block boundary, so the item (and every field read
    // from it) is uniform over the block.
    int64_t blk = blockIdx.x;
    int k = 0;
    int64_t n = 0;
    for (; k < tab.nitems; ++k) {
        const NudftItem& c = tab.it[k];
        n = (int64_t)c.nb * c.ny * (ceil_div(c.nx, KC) * KC / 4);
        const int64_t nblk = ceil_div(n, 256);
        if (blk < nblk) break;
        blk -= nblk;
    }
    if (k >= tab.nitems) return;
    const int64_t gq = blk * 256 + threadIdx.x;   // index of a 4-pixel group within the item
    if (gq >= n) return;
    const NudftItem& it = tab.it[k];
    const int rowlen = (int)ceil_div(it.nx, KC) * KC;
    const int gpr = rowlen / 4;                           // groups per padded row
    const int i = (int)gq;
    const int b = i / (gpr * it.ny);
    const int rem = i - b * gpr * it.ny;
    const int y = rem / gpr, x0 = (rem - y * gpr) * 4;
    const int64_t npix = (int64_t)it.nx * it.ny;
    const float2* im = it.img + b * npix + (int64_t)y * it.nx;
    const float2* sm = it.smaps + b * it.smaps_bs + (int64_t)y * it.nx;
    // Four pixels as two 16-byte loads where the group lies inside the row and
    // both arrays are 16-byte aligned there (every coil's map then is too,
    // since a map has an even pixel count); one by one otherwise.
    const bool wide = x0 + 3 < it.nx && (npix & 1) == 0 &&
                      ((reinterpret_cast<uintptr_t>(im + x0) | reinterpret_cast<uintptr_t>(sm + x0)) & 15) == 0;
    auto load4 = [&](const float2* p, float2 (&v)[4]) {
        if (wide) {
            const float4 lo = *reinterpret_cast<const float4*>(p + x0);
            const float4 hi = *reinterpret_cast<const float4*>(p + x0 + 2);
            v[0] = make_float2(lo.x, lo.y);
            v[1] = make_float2(lo.z, lo.w);
            v[2] = make_float2(hi.x, hi.y);
            v[3] = make_float2(hi.z, hi.w);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = x0 + j < it.nx ? p[x0 + j] : make_float2(0.f, 0.f);
        }
    };
    float2 xv[4];
    load4(im, xv);
    // The activity flag is read after the image loads are issued (the image
    // of an inactive slice is still a valid buffer), so the two loads overlap.
    if (it.active && it.active[(int64_t)b * it.active_stride] == 0) return;
    float2* dst = it.wimg + ((int64_t)b * it.nc * it.ny + y) * rowlen + x0;
    const int64_t coil_stride = (int64_t)it.ny * rowlen;
#pragma unroll 4
    for (int g = 0; g < it.nc; ++g) {
        float2 sv[4], v[4];
        load4(sm + g * npix, sv);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = cmul(sv[j], xv[j]);   // zero past nx: xv is zero there
        float4* d4 = reinterpret_cast<float4*>(dst + g * coil_stride);
        d4[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
        d4[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
    }
}

// Split-BF16 form of the pre-pass: s_g (.) x_b is split and packed once per
// call into the forward's A-operand chunks, in LDS order, so every sample
// tile of the forward only copies 16-byte chunks.  Layout per (slice, coil):
// [K-step s][chunk (h, m)][row y < yp][16 B], rows past ny are zero.
__global__ __launch_bounds__(256) void k_coil_weight_bf16(const NudftTable tab) {
    // Each item starts on a block boundary (item uniform over the block).
    int64_t blk = blockIdx.x;
    int k = 0;
    int64_t u = 0;
    for (; k < tab.nitems; ++k) {
        const NudftItem& c = tab.it[k];
        u = fwd_split_units(c.nx, c.ny, c.nc, c.nb);
        const int64_t nblk = ceil_div(u, 256);
        if (blk < nblk) break;
        blk -= nblk;
    }
    if (k >= tab.nitems) return;
    const int64_t gu = blk * 256 + threadIdx.x;   // one (slice, coil, step, row) unit of the item
    if (gu >= u) return;
    const NudftItem& it = tab.it[k];
    const int yp = fwd_padded_rows(it.ny);
    const int nsteps = (int)ceil_div(it.nx, KC);
    const int i = (int)gu;
    const int y = i % yp;
    const int r1 = i / yp;
    const int s = r1 % nsteps;
    const int bg = r1 / nsteps;
    const int g = bg % it.nc, b = bg / it.nc;
    if (it.active && it.active[(int64_t)b * it.active_stride] == 0) return;
    float2 v[KC];
    const int64_t npix = (int64_t)it.nx * it.ny;
    const float2* sm = it.smaps + b * it.smaps_bs + g * npix + (int64_t)y * it.nx;
    const float2* im = it.img + b * npix + (int64_t)y * it.nx;
#pragma unroll
    for (int j = 0; j < KC; ++j) {
        const int x = s * KC + j;
        v[j] = (y < it.ny && x < it.nx) ? cmul(sm[x], im[x]) : make_float2(0.f, 0.f);
    }
    // Chunk planes of a K-step are yp rows long here (kRows in LDS).
    char* base = reinterpret_cast<char*>(it.wimg) + (((int64_t)bg * nsteps + s) * PolBF16::kChunks * yp) * 16;
    PolBF16::store_a_rows(base, y, yp, v);
}

// Split-FP16 form of the pre-pass: one wave per (slice, coil, padded row).
// The wave first finds the row's largest real or imaginary magnitude, scales
// the row by the power of two that puts it in [2^14, 2^15), then splits and
// packs it as k_coil_weight_bf16 does.  The inverse scale of each row is kept
// after the operand chunks (fwd_rowscale) for the forward's epilogue.
__global__ __launch_bounds__(256) void k_coil_weight_f16(const NudftTable tab) {
    const int lane = threadIdx.x & 63;
    // Each item starts on a block boundary (item uniform over the block).
    int64_t blk = blockIdx.x;
    int k = 0;
    int64_t u = 0;
    for (; k < tab.nitems; ++k) {
        const NudftItem& c = tab.it[k];
        u = (int64_t)c.nb * c.nc * fwd_padded_rows(c.ny);
        const int64_t nblk = ceil_div(u, 4);
        if (blk < nblk) break;
        blk -= nblk;
    }
    if (k >= tab.nitems) return;
    const int64_t gr = blk * 4 + (threadIdx.x >> 6);   // one (slice, coil, row) unit of the item
    if (gr >= u) return;
    const NudftItem& it = tab.it[k];
    const int yp = fwd_padded_rows(it.ny);
    const int nsteps = (int)ceil_div(it.nx, KC);
    const int i = (int)gr;
    const int y = i % yp;
    const int bg = i / yp;
    const int g = bg % it.nc, b = bg / it.nc;
    if (it.active && it.active[(int64_t)b * it.active_stride] == 0) return;
    const int64_t npix = (int64_t)it.nx * it.ny;
    const int yc = y < it.ny ? y : 0;
    const float2* sm = it.smaps + b * it.smaps_bs + g * npix + (int64_t)yc * it.nx;
    const float2* im = it.img + b * npix + (int64_t)yc * it.nx;
    auto row_step = [&](int s, float2 (&v)[KC]) {
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const int x = s * KC + j;
            v[j] = (y < it.ny && x < it.nx) ? cmul(sm[x], im[x]) : make_float2(0.f, 0.f);
        }
    };
    float m = 0.f;
    for (int s = lane; s < nsteps; s += 64) {
        float2 v[KC];
        row_step(s, v);
#pragma unroll
        for (int j = 0; j < KC; ++j) m = fmaxf(m, fmaxf(fabsf(v[j].x), fabsf(v[j].y)));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    const int se = split_scale_exp(m);
    const float sc = ldexpf(1.0f, se);
    char* wbase = reinterpret_cast<char*>(it.wimg);
    for (int s = lane; s < nsteps; s += 64) {
        float2 v[KC];
        row_step(s, v);
#pragma unroll
        for (int j = 0; j < KC; ++j) v[j] = cscale(v[j], sc);
        PolF16::store_a_rows(wbase + (((int64_t)bg * nsteps + s) * PolF16::kChunks * yp) * 16, y, yp, v);
    }
    if (lane == 0) fwd_rowscale(it.wimg, it.nx, it.ny, it.nc, it.nb)[(int64_t)bg * yp + y] = ldexpf(1.0f, -se);
}

// Split-FP16 adjoint: scale exponent of each (slice, coil, sample split),
// from the largest |Re d| + |Im d| (>= |Re W|, |Im W| for W = d conj(Ey)) of
// the split's samples; one block per unit.
__global__ __launch_bounds__(256) void k_adj_scale(const NudftTable tab) {
    __shared__ float wmax[4];
    int64_t u = blockIdx.x;
    int k = 0;
    for (; k < tab.nitems; ++k) {
        const NudftItem& c = tab.it[k];
        const int64_t n = (int64_t)c.nb * c.nc * c.ksplit;
        if (u < n) break;
        u -= n;
    }
    if (k >= tab.nitems) return;
    const NudftItem& it = tab.it[k];
    const int sp = (int)(u % it.ksplit);
    const int64_t bg = u / it.ksplit;
    const int b = (int)(bg / it.nc);
    if (it.active && it.active[(int64_t)b * it.active_stride] == 0) return;
    const int64_t kbeg = (int64_t)sp * it.kper;
    const int64_t kend = min(it.nk, kbeg + it.kper);
    const float2* d = it.data + bg * it.nk;
    float m = 0.f;
    for (int64_t kk = kbeg + threadIdx.x; kk < kend; kk += 256) {
        const float2 v = d[kk];
        m = fmaxf(m, fabsf(v.x) + fabsf(v.y));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
        adj_scale_exp(it.part, it.nx, it.ny, it.nc, it.nb, it.ksplit)[bg * it.ksplit + sp] = split_scale_exp(m);
    }
}

// Adjoint phase tables: exp(+i 2 pi f r) for every sample and every centred x
// (then y) offset, with the reduction of phase.h, i.e. the values the adjoint
// would otherwise form per step; one thread per table element.  Filled once
// per trajectory (once per solve).
__global__ __launch_bounds__(256) void k_adj_phases(const NudftTable tab, int64_t total) {
    // Grid-stride: any table size is covered by a bounded grid.
    for (int64_t g0 = (int64_t)blockIdx.x * 256 + threadIdx.x; g0 < total; g0 += (int64_t)gridDim.x * 256) {
        int64_t g = g0;
        int k = 0;
        for (; k < tab.nitems; ++k) {
            const NudftItem& c = tab.it[k];
            const int64_t n = adj_table_elems(c.nx, c.ny, c.nk, c.traj_bs ? c.nb : 1);
            if (g < n) break;
            g -= n;
        }
        if (k >= tab.nitems) return;
        const NudftItem& it = tab.it[k];
        const int64_t nx = it.nx, ny = it.ny;
        const int64_t per = it.nk * (nx + ny);            // elements per trajectory
        const int64_t bt = g / per;
        int64_t r = g - bt * per;
        const double* traj = it.traj + bt * it.traj_bs;
        if (r < it.nk * nx) {
            const int64_t kk = r / nx;
            const int x = (int)(r - kk * nx);
            it.ephx[bt * it.ephx_bs + r] = phase_pos(traj[2 * kk] * kQuarterTurnsPerRad, (double)(x - it.nx / 2));
        } else {
            r -= it.nk * nx;
            const int64_t kk = r / ny;
            const int y = (int)(r - kk * ny);
            it.ephy[bt * it.ephy_bs + r] =
                phase_pos(traj[2 * kk + 1] * kQuarterTurnsPerRad, (double)(y - it.ny / 2));
        }
    }
}

// ---------------------------------------------------------------------------
// Forward: tile = (slice, coil, 64 samples); rows = every y in passes of 256.
// In the split forms the next B stage is produced between the MFMA groups of
// the current one (mma_with); in FP32 it follows them.
// ---------------------------------------------------------------------------
template <class P, int NT>
__global__ __launch_bounds__(kThreads, 2) void nudft_fwd(const NudftTable tab) {
    __shared__ __attribute__((aligned(16))) char smem[2 * (P::kABytes + P::kBBytes)];
    __shared__ float2 red[2][kFwdCols];
    char* const sA0 = smem;
    char* const sB0 = smem + 2 * P::kABytes;

    const int tile = xcd_remap(blockIdx.x, tab.total_tiles);
    const NudftItem& it = tab.it[find_item(tab, tile)];
    const int nx = it.nx, ny = it.ny, nc = it.nc;
    const int64_t nk = it.nk;
    int local = tile - it.tile_begin;
    const int nkb = (int)ceil_div(nk, kFwdCols);
    const int kb = local % nkb;
    local /= nkb;
    const int g = local % nc;
    const int b = local / nc;
    if (it.active && it.active[(int64_t)b * it.active_stride] == 0) return;

    const int tid = threadIdx.x, lane = tid & 63;
    // Derived through readfirstlane so the compiler knows it is uniform: the
    // LDS destinations of the A stage's direct loads are then scalar
    // registers, with no per-step readfirstlane (forward 1-2 % faster).
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave & 1, wn = wave >> 1, h = lane >> 5, l32 = lane & 31;
    const int64_t k0 = (int64_t)kb * kFwdCols;
    const int pitch = (int)ceil_div(nx, KC) * KC;
    const double* traj = it.traj + b * it.traj_bs;
    const float2* wi = it.wimg + ((int64_t)b * nc + g) * ny * pitch;
    const int xh = nx / 2, yh = ny / 2;

    // B producer: sample column pc, K pair pj.  Ex[k][x0+j] = base(x0) * w_j.
    const int pc = tid & 63, pj = (tid >> 6) * 2;
    const bool p_ok = k0 + pc < nk;
    const double fx4 = p_ok ? traj[2 * (k0 + pc)] * kQuarterTurnsPerRad : 0.0;
    // (w0, w1 carry the B scale of the split forms: exact, a power of two)
    const float2 w0 = cscale(phase_neg(fx4, (double)pj), P::kBScale);
    const float2 w1 = cscale(phase_neg(fx4, (double)(pj + 1)), P::kBScale);
    const float2 wk = phase_neg(fx4, (double)KC);      // one K-step
    // Epilogue: this lane's sample column.
    const int64_t ke = k0 + wn * 32 + l32;
    const bool e_ok = ke < nk;
    const double fy4 = e_ok ? traj[2 * ke + 1] * kQuarterTurnsPerRad : 0.0;

    const int nsteps = pitch / KC;
    float2 dsum = make_float2(0.f, 0.f);

    // Rows are covered in passes of 2 * NT * 32; the host picks NT per shape so
    // the passes are even (e.g. 384 rows = 2 passes of 192, NT = 3).
    constexpr int nt = NT;
    constexpr int prows = 2 * NT * 32;
    for (int y0 = 0; y0 < ny; y0 += prows) {
        const int wrow0 = y0 + wm * (nt * 32);
        const int nvalid = wrow0 >= ny ? 0 : min(nt, (ny - wrow0 + 31) / 32);
        const int yrow = y0 + tid;
        const bool row_ok = yrow < ny && tid < prows;
        // FP32: rows past ny load row ny-1 (always in bounds) and are zeroed when
        // staged.  Split-BF16: the pre-pass already holds zero rows up to yp.
        const float4* src = reinterpret_cast<const float4*>(wi + (int64_t)min(yrow, ny - 1) * pitch);
        const float rmask = row_ok ? 1.0f : 0.0f;
        const int yp = fwd_padded_rows(ny);
        const char* wsplit = reinterpret_cast<const char*>(it.wimg) +
                             ((int64_t)(b * nc + g) * nsteps * kSplitUnitBytes / 16 * yp + (int64_t)min(yrow, yp - 1)) * 16;
        float4 pre[KC / 2];

        // FP32: global -> registers (prefetched one step ahead) -> LDS planes.
        // Split-BF16: the pre-split chunks go global -> LDS directly
        // (global_load_lds_dwordx4: lane i of a wave lands at base + 16 i, and the
        // LDS chunk planes hold consecutive rows), issued one step ahead.
        auto load_a_to = [&](int s, int st) {
            if constexpr (P::kPresplitA) {
                char* dst = sA0 + st * P::kABytes + wave * 64 * 16;   // wave-uniform
                const char* g = wsplit + (int64_t)s * P::kChunks * yp * 16;
#pragma unroll
                for (int c = 0; c < P::kChunks; ++c)
                    __builtin_amdgcn_global_load_lds(g + (int64_t)c * yp * 16, dst + c * kRows * 16, 16, 0, 0);
            }
        };
        auto load_a = [&](int s) {
            if constexpr (P::kPresplitA) {
                const int st = s & 1;
                char* dst = sA0 + st * P::kABytes + wave * 64 * 16;   // wave-uniform
                const char* g = wsplit + (int64_t)s * P::kChunks * yp * 16;
#pragma unroll
                for (int c = 0; c < P::kChunks; ++c)
                    __builtin_amdgcn_global_load_lds(g + (int64_t)c * yp * 16, dst + c * kRows * 16, 16, 0, 0);
            } else {
#pragma unroll
                for (int j = 0; j < KC / 2; ++j) pre[j] = src[s * (KC / 2) + j];
            }
        };
        auto store_a = [&](int st) {
            if constexpr (!P::kPresplitA) {
                float2 v[KC];
#pragma unroll
                for (int j = 0; j < KC / 2; ++j) {
                    v[2 * j] = make_float2(pre[j].x * rmask, pre[j].y * rmask);
                    v[2 * j + 1] = make_float2(pre[j].z * rmask, pre[j].w * rmask);
                }
                P::store_a(sA0 + st * P::kABytes, tid, v);
            }
        };
        // LDS writes by global_load_lds complete with the vector-memory counter.
        auto wait_a = [&]() {
            if constexpr (P::kPresplitA) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        };
        // B stage s: Ex[k][s KC + pj + j] = xb(s) w_j with the step base
        // xb(s) = Ex(s KC - nx/2).  Steps are staged in order within a pass, so
        // xb advances by one factor E(KC) per step and is regenerated with the
        // FP64 reduction every kXAnchor steps (at most kXAnchor - 1 roundings
        // of drift).  Samples past nk (fx4 = 0) stage unit phases; their
        // outputs are never stored.
        float2 xb = make_float2(1.f, 0.f);
        auto store_b = [&](int st, int s) {
            if (s % kXAnchor == 0) xb = phase_neg(fx4, (double)(s * KC - xh));
            else xb = cmul(xb, wk);
            P::store_b(sB0 + st * P::kBBytes, pc, pj, cmul(xb, w0), cmul(xb, w1));
        };

        floatx16 acc_re[NT], acc_im[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc_re[t] = floatx16{0};
            acc_im[t] = floatx16{0};
        }
        load_a(0);
        store_a(0);
        store_b(0, 0);
        wait_a();
        __syncthreads();
        if constexpr (P::kPresplitA) {
            // Split forms: the next stage's B phases are produced in six pieces
            // between the MFMA groups of this stage, branch-free (lanes past
            // the last sample store zeros; the last step produces its own
            // stage again into the idle buffer, where nothing reads it).  As
            // in FP32, the step base advances by one factor E(KC) per step and
            // is regenerated with the FP64 reduction every kXAnchor steps: the
            // steps run in unrolled blocks of kXAnchor, so whether a step
            // regenerates is known at compile time and the loop stays one
            // basic block; steps past the last whole block regenerate always.
            auto split_step = [&](int s, bool exact) {
                const int cur = s & 1;
                const int sn = s + 1 < nsteps ? s + 1 : s;
                QuarterTurn qt;
                SinCos sc;
                float2 e0, e1;
                typename P::BWords r0, r1;
                auto prod = [&](int piece) {
                    if (piece == 0) {
                        // The next A stage's copies start here, after this
                        // stage's operand reads: issued before them, they would
                        // make those reads wait for the copies to land.
                        load_a_to(sn, cur ^ 1);
                        if (exact) qt = reduce_quarter_turns(fx4 * (double)(sn * KC - xh));
                        else xb = cmul(xb, wk);
                    } else if (piece == 1) {
                        if (exact) sc = sincos_octant(qt.th);
                    } else if (piece == 2) {
                        if (exact) {
                            const SinCos r = rotate_quadrant(sc, qt.q);
                            xb = make_float2(r.c, -r.s);
                        }
                        e0 = cmul(xb, w0);
                        e1 = cmul(xb, w1);
                    } else if (piece == 3) {
                        // No sample mask: a column past nk has finite phases
                        // (frequency 0) and its output is never stored.
                        r0 = P::split_b4(e0);
                    } else if (piece == 4) {
                        r1 = P::split_b4(e1);
                    } else {
                        P::template store_b_words4<64>(sB0 + (cur ^ 1) * P::kBBytes, pc, pj, r0, r1);
                    }
                };
                P::template mma_with<NT, 64, false>(sA0 + cur * P::kABytes, sB0 + cur * P::kBBytes, wm * (nt * 32),
                                                    wn * 32, lane, acc_re, acc_im, prod);
                wait_a();
                __syncthreads();
            };
            int s = 0;
            for (; s + kXAnchor <= nsteps; s += kXAnchor) {
#pragma unroll
                for (int u = 0; u < kXAnchor; ++u) split_step(s + u, u == kXAnchor - 1);
            }
            for (; s < nsteps; ++s) split_step(s, true);
        } else {
            for (int s = 0; s < nsteps; ++s) {
                const int cur = s & 1;
                const bool more = s + 1 < nsteps;
                if (more) load_a(s + 1);
                P::template mma<NT>(sA0 + cur * P::kABytes, sB0 + cur * P::kBBytes, wm * (nt * 32), wn * 32, lane,
                                    nvalid, acc_re, acc_im);
                if (more) {
                    store_a(cur ^ 1);
                    store_b(cur ^ 1, s + 1);
                }
                wait_a();
                __syncthreads();
            }
        }

        // Epilogue: sum_y T[y][k] Ey[k][y] over this pass's rows.  Rows of a
        // lane are ybase + 32 t + 8 q + r (r < 4) and the phase factors as
        // Ey(ybase) E(32 t) E(8 q) E(r); Ey(ybase), E(1), E(8) and E(32) are
        // generated with the FP64 argument reduction and the other powers are
        // their products (a few FP32 roundings each).  The sum is taken in
        // Horner form, innermost over r:
        //   Ey(ybase) sum_t E(32 t) sum_q E(8 q) sum_r E(r) T[ybase + 32 t + 8 q + r].
        // Rows past ny within a live tile hold zero accumulators (their A rows
        // are zero), so no row test is needed.
        // Split-FP16: the phase scale and each row's pre-pass scale are undone
        // first, one after the other (each factor a normal power of two).
        constexpr float kInvB = 1.0f / P::kBScale;
        float2 part = make_float2(0.f, 0.f);
        if (e_ok && nvalid > 0) {
            const float* rsc = nullptr;
            if constexpr (P::kScaled)
                rsc = fwd_rowscale(it.wimg, nx, ny, nc, it.nb) + (int64_t)(b * nc + g) * fwd_padded_rows(ny) +
                      wrow0 + h * 4;
            const int ybase = wrow0 + h * 4 - yh;
            const float2 e0 = phase_neg(fy4, (double)ybase);
            float2 f1[4], f8[4], f32[NT];
            f1[1] = phase_neg(fy4, 1.0);
            f8[1] = phase_neg(fy4, 8.0);
#pragma unroll
            for (int j = 2; j < 4; ++j) {
                f1[j] = cmul(f1[j - 1], f1[1]);
                f8[j] = cmul(f8[j - 1], f8[1]);
            }
            if constexpr (NT > 1) f32[1] = phase_neg(fy4, 32.0);
#pragma unroll
            for (int j = 2; j < NT; ++j) f32[j] = cmul(f32[j - 1], f32[1]);
            float2 st = make_float2(0.f, 0.f);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (t < nvalid) {
                    float2 sq = make_float2(0.f, 0.f);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float4 rs4 = make_float4(1.f, 1.f, 1.f, 1.f);
                        if constexpr (P::kScaled) rs4 = *reinterpret_cast<const float4*>(rsc + t * 32 + q * 8);
                        const float rs[4] = {rs4.x, rs4.y, rs4.z, rs4.w};
                        float2 sr = make_float2(acc_re[t][q * 4] * kInvB * rs[0], acc_im[t][q * 4] * kInvB * rs[0]);
#pragma unroll
                        for (int r = 1; r < 4; ++r)
                            sr = cfma(f1[r], make_float2(acc_re[t][q * 4 + r] * kInvB * rs[r],
                                                         acc_im[t][q * 4 + r] * kInvB * rs[r]), sr);
                        sq = q == 0 ? sr : cfma(f8[q], sr, sq);
                    }
                    st = t == 0 ? sq : cfma(f32[t], sq, st);
                }
            }
            part = cmul(e0, st);
        }
        part.x += __shfl_xor(part.x, 32, 64);
        part.y += __shfl_xor(part.y, 32, 64);
        if (h == 0) red[wm][wn * 32 + l32] = part;
        __syncthreads();
        if (tid < kFwdCols) dsum = cadd(dsum, cadd(red[0][tid], red[1][tid]));
        __syncthreads();
    }
    if (tid < kFwdCols && k0 + tid < nk) it.data[((int64_t)b * nc + g) * nk + k0 + tid] = dsum;
}

// ---------------------------------------------------------------------------
// Adjoint: tile = (slice, sample split, coil group, 32 y rows, 128 x
// columns), 8 waves (2 row x 4 column waves, one workgroup per CU).  GEMM rows
// are (coil, y) for the tile's group of 2 NT coils: A = W = d conj(Ey), B =
// conj(Ex), K = samples of the split; the epilogue forms sum_g conj(s_g) X_g
// and writes the (split, group) partial image for the fixed-order reduction.  The 128-column tile
// lets every W value feed twice the MFMAs of a 64-column one, halving the
// vector work of W per matrix instruction.  Each thread forms half a W row
// (4 K values) and stages two conj(Ex) values and one conj(Ey) value per step
// from the phase tables (waves 4-7 stage the same conj(Ey) values as waves
// 0-3 into the tile's padding column, so every wave does the same work and
// the loop has no role branch).  In the split forms, steps whose look-ahead
// loads are whole steps run with the producers interleaved between the MFMA
// groups and the split's last steps take a plain loop; FP32 takes the plain
// loop throughout (its matrix instructions do not run alongside vector work).
// ---------------------------------------------------------------------------
template <class P, int NT>
__global__ __launch_bounds__(kThreads8, 1) void nudft_adj8(const NudftTable tab) {
    constexpr int BC = kAdjCols8;
    constexpr int kBBytes8 = P::template bbytes<BC>();
    __shared__ __attribute__((aligned(16))) char smem[2 * (P::kABytes + kBBytes8)];
    __shared__ __attribute__((aligned(16))) float2 sE[2][kAdjRows][KC + 2];   // conj(Ey); column KC takes duplicates
    __shared__ float sUnscale[2 * kNT];
    char* const sA0 = smem;
    char* const sB0 = smem + 2 * P::kABytes;

    const int tile = xcd_remap(blockIdx.x, tab.total_tiles);
    const NudftItem& it = tab.it[find_item(tab, tile)];
    const int nx = it.nx, ny = it.ny, nc = it.nc;
    const int64_t nk = it.nk;
    // y blocks fastest, then x blocks, then coil groups, then sample splits
    constexpr int gsz = 2 * NT;
    const int ncgroups = (nc + gsz - 1) / gsz;
    int local = tile - it.tile_begin;
    const int nxb = (nx + BC - 1) / BC, nyb = (ny + kAdjRows - 1) / kAdjRows;
    const int yb = local % nyb;
    local /= nyb;
    const int xb = local % nxb;
    local /= nxb;
    const int gi = local % ncgroups;
    local /= ncgroups;
    const int sp = local % it.ksplit;
    const int b = local / it.ksplit;
    if (it.active && it.active[(int64_t)b * it.active_stride] == 0) return;

    const int tid = threadIdx.x, lane = tid & 63;
    // Known uniform in FP32 (adjoint 0.5-1 % faster); the split forms keep
    // the vector form, which their interleaved loop schedules better.
    const int wave = P::kPresplitA ? tid >> 6 : __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave & 1, wn = wave >> 1, h = lane >> 5, l32 = lane & 31;
    const int x0 = xb * BC, y0 = yb * kAdjRows;
    const int64_t npix = (int64_t)nx * ny;
    const float2* sm = it.smaps + b * it.smaps_bs;
    const float2* dat = it.data + (int64_t)b * nc * nk;
    const int64_t kbeg = (int64_t)sp * it.kper;
    const int64_t kend = min(nk, kbeg + it.kper);
    const int nsteps = (int)ceil_div(kend - kbeg, KC);
    const int klast = (int)(kend - kbeg - 1);             // last sample of the split, relative
    // Phase rows of the split's samples (tables filled by k_adj_phases).
    const float2* phx = it.ephx + b * it.ephx_bs + kbeg * nx;
    const float2* phy = it.ephy + b * it.ephy_bs + kbeg * ny;
    const int32_t* aexp = nullptr;
    if constexpr (P::kScaled) aexp = adj_scale_exp(it.part, nx, ny, nc, it.nb, it.ksplit);

    // Producer roles.
    const int ey = tid & 31, ek = (tid >> 5) & 7;        // E: (y, k); waves 4-7 duplicate 0-3
    const int ecol = tid < 256 ? ek : KC;                // where this thread's E value goes
    const int bx = tid & 127, bk = (tid >> 7) * 2;       // B: (x, k pair)
    const int arow = tid & 255, ahalf = tid >> 8;        // A: row (coil, y), K half
    const int ac = arow >> 5, ay = arow & 31;
    const bool ey_ok = y0 + ey < ny;
    const bool bx_ok = x0 + bx < nx;
    const int yc = ey_ok ? y0 + ey : ny - 1;             // in-bounds table columns
    const int xc = bx_ok ? x0 + bx : nx - 1;
    const int xe = x0 + wn * 32 + l32;                   // epilogue column

    constexpr int nt = NT;
    {
        const int g0 = gi * gsz;                         // this workgroup's coil group
        const int ncg = min(gsz, nc - g0);
        const int kl = klast;
        const int nvalid = max(0, min(nt, ncg - wm * nt));
        // Rows of coils past the group's end read coil g0 and feed only
        // accumulator tiles that the epilogue never reads.
        const bool a_ok = ac < ncg;
        const float2* drow = dat + (int64_t)(g0 + (a_ok ? ac : 0)) * nk + kbeg;
        float2 dreg[4];

        float ascale = 1.0f;
        if constexpr (P::kScaled) {
            const int se = a_ok ? aexp[((int64_t)b * nc + g0 + ac) * it.ksplit + sp] : 0;
            ascale = ldexpf(1.0f, se);
            if (ay == 0 && ahalf == 0 && ac < gsz) sUnscale[ac] = ldexpf(1.0f, -se);
        }

        // d of this thread's 4 K values of step s (clamped to the split's
        // last sample in the last step; those samples meet a zero E).
        auto load_d = [&](int s) {
            if (s * KC + KC - 1 <= kl) {
                const float2* p = drow + s * KC + 4 * ahalf;
#pragma unroll
                for (int j = 0; j < 4; ++j) dreg[j] = p[j];
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) dreg[j] = drow[min(s * KC + 4 * ahalf + j, kl)];
            }
        };
        // Phases prefetched one step ahead (rows clamped to the split's last
        // sample; those samples are masked when staged).  Masks multiply (the
        // phases are finite), which keeps the loops free of branches.
        float2 fx0, fx1, fy;
        auto load_fx = [&](int s) {
            const int k = s * KC + bk;
            fx0 = phx[(int64_t)min(k, kl) * nx + xc];
            fx1 = phx[(int64_t)min(k + 1, kl) * nx + xc];
        };
        auto load_fy = [&](int s) { fy = phy[(int64_t)min(s * KC + ek, kl) * ny + yc]; };
        auto gen_e = [&](int st, int s) {
            const float m = (ey_ok && s * KC + ek <= kl) ? 1.f : 0.f;
            sE[st][ey][ecol] = make_float2(fy.x * m, fy.y * m);
        };
        auto gen_b = [&](int st, int s) {
            const int k = s * KC + bk;
            const float m0 = (bx_ok && k <= kl) ? P::kBScale : 0.f;     // mask and B scale
            const float m1 = (bx_ok && k + 1 <= kl) ? P::kBScale : 0.f;
            P::template store_b<BC>(sB0 + st * kBBytes8, bx, bk, make_float2(fx0.x * m0, fx0.y * m0),
                                    make_float2(fx1.x * m1, fx1.y * m1));
        };
        // W of this thread's row and K half: d conj(Ey) (with the coil's scale).
        auto gen_a = [&](int st, int est) {
            float2 w[4];
#pragma unroll
            for (int j = 0; j < 4; j += 2) {
                const float4 e2 = *reinterpret_cast<const float4*>(&sE[est][ay][4 * ahalf + j]);
                w[j] = cmul(dreg[j], make_float2(e2.x, e2.y));
                w[j + 1] = cmul(dreg[j + 1], make_float2(e2.z, e2.w));
                if constexpr (P::kScaled) {
                    w[j] = cscale(w[j], ascale);
                    w[j + 1] = cscale(w[j + 1], ascale);
                }
            }
            P::store_a_half(sA0 + st * P::kABytes, ac * 32 + ay, kRows, ahalf, w);
        };

        floatx16 acc_re[NT], acc_im[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            acc_re[t] = floatx16{0};
            acc_im[t] = floatx16{0};
        }
        // Prologue: E(0), d(0) -> A(0), B(0); E(1), d(1) and the next
        // phase values ready for the loop.
        load_fy(0);
        gen_e(0, 0);
        load_d(0);
        load_fx(0);
        __syncthreads();
        gen_a(0, 0);
        gen_b(0, 0);
        load_fx(1);
        if (nsteps > 1) {
            load_fy(1);
            gen_e(1, 1);
            load_d(1);
        }
        load_fy(2);
        __syncthreads();
        int s = 0;
        // Steady state of the split forms: every look-ahead load is a whole
        // step, no branch, producers interleaved.  (FP32 matrix instructions
        // do not run alongside vector work, so FP32 takes the plain loop.)
        // No masks here: every sample these steps stage lies inside the split
        // (B up to the third-last step, conj(Ey) up to the second-last, both
        // whole since every step but the last is), and a B column past nx
        // or a W row past ny, built from the clamped table entries (finite
        // phases), feeds only its own output column or row, which the
        // epilogue never stores.
        if constexpr (P::kPresplitA)
        for (; s < nsteps - 3; ++s) {
            const int cur = s & 1;
            float2 w[4];
            typename P::Words r0;
            // conj(Ey)(s+1) of this thread's W row, complete since the last
            // barrier: read before this step's products so that the
            // producer pieces do not wait for LDS.
            float2 ereg[4];
            {
                const float4 e01 = *reinterpret_cast<const float4*>(&sE[cur ^ 1][ay][4 * ahalf]);
                const float4 e23 = *reinterpret_cast<const float4*>(&sE[cur ^ 1][ay][4 * ahalf + 2]);
                ereg[0] = make_float2(e01.x, e01.y);
                ereg[1] = make_float2(e01.z, e01.w);
                ereg[2] = make_float2(e23.x, e23.y);
                ereg[3] = make_float2(e23.z, e23.w);
            }
            auto prod = [&](int piece) {
                if (piece == 0) {                 // W(s+1), first two values
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        w[j] = cmul(dreg[j], ereg[j]);
                        if constexpr (P::kScaled) w[j] = cscale(w[j], ascale);
                    }
                } else if (piece == 1) {          // W(s+1), last two values; store; d(s+2)
#pragma unroll
                    for (int j = 2; j < 4; ++j) {
                        w[j] = cmul(dreg[j], ereg[j]);
                        if constexpr (P::kScaled) w[j] = cscale(w[j], ascale);
                    }
                    P::store_a_half(sA0 + (cur ^ 1) * P::kABytes, ac * 32 + ay, kRows, ahalf, w);
                    const float2* q = drow + (s + 2) * KC + 4 * ahalf;
#pragma unroll
                    for (int j = 0; j < 4; ++j) dreg[j] = q[j];
                } else if (piece == 2) {          // conj(Ex) of step s+1: first value
                    r0 = P::split_b(cscale(fx0, P::kBScale));
                } else if (piece == 3) {          // second value; store B(s+1); next phases
                    P::template store_b_words<BC>(sB0 + (cur ^ 1) * kBBytes8, bx, bk, r0,
                                                  P::split_b(cscale(fx1, P::kBScale)));
                    const float2* q = phx + (int64_t)((s + 2) * KC + bk) * nx + xc;
                    fx0 = q[0];
                    fx1 = q[nx];
                } else if (piece == 4) {          // conj(Ey) of step s+2; fy(s+3)
                    sE[cur][ey][ecol] = fy;
                    load_fy(s + 3);
                }
            };
            P::template mma_with<NT, BC, true>(sA0 + cur * P::kABytes, sB0 + cur * kBBytes8, wm * (nt * 32),
                                               wn * 32, lane, acc_re, acc_im, prod);
            __syncthreads();
        }
        for (; s < nsteps; ++s) {
            const int cur = s & 1;
            P::template mma<NT, BC>(sA0 + cur * P::kABytes, sB0 + cur * kBBytes8, wm * (nt * 32), wn * 32, lane,
                                    nvalid, acc_re, acc_im);
            if (s + 1 < nsteps) {
                gen_a(cur ^ 1, cur ^ 1);              // W(s+1) from d(s+1) and E(s+1)
                if (s + 2 < nsteps) load_d(s + 2);
                gen_b(cur ^ 1, s + 1);                // uses fx(s+1)
                if (s + 2 < nsteps) gen_e(cur, s + 2);   // uses fy(s+2)
                load_fx(s + 2);
                load_fy(s + 3);
            }
            __syncthreads();
        }
        // Coil combine of this group, then the two row-waves of each x
        // quarter meet through LDS and the group's partial image is written.
        float2 part[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) part[i] = make_float2(0.f, 0.f);
        if (xe < nx) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if (t < nvalid) {
                    const int g = g0 + wm * nt + t;
                    const float2* sg = sm + (int64_t)g * npix;
                    constexpr float kInvB = 1.0f / P::kBScale;
                    float us = 1.0f;
                    if constexpr (P::kScaled) us = sUnscale[wm * nt + t];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int y = y0 + (i >> 2) * 8 + h * 4 + (i & 3);
                        if (y < ny)
                            part[i] = cadd(part[i], cmulc(sg[(int64_t)y * nx + xe],
                                                          make_float2(acc_re[t][i] * kInvB * us,
                                                                      acc_im[t][i] * kInvB * us)));
                    }
                }
            }
        }
        float2* red = reinterpret_cast<float2*>(smem);   // 4 (wn) x 16 x 64 complex
        if (wm == 1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) red[(wn * 16 + i) * 64 + lane] = part[i];
        }
        __syncthreads();
        if (wm == 0 && xe < nx) {
            const int plane = sp * ncgroups + gi;
            float2* out = it.part + ((int64_t)plane * it.nb + b) * npix;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int y = y0 + (i >> 2) * 8 + h * 4 + (i & 3);
                if (y < ny) out[(int64_t)y * nx + xe] = cadd(part[i], red[(wn * 16 + i) * 64 + lane]);
            }
        }
    }
}

}  // namespace

int64_t fwd_tiles(int nx, int ny, int nc, int64_t nk, int nb) {
    (void)nx; (void)ny;
    return (int64_t)nb * nc * ceil_div(nk, kFwdCols);
}

int64_t fwd_wimg_elems(int nx, int ny, int nc, int nb) {  // FP32 form, complex elements
    return (int64_t)nb * nc * ny * (ceil_div(nx, KC) * KC);
}

int64_t adj_tiles_per_split(int nx, int ny, int nb) {
    return (int64_t)nb * ceil_div(nx, kAdjCols) * ceil_div(ny, kAdjRows);
}

int64_t adj_tiles(int nx, int ny, int nc, int nb, int ksplit) {
    return adj_tiles_per_split(nx, ny, nb) * adj_coil_groups(nc) * ksplit;
}

void adj_split(int nx, int ny, int nc, int64_t nk, int nb, int precision,
               int32_t* ksplit, int32_t* kper) {
    // The split depends on the slice shape only (not on nb or on other
    // problems in a grouped launch), so every slice is summed in the same
    // order alone and in a batch: results are batch-invariant bit for bit.
    (void)precision; (void)nb;
    // Workgroups per sample range: 128 x 32 pixel tiles times coil groups.
    const int64_t per_split = adj_tiles_per_split(nx, ny, 1) * adj_coil_groups(nc);
    // At least 256 samples per range: short sample ranges (one GPU's share of
    // a k-space split, 4096 samples per coil at 256^2) then still fill the
    // GPU; 512 left half of it idle there (adjoint 9 % slower in FP32, 30 %
    // in the split forms), and 128 spends more on each workgroup's coil
    // combine and on the partial images than it gains.  At most 65536
    // samples per range, which bounds the length of the FP32 accumulations.
    const int64_t smax = std::max<int64_t>(1, nk / 256);
    const int64_t smin = std::min<int64_t>(smax, ceil_div(nk, 65536));
    // The fewest ranges whose workgroups fill whole rounds of the 256 CUs to
    // at least 90 % (one workgroup per CU): e.g. 16 ranges of 2048 samples at
    // 256^2 with 8 coils (256 workgroups), 5 at 384^2 with 32 coils (720
    // workgroups in three rounds, where 8 ranges, 288 workgroups, left the
    // second round almost empty and ran the adjoint at 56 % of the forward's
    // rate).  A problem too small to fill one round takes the most ranges;
    // one that never reaches 90 % takes the best-filled count.
    constexpr int64_t kCUs = 256;
    int64_t s = -1, best = smin;
    double best_fill = 0.0;
    for (int64_t c = smin; c <= smax && c <= 4 * kCUs; ++c) {
        const int64_t w = c * per_split, rounds = ceil_div(w, kCUs);
        const double fill = (double)w / (double)(rounds * kCUs);
        if (w >= kCUs && fill >= 0.9) {
            s = c;
            break;
        }
        if (fill > best_fill + 1e-9) {
            best_fill = fill;
            best = c;
        }
    }
    if (s < 0) s = smax * per_split < kCUs ? smax : best;
    int64_t per = ceil_div(ceil_div(nk, s), KC) * KC;
    s = ceil_div(nk, per);
    *ksplit = (int32_t)s;
    *kper = (int32_t)per;
}

hipError_t launch_coil_weight(const NudftTable& t, int precision, hipStream_t s) {
    if (t.cw_total <= 0) return hipSuccess;
    if (precision == MRI_BF16X3) {
        int64_t blocks = 0;
        for (int i = 0; i < t.nitems; ++i)
            blocks += ceil_div(fwd_split_units(t.it[i].nx, t.it[i].ny, t.it[i].nc, t.it[i].nb), 256);
        hipLaunchKernelGGL(k_coil_weight_bf16, dim3((unsigned)blocks), dim3(256), 0, s, t);
        return hipGetLastError();
    }
    if (precision == MRI_FP16X3) {
        int64_t blocks = 0;
        for (int i = 0; i < t.nitems; ++i) blocks += ceil_div(fwd_rowscale_floats(t.it[i].ny, t.it[i].nc, t.it[i].nb), 4);
        hipLaunchKernelGGL(k_coil_weight_f16, dim3((unsigned)blocks), dim3(256), 0, s, t);
        return hipGetLastError();
    }
    int64_t blocks = 0;
    for (int i = 0; i < t.nitems; ++i)
        blocks += ceil_div((int64_t)t.it[i].nb * t.it[i].ny * (ceil_div(t.it[i].nx, KC) * KC / 4), 256);
    hipLaunchKernelGGL(k_coil_weight, dim3((unsigned)blocks), dim3(256), 0, s, t);
    return hipGetLastError();
}

namespace {

// Launch one kernel variant per row-tile class: items are grouped by their NT
// (each class keeps its own contiguous tile numbering).
// tiles_of gives an item's tile count for the kernel being launched.
template <class Pick, class Tiles, class Launch>
hipError_t launch_by_nt(const NudftTable& t, Pick nt_of, Tiles tiles_of, Launch launch) {
    for (int nt = 2; nt <= kNT; ++nt) {
        NudftTable sub;
        sub.nitems = 0;
        sub.total_tiles = 0;
        sub.cw_total = 0;
        for (int i = 0; i < t.nitems; ++i) {
            if (nt_of(t.it[i]) != nt) continue;
            sub.it[sub.nitems] = t.it[i];
            sub.it[sub.nitems].tile_begin = sub.total_tiles;
            sub.it[sub.nitems].ntiles = (int32_t)tiles_of(t.it[i]);
            sub.total_tiles += sub.it[sub.nitems].ntiles;
            ++sub.nitems;
        }
        if (sub.total_tiles == 0) continue;
        const hipError_t e = launch(sub, nt);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class P>
hipError_t fwd_variant(const NudftTable& t, int nt, hipStream_t s) {
    const dim3 g(t.total_tiles), b(kThreads);
    if (nt == 2) hipLaunchKernelGGL((nudft_fwd<P, 2>), g, b, 0, s, t);
    else if (nt == 3) hipLaunchKernelGGL((nudft_fwd<P, 3>), g, b, 0, s, t);
    else hipLaunchKernelGGL((nudft_fwd<P, 4>), g, b, 0, s, t);
    return hipGetLastError();
}

template <class P>
hipError_t adj8_variant(const NudftTable& t, int nt, hipStream_t s) {
    const dim3 g(t.total_tiles), b(kThreads8);
    if (nt == 2) hipLaunchKernelGGL((nudft_adj8<P, 2>), g, b, 0, s, t);
    else if (nt == 3) hipLaunchKernelGGL((nudft_adj8<P, 3>), g, b, 0, s, t);
    else hipLaunchKernelGGL((nudft_adj8<P, 4>), g, b, 0, s, t);
    return hipGetLastError();
}

// Tiles of the adjoint: (slice, 32 y, 128 x, sample split).
int64_t adj8_tiles(const NudftItem& it) { return adj_tiles(it.nx, it.ny, it.nc, it.nb, it.ksplit); }

}  // namespace

hipError_t launch_nudft_forward(const NudftTable& t, int precision, hipStream_t s) {
    if (t.total_tiles <= 0) return hipSuccess;
    return launch_by_nt(t, [](const NudftItem& it) { return fwd_nt(it.ny); },
                        [](const NudftItem& it) { return (int64_t)it.ntiles; },
                        [&](const NudftTable& sub, int nt) {
                            return precision == MRI_BF16X3   ? fwd_variant<PolBF16>(sub, nt, s)
                                   : precision == MRI_FP16X3 ? fwd_variant<PolF16>(sub, nt, s)
                                                             : fwd_variant<PolF32>(sub, nt, s);
                        });
}

hipError_t launch_adj_phases(const NudftTable& t, hipStream_t s) {
    int64_t n = 0;
    for (int i = 0; i < t.nitems; ++i)
        n += adj_table_elems(t.it[i].nx, t.it[i].ny, t.it[i].nk, t.it[i].traj_bs ? t.it[i].nb : 1);
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), (int64_t)1 << 20);
    hipLaunchKernelGGL(k_adj_phases, dim3((unsigned)blocks), dim3(256), 0, s, t, n);
    return hipGetLastError();
}

hipError_t launch_nudft_adjoint(const NudftTable& t, int precision, hipStream_t s) {
    if (t.total_tiles <= 0) return hipSuccess;
    if (precision == MRI_FP16X3) {
        int64_t units = 0;
        for (int i = 0; i < t.nitems; ++i) units += (int64_t)t.it[i].nb * t.it[i].nc * t.it[i].ksplit;
        hipLaunchKernelGGL(k_adj_scale, dim3((unsigned)units), dim3(256), 0, s, t);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (precision == MRI_FP32)
        return launch_by_nt(t, [](const NudftItem& it) { return adj_nt(it.nc); }, adj8_tiles,
                            [&](const NudftTable& sub, int nt) { return adj8_variant<PolF32>(sub, nt, s); });
    return launch_by_nt(t, [](const NudftItem& it) { return adj_nt(it.nc); }, adj8_tiles,
                        [&](const NudftTable& sub, int nt) {
                            return precision == MRI_BF16X3 ? adj8_variant<PolBF16>(sub, nt, s)
                                                           : adj8_variant<PolF16>(sub, nt, s);
                        });
}

}  // namespace mri
