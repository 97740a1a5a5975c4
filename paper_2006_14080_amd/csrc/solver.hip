// Vector kernels of the ADMM-TV solve (eq. (6)-(13), Alg. 2, Alg. 4): the
// finite-difference transform and its adjoint, soft thresholding, the
// right-hand side, the CG updates, the dual update, and the reduction that
// finishes each application of the normal matrix A = F^H F + (beta/2) Theta^H Theta.
//
// All are memory-bound.  A block covers a tile of 64 columns x 16 rows of one
// slice; each thread owns one column and four consecutive rows, so a wave
// reads 64 consecutive pixels of a row (coalesced) and the stencils of Theta,
// Theta^H and Theta^H Theta get their vertical neighbours from rows the
// thread loads anyway (six rows for four outputs of the 5-point stencil) and
// their horizontal neighbours from the adjacent lanes (wave shuffles), with
// real loads only where a neighbour lies outside the wave's 64 columns or
// wraps around.  Every thread issues all its loads before any store.  Arrays
// a kernel touches once per pixel are read and written with non-temporal
// (streaming) accesses; arrays a stencil reads at neighbouring pixels use
// ordinary loads, so their lines stay in cache for the neighbours.  Vector
// arithmetic is FP32; inner products and norms accumulate in FP64 and are
// summed in a fixed order: wave shuffles, waves in index order, per-block
// partials written to memory, then one finalize block per slice (k_finalize)
// sums the partials in block order and applies the scalar logic of Alg. 2 /
// Alg. 4.  No atomics and no device-wide fences, so results are reproducible
// and nothing serialises the grid.
#include "device.h"
#include "solver.h"

namespace mri {
namespace {

// The tile of one block and this thread's place in it: column x, rows
// y0 .. y0 + kVecRows - 1 (those below ny, in a column below nx, are outputs).
struct Tile {
    int item, b, blk;
    int lane, x, y0;
    bool xok;
};

// Blocks are remapped so each XCD works on one contiguous band of rows: the
// stencils' neighbouring rows are then in that XCD's own L2.  Tiles are
// numbered column-tile fastest within a slice.
__device__ __forceinline__ Tile locate(const SolveTable& t) {
    const int g = xcd_remap(blockIdx.x, t.total_blocks);
    int i = 0;
    while (i + 1 < t.nitems && g >= t.it[i + 1].block_begin) ++i;
    const SolveItem& it = t.it[i];
    const int local = g - it.block_begin;
    Tile l;
    l.item = i;
    l.b = local / it.nblk;
    l.blk = local % it.nblk;
    const int ntx = (it.nx + kTileX - 1) / kTileX;
    const int tx = l.blk % ntx, ty = l.blk / ntx;
    l.lane = threadIdx.x % kTileX;
    l.x = tx * kTileX + l.lane;
    l.y0 = ty * kTileY + (threadIdx.x / kTileX) * kVecRows;
    l.xok = l.x < it.nx;
    return l;
}

// Row y0 + i of the thread's band for loads: rows past the image wrap to row
// 0 just past the end (the periodic neighbour of the last row) and otherwise
// clamp to the last row (their values are never used).
__device__ __forceinline__ int load_row(const Tile& l, int i, int ny) {
    const int r = l.y0 + i;
    return r < ny ? r : (r == ny ? 0 : ny - 1);
}
// The row above y0 (periodic), clamped like load_row.
__device__ __forceinline__ int row_above(const Tile& l, int ny) {
    return l.y0 == 0 ? ny - 1 : min(l.y0 - 1, ny - 1);
}
__device__ __forceinline__ bool row_ok(const Tile& l, int i, int ny) { return l.xok && l.y0 + i < ny; }

// Streaming (non-temporal) complex loads and stores.
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_nt(const float2* p) {
    const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st_nt(float2* p, float2 v) {
    __builtin_nontemporal_store(f2v{v.x, v.y}, reinterpret_cast<f2v*>(p));
}

// Horizontal periodic neighbours.  The lanes of a wave hold 64 adjacent
// columns of a row, so a value's left and right neighbours come from the
// adjacent lanes (wave shuffles); the first lane (left) and the last lane or
// the image's last column (right) take the edge values that wave_edges*
// loads with the thread's other loads.  left_of / right_of pick the shuffled
// or the edge value and must be called by every lane.
__device__ __forceinline__ float2 left_of(const Tile& l, float2 c, float2 edge) {
    const float2 v = make_float2(__shfl_up(c.x, 1, 64), __shfl_up(c.y, 1, 64));
    return l.lane == 0 ? edge : v;
}
__device__ __forceinline__ float2 right_of(const Tile& l, int nx, float2 c, float2 edge) {
    const float2 v = make_float2(__shfl_down(c.x, 1, 64), __shfl_down(c.y, 1, 64));
    return (l.lane == kTileX - 1 || l.x + 1 >= nx) ? edge : v;
}

// The edge columns of a wave's rows in one load instruction: lanes 0 .. R-1
// load the left neighbours of the wave's first column in its rows 0 .. R-1,
// lanes R .. 2R-1 the right neighbours of its last column (the column after
// the tile, or column 0 when the image's last column lies in the tile); every
// lane then receives all of them by shuffles, for left_of / right_of.
__device__ __forceinline__ void wave_edges(const float2* a, const Tile& l, int nx, int ny,
                                           float2 (&el)[kVecRows], float2 (&er)[kVecRows]) {
    static_assert(2 * kVecRows <= kTileX, "edge lanes");
    const int x0 = l.x - l.lane;
    float2 v = make_float2(0.f, 0.f);
    if (l.lane < 2 * kVecRows) {
        const int j = l.lane % kVecRows;
        const int col = l.lane < kVecRows ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + kTileX < nx ? x0 + kTileX : 0);
        v = a[(int64_t)load_row(l, j, ny) * nx + col];
    }
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        el[j] = make_float2(__shfl(v.x, j, 64), __shfl(v.y, j, 64));
        er[j] = make_float2(__shfl(v.x, kVecRows + j, 64), __shfl(v.y, kVecRows + j, 64));
    }
}
// Only the left edges (lanes 0 .. R-1 load).
__device__ __forceinline__ void wave_edges_left(const float2* a, const Tile& l, int nx, int ny,
                                                float2 (&el)[kVecRows]) {
    const int x0 = l.x - l.lane;
    float2 v = make_float2(0.f, 0.f);
    if (l.lane < kVecRows) v = a[(int64_t)load_row(l, l.lane, ny) * nx + (x0 == 0 ? nx - 1 : x0 - 1)];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) el[j] = make_float2(__shfl(v.x, j, 64), __shfl(v.y, j, 64));
}
// Only the right edges (lanes 0 .. R-1 load).
__device__ __forceinline__ void wave_edges_right(const float2* a, const Tile& l, int nx, int ny,
                                                 float2 (&er)[kVecRows]) {
    const int x0 = l.x - l.lane;
    float2 v = make_float2(0.f, 0.f);
    if (l.lane < kVecRows) v = a[(int64_t)load_row(l, l.lane, ny) * nx + (x0 + kTileX < nx ? x0 + kTileX : 0)];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) er[j] = make_float2(__shfl(v.x, j, 64), __shfl(v.y, j, 64));
}

// The block's row groups (one per wave, kVecRows rows each) pass rows to
// their neighbours through LDS: the row above a group is the previous group's
// last row and the row below is the next group's first row, so only the
// first group loads the row above the tile and only the last group the row
// below it.  Every thread of the block must call it.
constexpr int kRowGroups = kVecThreads / kTileX;
__device__ __forceinline__ void swap_rows(const Tile& l, float2 first, float2 last, float2& above, float2& below) {
    __shared__ float2 s[2][kRowGroups][kTileX];
    const int g = threadIdx.x / kTileX;
    s[0][g][l.lane] = first;
    s[1][g][l.lane] = last;
    __syncthreads();
    if (g > 0) above = s[1][g - 1][l.lane];
    if (g < kRowGroups - 1) below = s[0][g + 1][l.lane];
}
__device__ __forceinline__ int row_group() { return threadIdx.x / kTileX; }

__device__ __forceinline__ double cnorm2(float2 a) {
    return (double)a.x * a.x + (double)a.y * a.y;
}

// Block partials (two FP64 values per block) -> red[b][0..1][blk], summed in
// a fixed order: wave shuffles, then the block's waves in index order.
__device__ __forceinline__ void block_partials(double v0, double v1, const SolveItem& it, int b, int blk) {
    __shared__ double sm[2][kVecThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    v0 = wave_sum(v0);
    v1 = wave_sum(v1);
    if (lane == 0) {
        sm[0][w] = v0;
        sm[1][w] = v1;
    }
    __syncthreads();
    if (tid == 0) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < kVecThreads / 64; ++k) {
            s0 += sm[0][k];
            s1 += sm[1][k];
        }
        double* red = it.red + (int64_t)b * 2 * it.nblk;
        red[blk] = s0;
        red[it.nblk + blk] = s1;
    }
}

__device__ __forceinline__ bool finite(double v) { return isfinite(v); }

__device__ __forceinline__ void fail_numeric(SolveScalars& s) {
    s.status = MRI_ENUMERIC;
    s.admm_active = 0;
    s.cg_active = 0;
}

// ---- initialisation: rho = x0 (or 0), eta = 0, scalars reset ---------------
__global__ __launch_bounds__(kVecThreads) void k_solve_init(const SolveTable tab) {
    const Tile l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    const int64_t base = (int64_t)l.b * it.npix, ebase = 2 * base;
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        if (!row_ok(l, j, it.ny)) break;
        const int64_t pix = (int64_t)(l.y0 + j) * it.nx + l.x;
        const float2 v = it.x0 ? it.x0[base + pix] : make_float2(0.f, 0.f);
        st_nt(it.rho + base + pix, v);
        st_nt(it.rho0 + base + pix, v);
        st_nt(it.eta + ebase + pix, make_float2(0.f, 0.f));
        st_nt(it.eta + ebase + it.npix + pix, make_float2(0.f, 0.f));
    }
    if (l.blk == 0 && threadIdx.x == 0) {
        SolveScalars& s = it.sc[l.b];
        s.tau = s.alpha_cg = s.beta_cg = s.pap = 0.0;
        s.alpha_admm = 1.0;
        s.admm_active = 1;
        s.cg_active = 0;
        s.admm_iters = 0;
        s.cg_steps = 0;
        s.status = MRI_OK;
        s.cg_it = 0;
        s.pad = 0;
        if (it.admm_max <= 0) s.admm_active = 0;
    }
}

// ---- eq. (9)-(10): mu = S_{lambda/beta}(Theta rho + eta) ---------------------
// Theta rho at (y, x) = (rho(y, x+1) - rho(y, x), rho(y+1, x) - rho(y, x)).
__global__ __launch_bounds__(kVecThreads) void k_mu(const SolveTable tab) {
    const Tile l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    if (!it.sc[l.b].admm_active) return;
    const int nx = it.nx, ny = it.ny;
    const int xc = min(l.x, nx - 1);
    const float2* rho = it.rho + (int64_t)l.b * it.npix;
    const float2* eta = it.eta + (int64_t)l.b * 2 * it.npix;
    float2* mu = it.mu + (int64_t)l.b * 2 * it.npix;
    float2 r[kVecRows + 1], e0[kVecRows], e1[kVecRows], er[kVecRows];
    wave_edges_right(rho, l, nx, ny, er);
#pragma unroll
    for (int i = 0; i < kVecRows; ++i) r[i] = rho[(int64_t)load_row(l, i, ny) * nx + xc];
    float2 unused = make_float2(0.f, 0.f);
    r[kVecRows] = make_float2(0.f, 0.f);
    if (row_group() == kRowGroups - 1) r[kVecRows] = rho[(int64_t)load_row(l, kVecRows, ny) * nx + xc];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        const int64_t pix = (int64_t)load_row(l, j, ny) * nx + xc;
        e0[j] = ld_nt(eta + pix);
        e1[j] = ld_nt(eta + it.npix + pix);
    }
    swap_rows(l, r[0], r[kVecRows - 1], unused, r[kVecRows]);
    float2 rr[kVecRows];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) rr[j] = right_of(l, nx, r[j], er[j]);
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        if (!row_ok(l, j, ny)) break;
        const int64_t pix = (int64_t)(l.y0 + j) * nx + l.x;
        const float2 z[2] = {cadd(csub(rr[j], r[j]), e0[j]), cadd(csub(r[j + 1], r[j]), e1[j])};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float mag = sqrtf(z[c].x * z[c].x + z[c].y * z[c].y);
            const float sc = mag > it.thr ? 1.0f - it.thr / mag : 0.0f;
            st_nt(mu + c * it.npix + pix, cscale(z[c], sc));
        }
    }
}

// ---- eq. (13): b = F^H d + (beta/2) Theta^H (mu - eta) -----------------------
// Theta^H g at (y, x) = g0(y, x-1) - g0(y, x) + g1(y-1, x) - g1(y, x), g = mu - eta.
__global__ __launch_bounds__(kVecThreads) void k_rhs(const SolveTable tab) {
    const Tile l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    if (!it.sc[l.b].admm_active) return;
    const int nx = it.nx, ny = it.ny;
    const int xc = min(l.x, nx - 1);
    const int64_t e = (int64_t)l.b * 2 * it.npix;
    const float2* mu0 = it.mu + e;
    const float2* mu1 = mu0 + it.npix;
    const float2* et0 = it.eta + e;
    const float2* et1 = et0 + it.npix;
    const int64_t base = (int64_t)l.b * it.npix;
    // g1 on the row above the band and the band's rows; g0 on the band's rows
    float2 g1[kVecRows + 1], g0[kVecRows], fh[kVecRows], el[kVecRows], ml[kVecRows], tl[kVecRows];
    wave_edges_left(mu0, l, nx, ny, ml);      // g0 at x - 1 for lane 0
    wave_edges_left(et0, l, nx, ny, tl);
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) el[j] = csub(ml[j], tl[j]);
    g1[0] = make_float2(0.f, 0.f);
    if (row_group() == 0) {
        const int64_t pa = (int64_t)row_above(l, ny) * nx + xc;
        g1[0] = csub(mu1[pa], et1[pa]);
    }
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        const int64_t pix = (int64_t)load_row(l, j, ny) * nx + xc;
        g1[j + 1] = csub(mu1[pix], et1[pix]);
        g0[j] = csub(mu0[pix], et0[pix]);
        fh[j] = ld_nt(it.fhd + base + pix);
    }
    float2 unused = make_float2(0.f, 0.f);
    swap_rows(l, g1[1], g1[kVecRows], g1[0], unused);
    float2 gl[kVecRows];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) gl[j] = left_of(l, g0[j], el[j]);
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        if (!row_ok(l, j, ny)) break;
        const float2 th = cadd(csub(gl[j], g0[j]), csub(g1[j], g1[j + 1]));
        st_nt(it.b + base + (int64_t)(l.y0 + j) * nx + l.x, cadd(fh[j], cscale(th, it.half_beta)));
    }
}

// ---- finish one application of A (or F^H d) from the adjoint's partials ------
// kFinishFhd:    fhd = sum of partials
// kFinishCgInit: q = A src; r = b - q; p = r; xnew = src; tau = r^H r   (Alg. 2 start)
// kFinishCgStep: q = A p; pAp = Re(p^H q)                               (Alg. 2 step)
// with A v = F^H F v + (beta/2) Theta^H Theta v and Theta^H Theta v the
// periodic 5-point stencil 4 v - (four neighbours).
template <int mode>
__global__ __launch_bounds__(kVecThreads) void k_adj_finish(const SolveTable tab) {
    const Tile l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    SolveScalars& sc = it.sc[l.b];
    if constexpr (mode == kFinishCgInit) {
        if (!sc.admm_active) return;
    }
    if constexpr (mode == kFinishCgStep) {
        if (!sc.cg_active) return;
    }
    const int nx = it.nx, ny = it.ny;
    const int xc = min(l.x, nx - 1);
    const int64_t base = (int64_t)l.b * it.npix;
    const int64_t stride = (int64_t)it.nb * it.npix;
    int64_t pc[kVecRows];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) pc[j] = (int64_t)load_row(l, j, ny) * nx + xc;
    // The stencil's and the CG start's operands first (rows above, within and
    // below the band, edge columns, b), then the partial images.
    const float2* src = mode == kFinishCgStep ? it.p + base : (it.warm ? it.rho + base : it.rho0 + base);
    float2 c[kVecRows + 2], el[kVecRows], er[kVecRows], bv[kVecRows];
    if constexpr (mode != kFinishFhd) {
        wave_edges(src, l, nx, ny, el, er);
        c[0] = c[kVecRows + 1] = make_float2(0.f, 0.f);
        if (row_group() == 0) c[0] = src[(int64_t)row_above(l, ny) * nx + xc];
#pragma unroll
        for (int i = 0; i < kVecRows; ++i) c[i + 1] = src[(int64_t)load_row(l, i, ny) * nx + xc];
        if (row_group() == kRowGroups - 1) c[kVecRows + 1] = src[(int64_t)load_row(l, kVecRows, ny) * nx + xc];
        if constexpr (mode == kFinishCgInit) {
#pragma unroll
            for (int j = 0; j < kVecRows; ++j) bv[j] = ld_nt(it.b + base + pc[j]);
        }
    }
    // Partial images in plane order (FP64).
    double sr[kVecRows], si[kVecRows];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) sr[j] = si[j] = 0.0;
    const float2* pp = it.part + base;
#pragma unroll 2
    for (int s = 0; s < it.ksplit; ++s) {
        float2 v[kVecRows];
#pragma unroll
        for (int j = 0; j < kVecRows; ++j) v[j] = ld_nt(pp + s * stride + pc[j]);
#pragma unroll
        for (int j = 0; j < kVecRows; ++j) {
            sr[j] += v[j].x;
            si[j] += v[j].y;
        }
    }
    if constexpr (mode == kFinishFhd) {
#pragma unroll
        for (int j = 0; j < kVecRows; ++j)
            if (row_ok(l, j, ny)) st_nt(it.fhd + base + pc[j], make_float2((float)sr[j], (float)si[j]));
    } else {
        swap_rows(l, c[1], c[kVecRows], c[0], c[kVecRows + 1]);
        float2 q[kVecRows];
#pragma unroll
        for (int j = 0; j < kVecRows; ++j) {
            const float2 lft = left_of(l, c[j + 1], el[j]);
            const float2 rgt = right_of(l, nx, c[j + 1], er[j]);
            float2 lap = cscale(c[j + 1], 4.0f);
            lap = csub(lap, rgt);
            lap = csub(lap, lft);
            lap = csub(lap, c[j + 2]);
            lap = csub(lap, c[j]);
            q[j] = cadd(make_float2((float)sr[j], (float)si[j]), cscale(lap, it.half_beta));
        }
        double v0 = 0.0;
#pragma unroll
        for (int j = 0; j < kVecRows; ++j) {
            if (!row_ok(l, j, ny)) break;
            const int64_t o = base + pc[j];
            const float2 cj = c[j + 1];
            if constexpr (mode == kFinishCgStep) {
                st_nt(it.q + o, q[j]);
                v0 += (double)cj.x * q[j].x + (double)cj.y * q[j].y;
            } else {
                // Plain (cached) stores: with three output streams the
                // streaming form ran the CG start 6 % slower on multi-GB
                // arrays; the kernels that read r, p and x next are unchanged.
                const float2 r = csub(bv[j], q[j]);
                it.r[o] = r;
                it.p[o] = r;
                it.xnew[o] = cj;
                v0 += cnorm2(r);
            }
        }
        block_partials(v0, 0.0, it, l.b, l.blk);
    }
}

// ---- Alg. 2 step: x += alpha d; r -= alpha A d; tau' = r^H r ------------------
__global__ __launch_bounds__(kVecThreads) void k_cg_update(const SolveTable tab) {
    const Tile l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    const SolveScalars& sc = it.sc[l.b];
    if (!sc.cg_active) return;
    const float a = (float)sc.alpha_cg;
    const int nx = it.nx, ny = it.ny;
    const int xc = min(l.x, nx - 1);
    const int64_t base = (int64_t)l.b * it.npix;
    float2 x[kVecRows], r[kVecRows];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        const int64_t o = base + (int64_t)load_row(l, j, ny) * nx + xc;
        const float2 p = ld_nt(it.p + o), q = ld_nt(it.q + o);
        x[j] = ld_nt(it.xnew + o);
        r[j] = ld_nt(it.r + o);
        x[j] = make_float2(fmaf(a, p.x, x[j].x), fmaf(a, p.y, x[j].y));
        r[j] = make_float2(fmaf(-a, q.x, r[j].x), fmaf(-a, q.y, r[j].y));
    }
    double v0 = 0.0;
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        if (!row_ok(l, j, ny)) break;
        const int64_t o = base + (int64_t)(l.y0 + j) * nx + l.x;
        st_nt(it.xnew + o, x[j]);
        st_nt(it.r + o, r[j]);
        v0 += cnorm2(r[j]);
    }
    block_partials(v0, 0.0, it, l.b, l.blk);
}

// ---- Alg. 2 direction: d = r + (tau'/tau) d -----------------------------------
__global__ __launch_bounds__(kVecThreads) void k_cg_dir(const SolveTable tab) {
    const Tile l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    const SolveScalars& sc = it.sc[l.b];
    if (!sc.cg_active) return;
    const float bc = (float)sc.beta_cg;
    const int nx = it.nx, ny = it.ny;
    const int xc = min(l.x, nx - 1);
    const int64_t base = (int64_t)l.b * it.npix;
    float2 d[kVecRows];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        const int64_t o = base + (int64_t)load_row(l, j, ny) * nx + xc;
        const float2 r = ld_nt(it.r + o), p = ld_nt(it.p + o);
        d[j] = make_float2(fmaf(bc, p.x, r.x), fmaf(bc, p.y, r.y));
    }
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        if (!row_ok(l, j, ny)) break;
        st_nt(it.p + base + (int64_t)(l.y0 + j) * nx + l.x, d[j]);
    }
}

// ---- eq. (8) and Alg. 4: eta += Theta rho' - mu; alpha; rho = rho' ------------
__global__ __launch_bounds__(kVecThreads) void k_dual(const SolveTable tab) {
    const Tile l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    if (!it.sc[l.b].admm_active) return;
    const int nx = it.nx, ny = it.ny;
    const int xc = min(l.x, nx - 1);
    const int64_t base = (int64_t)l.b * it.npix;
    const float2* xn = it.xnew + base;
    float2* eta = it.eta + 2 * base;
    const float2* mu = it.mu + 2 * base;
    float2 c[kVecRows + 1], e0[kVecRows], e1[kVecRows], m0[kVecRows], m1[kVecRows], old[kVecRows], er[kVecRows];
    wave_edges_right(xn, l, nx, ny, er);
#pragma unroll
    for (int i = 0; i < kVecRows; ++i) c[i] = xn[(int64_t)load_row(l, i, ny) * nx + xc];
    c[kVecRows] = make_float2(0.f, 0.f);
    if (row_group() == kRowGroups - 1) c[kVecRows] = xn[(int64_t)load_row(l, kVecRows, ny) * nx + xc];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        const int64_t pix = (int64_t)load_row(l, j, ny) * nx + xc;
        e0[j] = ld_nt(eta + pix);
        e1[j] = ld_nt(eta + it.npix + pix);
        m0[j] = ld_nt(mu + pix);
        m1[j] = ld_nt(mu + it.npix + pix);
        old[j] = ld_nt(it.rho + base + pix);
    }
    float2 unused = make_float2(0.f, 0.f);
    swap_rows(l, c[0], c[kVecRows - 1], unused, c[kVecRows]);
    float2 rr[kVecRows];
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) rr[j] = right_of(l, nx, c[j], er[j]);
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        if (!row_ok(l, j, ny)) break;
        const int64_t pix = (int64_t)(l.y0 + j) * nx + l.x;
        st_nt(eta + pix, cadd(e0[j], csub(csub(rr[j], c[j]), m0[j])));
        st_nt(eta + it.npix + pix, cadd(e1[j], csub(csub(c[j + 1], c[j]), m1[j])));
        num += cnorm2(csub(c[j], old[j]));
        den += cnorm2(old[j]);
        st_nt(it.rho + base + pix, c[j]);
    }
    block_partials(num, den, it, l.b, l.blk);
}

// ---- per-slice scalar logic of Alg. 2 / Alg. 4 ----------------------------------
// One block per slice sums the block partials of the preceding kernel in
// block order and updates the slice's scalars.  It runs under the same
// condition as the kernel that wrote the partials (flags are unchanged in
// between), so every written partial is consumed exactly once.
__global__ __launch_bounds__(kVecThreads) void k_finalize(const SolveTable tab, int mode) {
    const int g = blockIdx.x;
    int i = 0;
    while (i + 1 < tab.nitems && g >= tab.it[i + 1].slice_begin) ++i;
    const SolveItem& it = tab.it[i];
    const int b = g - it.slice_begin;
    SolveScalars& s = it.sc[b];
    const bool run = (mode == kFinCgInit || mode == kFinDual) ? s.admm_active != 0 : s.cg_active != 0;
    if (!run) return;
    __shared__ double tot[2][kVecThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double* red = it.red + (int64_t)b * 2 * it.nblk;
    double a0 = 0.0, a1 = 0.0;
    for (int k = tid; k < it.nblk; k += kVecThreads) {
        a0 += red[k];
        a1 += red[it.nblk + k];
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) {
        tot[0][w] = a0;
        tot[1][w] = a1;
    }
    __syncthreads();
    if (tid != 0) return;
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int k = 0; k < kVecThreads / 64; ++k) {
        t0 += tot[0][k];
        t1 += tot[1][k];
    }
    if (!finite(t0) || !finite(t1)) {
        fail_numeric(s);
        return;
    }
    switch (mode) {
        case kFinCgInit:            // tau = r^H r of r = b - A x0
            s.tau = t0;
            s.cg_it = 0;
            s.cg_active = (t0 > it.atol2 && it.cg_max > 0) ? 1 : 0;
            break;
        case kFinCgStep:            // alpha = tau / Re(d^H A d), breakdown guard
            s.pap = t0;
            if (t0 > 0.0)
                s.alpha_cg = s.tau / t0;
            else
                s.cg_active = 0;
            break;
        case kFinCgUpdate:          // tau' = r^H r; beta = tau'/tau; stopping tests
            s.beta_cg = t0 / s.tau;
            s.tau = t0;
            s.cg_steps += 1;
            s.cg_it += 1;
            s.cg_active = (t0 > it.atol2 && s.cg_it < it.cg_max) ? 1 : 0;
            break;
        default: {                  // kFinDual: alpha = ||rho' - rho||^2 / ||rho||^2 (Alg. 4)
            const double a = t1 > 0.0 ? t0 / t1 : (t0 > 0.0 ? 1.0 : 0.0);
            s.alpha_admm = a;
            s.admm_iters += 1;
            if (!(a > it.rtol2) || s.admm_iters >= it.admm_max) {
                s.admm_active = 0;
                s.cg_active = 0;
            }
        }
    }
}

// ---- output and per-slice report ---------------------------------------------
__global__ __launch_bounds__(kVecThreads) void k_solve_final(const SolveTable tab) {
    const Tile l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    const int64_t base = (int64_t)l.b * it.npix;
#pragma unroll
    for (int j = 0; j < kVecRows; ++j) {
        if (!row_ok(l, j, it.ny)) break;
        const int64_t o = base + (int64_t)(l.y0 + j) * it.nx + l.x;
        it.x_out[o] = ld_nt(it.rho + o);
    }
    if (it.stats && l.blk == 0 && threadIdx.x == 0) {
        const SolveScalars& s = it.sc[l.b];
        mri_admm_stats st;
        st.admm_iters_run = s.admm_iters;
        st.cg_steps_run = s.cg_steps;
        st.alpha = s.alpha_admm;
        st.tau = s.tau;
        st.status = s.status;
        st.pad = 0;
        it.stats[l.b] = st;
    }
}

// ---- plain kernels behind the single-operator entry points ------------------
__global__ __launch_bounds__(kVecThreads) void k_sum_partials(const float2* __restrict__ part, int ksplit,
                                                              int64_t n, float2* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
    if (i >= n) return;
    double sr = 0.0, si = 0.0;
    int s = 0;
    for (; s + 8 <= ksplit; s += 8) {      // loads first, additions in plane order
        float2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = part[(s + j) * n + i];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sr += v[j].x;
            si += v[j].y;
        }
    }
    for (; s < ksplit; ++s) {
        const float2 v = part[s * n + i];
        sr += v.x;
        si += v.y;
    }
    out[i] = make_float2((float)sr, (float)si);
}

// Periodic neighbours of pixel p in an ny x nx image (the single-operator
// transforms, which run once per call).
struct Nb {
    int64_t xp, xm, yp, ym;   // (i, j+1), (i, j-1), (i+1, j), (i-1, j)
};
__device__ __forceinline__ Nb neighbours(int p, int nx, int ny) {
    const int i = p / nx, j = p - i * nx;
    const int jp = j + 1 == nx ? 0 : j + 1, jm = j == 0 ? nx - 1 : j - 1;
    const int ip = i + 1 == ny ? 0 : i + 1, im = i == 0 ? ny - 1 : i - 1;
    Nb n;
    n.xp = (int64_t)i * nx + jp;
    n.xm = (int64_t)i * nx + jm;
    n.yp = (int64_t)ip * nx + j;
    n.ym = (int64_t)im * nx + j;
    return n;
}

__global__ __launch_bounds__(kVecThreads) void k_tv_forward(int nx, int ny, const float2* __restrict__ x,
                                                            float2* __restrict__ g) {
    const int npix = nx * ny;
    const int p = blockIdx.x * kVecThreads + threadIdx.x;
    if (p >= npix) return;
    const int64_t b = blockIdx.y;
    const float2* xb = x + b * npix;
    const Nb nb = neighbours(p, nx, ny);
    const float2 c = xb[p];
    g[2 * b * npix + p] = csub(xb[nb.xp], c);
    g[(2 * b + 1) * npix + p] = csub(xb[nb.yp], c);
}

__global__ __launch_bounds__(kVecThreads) void k_tv_adjoint(int nx, int ny, const float2* __restrict__ g,
                                                            float2* __restrict__ x) {
    const int npix = nx * ny;
    const int p = blockIdx.x * kVecThreads + threadIdx.x;
    if (p >= npix) return;
    const int64_t b = blockIdx.y;
    const float2* g0 = g + 2 * b * npix;
    const float2* g1 = g0 + npix;
    const Nb nb = neighbours(p, nx, ny);
    x[b * npix + p] = cadd(csub(g0[nb.xm], g0[p]), csub(g1[nb.ym], g1[p]));
}

inline dim3 grid_of(const SolveTable& t) { return dim3(t.total_blocks); }

}  // namespace

hipError_t launch_solve_init(const SolveTable& t, hipStream_t s) {
    hipLaunchKernelGGL(k_solve_init, grid_of(t), dim3(kVecThreads), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_mu(const SolveTable& t, hipStream_t s) {
    hipLaunchKernelGGL(k_mu, grid_of(t), dim3(kVecThreads), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_rhs(const SolveTable& t, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs, grid_of(t), dim3(kVecThreads), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_adj_finish(const SolveTable& t, int mode, hipStream_t s) {
    if (mode == kFinishFhd) hipLaunchKernelGGL(k_adj_finish<kFinishFhd>, grid_of(t), dim3(kVecThreads), 0, s, t);
    else if (mode == kFinishCgInit)
        hipLaunchKernelGGL(k_adj_finish<kFinishCgInit>, grid_of(t), dim3(kVecThreads), 0, s, t);
    else hipLaunchKernelGGL(k_adj_finish<kFinishCgStep>, grid_of(t), dim3(kVecThreads), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_cg_update(const SolveTable& t, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_update, grid_of(t), dim3(kVecThreads), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_cg_dir(const SolveTable& t, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_dir, grid_of(t), dim3(kVecThreads), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_dual(const SolveTable& t, hipStream_t s) {
    hipLaunchKernelGGL(k_dual, grid_of(t), dim3(kVecThreads), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_finalize(const SolveTable& t, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(t.total_slices), dim3(kVecThreads), 0, s, t, mode);
    return hipGetLastError();
}
hipError_t launch_solve_final(const SolveTable& t, hipStream_t s) {
    hipLaunchKernelGGL(k_solve_final, grid_of(t), dim3(kVecThreads), 0, s, t);
    return hipGetLastError();
}
hipError_t launch_sum_partials(const float2* part, int ksplit, int64_t n, float2* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)ceil_div(n, kVecThreads)), dim3(kVecThreads), 0, s,
                       part, ksplit, n, out);
    return hipGetLastError();
}
hipError_t launch_tv_forward(int nx, int ny, int nb, const float2* x, float2* g, hipStream_t s) {
    const int64_t npix = (int64_t)nx * ny;
    if (npix <= 0 || nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tv_forward, dim3((unsigned)ceil_div(npix, kVecThreads), nb), dim3(kVecThreads), 0, s,
                       nx, ny, x, g);
    return hipGetLastError();
}
hipError_t launch_tv_adjoint(int nx, int ny, int nb, const float2* g, float2* x, hipStream_t s) {
    const int64_t npix = (int64_t)nx * ny;
    if (npix <= 0 || nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tv_adjoint, dim3((unsigned)ceil_div(npix, kVecThreads), nb), dim3(kVecThreads), 0, s,
                       nx, ny, g, x);
    return hipGetLastError();
}

}  // namespace mri
