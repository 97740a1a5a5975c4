// Vector kernels of the ADMM-TV solve (eq. (6)-(13), Alg. 2, Alg. 4): the
// finite-difference transform and its adjoint, soft thresholding, the
// right-hand side, the CG updates, the dual update, and the reduction that
// finishes each application of the normal matrix A = F^H F + (beta/2) Theta^H Theta.
//
// All are memory-bound: each thread takes kVecPix pixels kVecThreads apart
// (coalesced along x), issuing the loads of all of them before any store so
// a wave keeps several requests in flight per array.  Vector
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

struct Loc {
    int item, b, blk;
    int pix0;           // first pixel of this thread; its others follow every kVecThreads
};

// Blocks are remapped so each XCD works on one contiguous pixel range: the
// stencils' neighbouring rows are then in that XCD's own L2.
__device__ __forceinline__ Loc locate(const SolveTable& t) {
    const int g = xcd_remap(blockIdx.x, t.total_blocks);
    int i = 0;
    while (i + 1 < t.nitems && g >= t.it[i + 1].block_begin) ++i;
    const SolveItem& it = t.it[i];
    const int local = g - it.block_begin;
    Loc l;
    l.item = i;
    l.b = local / it.nblk;
    l.blk = local % it.nblk;
    l.pix0 = l.blk * kVecBlockPix + (int)threadIdx.x;
    return l;
}

__device__ __forceinline__ int pix_of(const Loc& l, int j) { return l.pix0 + j * kVecThreads; }

// Periodic neighbours of pixel p in an ny x nx image.
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
    const Loc l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    const int npix = (int)it.npix;
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int pix = pix_of(l, j);
        if (pix >= npix) break;
        const int64_t o = (int64_t)l.b * it.npix + pix;
        const float2 v = it.x0 ? it.x0[o] : make_float2(0.f, 0.f);
        it.rho[o] = v;
        it.rho0[o] = v;
        const int64_t e = (int64_t)l.b * 2 * it.npix + pix;
        it.eta[e] = make_float2(0.f, 0.f);
        it.eta[e + it.npix] = make_float2(0.f, 0.f);
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
__global__ __launch_bounds__(kVecThreads) void k_mu(const SolveTable tab) {
    const Loc l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    if (!it.sc[l.b].admm_active) return;
    const int npix = (int)it.npix;
    const float2* rho = it.rho + (int64_t)l.b * it.npix;
    const float2* eta = it.eta + (int64_t)l.b * 2 * it.npix;
    float2* mu = it.mu + (int64_t)l.b * 2 * it.npix;
    float2 z0[kVecPix], z1[kVecPix];
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int pix = min(pix_of(l, j), npix - 1);
        const Nb n = neighbours(pix, it.nx, it.ny);
        const float2 r0 = rho[pix];
        z0[j] = cadd(csub(rho[n.xp], r0), eta[pix]);
        z1[j] = cadd(csub(rho[n.yp], r0), eta[pix + it.npix]);
    }
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int pix = pix_of(l, j);
        if (pix >= npix) break;
        const float2 z[2] = {z0[j], z1[j]};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float mag = sqrtf(z[c].x * z[c].x + z[c].y * z[c].y);
            const float sc = mag > it.thr ? 1.0f - it.thr / mag : 0.0f;
            mu[pix + c * it.npix] = cscale(z[c], sc);
        }
    }
}

// ---- eq. (13): b = F^H d + (beta/2) Theta^H (mu - eta) -----------------------
__global__ __launch_bounds__(kVecThreads) void k_rhs(const SolveTable tab) {
    const Loc l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    if (!it.sc[l.b].admm_active) return;
    const int npix = (int)it.npix;
    const int64_t e = (int64_t)l.b * 2 * it.npix;
    const float2* mu0 = it.mu + e;
    const float2* mu1 = mu0 + it.npix;
    const float2* et0 = it.eta + e;
    const float2* et1 = et0 + it.npix;
    const int64_t base = (int64_t)l.b * it.npix;
    float2 out[kVecPix];
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int p = min(pix_of(l, j), npix - 1);
        const Nb n = neighbours(p, it.nx, it.ny);
        // Theta^H g = g0(i, j-1) - g0(i, j) + g1(i-1, j) - g1(i, j), g = mu - eta
        const float2 g0m = csub(mu0[n.xm], et0[n.xm]), g0 = csub(mu0[p], et0[p]);
        const float2 g1m = csub(mu1[n.ym], et1[n.ym]), g1 = csub(mu1[p], et1[p]);
        const float2 th = cadd(csub(g0m, g0), csub(g1m, g1));
        out[j] = cadd(it.fhd[base + p], cscale(th, it.half_beta));
    }
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int p = pix_of(l, j);
        if (p >= npix) break;
        it.b[base + p] = out[j];
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
    const Loc l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    SolveScalars& sc = it.sc[l.b];
    if constexpr (mode == kFinishCgInit) {
        if (!sc.admm_active) return;
    }
    if constexpr (mode == kFinishCgStep) {
        if (!sc.cg_active) return;
    }
    const int npix = (int)it.npix;
    const int64_t base = (int64_t)l.b * it.npix;
    const int64_t stride = (int64_t)it.nb * it.npix;
    // Partial images in plane order (FP64), all pixels of the thread at once.
    double sr[kVecPix], si[kVecPix];
    int pc[kVecPix];
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        pc[j] = min(pix_of(l, j), npix - 1);
        sr[j] = si[j] = 0.0;
    }
    const float2* pp = it.part + base;
    for (int s = 0; s < it.ksplit; ++s) {
        float2 v[kVecPix];
#pragma unroll
        for (int j = 0; j < kVecPix; ++j) v[j] = pp[s * stride + pc[j]];
#pragma unroll
        for (int j = 0; j < kVecPix; ++j) {
            sr[j] += v[j].x;
            si[j] += v[j].y;
        }
    }
    double v0 = 0.0;
    if constexpr (mode == kFinishFhd) {
#pragma unroll
        for (int j = 0; j < kVecPix; ++j)
            if (pix_of(l, j) < npix) it.fhd[base + pc[j]] = make_float2((float)sr[j], (float)si[j]);
    } else {
        const float2* src = mode == kFinishCgStep ? it.p + base : (it.warm ? it.rho + base : it.rho0 + base);
        float2 q[kVecPix], c[kVecPix], bv[kVecPix];
#pragma unroll
        for (int j = 0; j < kVecPix; ++j) {
            const Nb n = neighbours(pc[j], it.nx, it.ny);
            c[j] = src[pc[j]];
            float2 lap = cscale(c[j], 4.0f);
            lap = csub(lap, src[n.xp]);
            lap = csub(lap, src[n.xm]);
            lap = csub(lap, src[n.yp]);
            lap = csub(lap, src[n.ym]);
            q[j] = cadd(make_float2((float)sr[j], (float)si[j]), cscale(lap, it.half_beta));
            if constexpr (mode == kFinishCgInit) bv[j] = it.b[base + pc[j]];
        }
#pragma unroll
        for (int j = 0; j < kVecPix; ++j) {
            if (pix_of(l, j) >= npix) break;
            const int64_t o = base + pc[j];
            if constexpr (mode == kFinishCgStep) {
                it.q[o] = q[j];
                v0 += (double)c[j].x * q[j].x + (double)c[j].y * q[j].y;
            } else {
                const float2 r = csub(bv[j], q[j]);
                it.r[o] = r;
                it.p[o] = r;
                it.xnew[o] = c[j];
                v0 += cnorm2(r);
            }
        }
        block_partials(v0, 0.0, it, l.b, l.blk);
    }
}

// ---- Alg. 2 step: x += alpha d; r -= alpha A d; tau' = r^H r ------------------
__global__ __launch_bounds__(kVecThreads) void k_cg_update(const SolveTable tab) {
    const Loc l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    const SolveScalars& sc = it.sc[l.b];
    if (!sc.cg_active) return;
    const float a = (float)sc.alpha_cg;
    const int npix = (int)it.npix;
    const int64_t base = (int64_t)l.b * it.npix;
    float2 x[kVecPix], r[kVecPix];
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int64_t o = base + min(pix_of(l, j), npix - 1);
        const float2 p = it.p[o], q = it.q[o];
        x[j] = it.xnew[o];
        r[j] = it.r[o];
        x[j] = make_float2(fmaf(a, p.x, x[j].x), fmaf(a, p.y, x[j].y));
        r[j] = make_float2(fmaf(-a, q.x, r[j].x), fmaf(-a, q.y, r[j].y));
    }
    double v0 = 0.0;
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int pix = pix_of(l, j);
        if (pix >= npix) break;
        it.xnew[base + pix] = x[j];
        it.r[base + pix] = r[j];
        v0 += cnorm2(r[j]);
    }
    block_partials(v0, 0.0, it, l.b, l.blk);
}

// ---- Alg. 2 direction: d = r + (tau'/tau) d -----------------------------------
__global__ __launch_bounds__(kVecThreads) void k_cg_dir(const SolveTable tab) {
    const Loc l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    const SolveScalars& sc = it.sc[l.b];
    if (!sc.cg_active) return;
    const float bc = (float)sc.beta_cg;
    const int npix = (int)it.npix;
    const int64_t base = (int64_t)l.b * it.npix;
    float2 d[kVecPix];
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int64_t o = base + min(pix_of(l, j), npix - 1);
        const float2 r = it.r[o], p = it.p[o];
        d[j] = make_float2(fmaf(bc, p.x, r.x), fmaf(bc, p.y, r.y));
    }
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int pix = pix_of(l, j);
        if (pix >= npix) break;
        it.p[base + pix] = d[j];
    }
}

// ---- eq. (8) and Alg. 4: eta += Theta rho' - mu; alpha; rho = rho' ------------
__global__ __launch_bounds__(kVecThreads) void k_dual(const SolveTable tab) {
    const Loc l = locate(tab);
    const SolveItem& it = tab.it[l.item];
    if (!it.sc[l.b].admm_active) return;
    const int npix = (int)it.npix;
    const int64_t base = (int64_t)l.b * it.npix;
    const float2* xn = it.xnew + base;
    float2* eta = it.eta + (int64_t)l.b * 2 * it.npix;
    const float2* mu = it.mu + (int64_t)l.b * 2 * it.npix;
    float2 c[kVecPix], e0[kVecPix], e1[kVecPix], old[kVecPix];
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int pix = min(pix_of(l, j), npix - 1);
        const Nb n = neighbours(pix, it.nx, it.ny);
        c[j] = xn[pix];
        const float2 d0 = csub(xn[n.xp], c[j]), d1 = csub(xn[n.yp], c[j]);
        e0[j] = cadd(eta[pix], csub(d0, mu[pix]));
        e1[j] = cadd(eta[pix + it.npix], csub(d1, mu[pix + it.npix]));
        old[j] = it.rho[base + pix];
    }
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int pix = pix_of(l, j);
        if (pix >= npix) break;
        eta[pix] = e0[j];
        eta[pix + it.npix] = e1[j];
        num += cnorm2(csub(c[j], old[j]));
        den += cnorm2(old[j]);
        it.rho[base + pix] = c[j];
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
    const Loc l = locate(tab);
    const SolveItem& it = tab.it[l.item];
#pragma unroll
    for (int j = 0; j < kVecPix; ++j) {
        const int pix = pix_of(l, j);
        if (pix >= (int)it.npix) break;
        const int64_t o = (int64_t)l.b * it.npix + pix;
        it.x_out[o] = it.rho[o];
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
