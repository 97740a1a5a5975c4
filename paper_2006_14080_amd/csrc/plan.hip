// Launch plans for ADMM solves (see plan.h): workspace layout, grouped launch
// tables, and the kernel sequence of Alg. 4 with the CG of Alg. 2.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.h"

namespace mri {

int check_shape(const mri_shape* s) {
    if (!s) return MRI_EINVAL;
    if (s->nx < 1 || s->ny < 1 || s->nx > MRI_MAX_DIM || s->ny > MRI_MAX_DIM) return MRI_EINVAL;
    if (s->ncoils < 1 || s->ncoils > MRI_MAX_COILS) return MRI_EINVAL;
    if (s->nk < 1 || s->nk > (int64_t)1 << 30) return MRI_EINVAL;
    if (s->batch < 1 || s->batch > MRI_MAX_BATCH) return MRI_EINVAL;
    if ((s->traj_batched != 0 && s->traj_batched != 1) || (s->smaps_batched != 0 && s->smaps_batched != 1))
        return MRI_EINVAL;
    // grid sizes must fit a 1-D launch
    if (fwd_tiles(s->nx, s->ny, s->ncoils, s->nk, s->batch) > (int64_t)1 << 30) return MRI_ENOTSUP;
    return MRI_OK;
}

int check_precision(int p) {
    if (p == MRI_FP32) return MRI_OK;
    if (p == MRI_BF16X3 || p == MRI_FP16X3) return MRI_OK;
    return MRI_EINVAL;
}

int check_solve_precision(int p) {
    return p == MRI_NUFFT ? MRI_OK : check_precision(p);
}

int check_params(const mri_admm_params* p) {
    if (!p) return MRI_EINVAL;
    if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return MRI_EINVAL;
    if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return MRI_EINVAL;
    if (p->admm_iters < 0 || p->cg_iters < 0) return MRI_EINVAL;
    if (!(p->rtol >= 0.0) || !(p->atol >= 0.0)) return MRI_EINVAL;
    if (p->cg_warm_start != 0 && p->cg_warm_start != 1) return MRI_EINVAL;
    return check_solve_precision(p->precision);
}

size_t forward_ws(const mri_shape& s) {
    const size_t f32 = sizeof(float2) * (size_t)fwd_wimg_elems(s.nx, s.ny, s.ncoils, s.batch);
    const size_t bf = kSplitUnitBytes * (size_t)fwd_split_units(s.nx, s.ny, s.ncoils, s.batch) +
                      sizeof(float) * (size_t)fwd_rowscale_floats(s.ny, s.ncoils, s.batch);
    return ws_align(f32 > bf ? f32 : bf);
}

// Adjoint workspace: partial images and scale exponents, then the phase
// tables (one per trajectory).
size_t adjoint_tables_offset(const mri_shape& s) {
    int32_t ks, kp;
    adj_split(s.nx, s.ny, s.ncoils, s.nk, s.batch, MRI_FP32, &ks, &kp);
    return ws_align(sizeof(float2) * (size_t)adj_partial_elems(s.nx, s.ny, s.ncoils, s.batch, ks) +
                    sizeof(int32_t) * (size_t)s.batch * s.ncoils * ks);
}

size_t adjoint_ws(const mri_shape& s) {
    const int nbt = s.traj_batched ? s.batch : 1;
    return adjoint_tables_offset(s) + ws_align(sizeof(float2) * (size_t)adj_table_elems(s.nx, s.ny, s.nk, nbt));
}

void bind_adj_tables(NudftItem& it, const mri_shape& s, void* part) {
    it.ephx = reinterpret_cast<float2*>(static_cast<char*>(part) + adjoint_tables_offset(s));
    it.ephx_bs = s.traj_batched ? s.nk * s.nx : 0;
    it.ephy = it.ephx + (s.traj_batched ? s.batch : 1) * s.nk * s.nx;
    it.ephy_bs = s.traj_batched ? s.nk * s.ny : 0;
}

// The NUFFT parameters of the MRI_NUFFT solve mode.
mri_nufft_params solve_nufft_params() {
    mri_nufft_params p;
    p.width = 6;
    p.pad = 0;
    p.sigma = 2.0;
    return p;
}

AdmmLayout admm_layout(const mri_shape& s, int precision) {
    AdmmLayout L;
    std::memset(&L, 0, sizeof(L));
    const int64_t npix = (int64_t)s.nx * s.ny;
    const size_t vec = ws_align(sizeof(float2) * npix * s.batch);
    const bool nufft = precision == MRI_NUFFT;
    NufftLayout nl;
    if (nufft) {
        if (nufft_layout(s, solve_nufft_params(), &nl) != MRI_OK) return L;   // total 0: unsupported
        L.ksplit = 1;
        L.kper = (int32_t)s.nk;
        L.nplanes = 1;
    } else {
        adj_split(s.nx, s.ny, s.ncoils, s.nk, s.batch, precision, &L.ksplit, &L.kper);
        L.nplanes = adj_partial_planes(s.ncoils, L.ksplit);
    }
    L.nblk = (int32_t)vec_tiles(s.nx, s.ny);
    size_t o = 0;
    L.rho = o;  o += vec;
    L.rho0 = o; o += vec;
    L.xnew = o; o += vec;
    L.b = o;    o += vec;
    L.r = o;    o += vec;
    L.p = o;    o += vec;
    L.q = o;    o += vec;
    L.fhd = o;  o += vec;
    L.eta = o;  o += 2 * vec;
    L.mu = o;   o += 2 * vec;
    L.dtmp = o; o += ws_align(sizeof(float2) * (size_t)s.ncoils * s.nk * s.batch);
    if (nufft) {
        L.part = o;  o += vec;
        L.nufft = o; o += ws_align(nl.total);
    } else {
        L.wimg = o; o += forward_ws(s);
        L.part = o; o += adjoint_ws(s);
    }
    L.red = o;  o += ws_align(sizeof(double) * 2 * (size_t)L.nblk * s.batch);
    L.sc = o;   o += ws_align(sizeof(SolveScalars) * (size_t)s.batch);
    L.total = o;
    return L;
}

namespace {

template <class T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

void append(NudftTable& t, const NudftItem& it, int64_t ntiles, int64_t cw_elems) {
    NudftItem& d = t.it[t.nitems++];
    d = it;
    d.tile_begin = t.total_tiles;
    d.ntiles = (int32_t)ntiles;
    d.cw_begin = t.cw_total;
    t.total_tiles += (int32_t)ntiles;
    t.cw_total += cw_elems;
}

}  // namespace

int build_plan(const SolveBinding* bind, int n, int precision, Plan* out) {
    if (n < 1 || n > kMaxItems) return MRI_EINVAL;
    if (precision == MRI_NUFFT && n != 1) return MRI_ENOTSUP;    // the NUFFT mode plans one problem
    for (int i = 0; i < n; ++i)
        if ((int64_t)bind[i].shape.nx * bind[i].shape.ny >= ((int64_t)1 << 31)) return MRI_ENOTSUP;
    Plan& P = *out;
    std::memset(&P, 0, sizeof(P));
    P.precision = precision;
    int64_t blocks = 0, tiles_f = 0, tiles_a = 0;
    int32_t slices = 0;
    for (int i = 0; i < n; ++i) {
        const SolveBinding& B = bind[i];
        const mri_shape& sh = B.shape;
        const mri_admm_params& prm = B.params;
        const AdmmLayout L = admm_layout(sh, precision);
        if (L.total == 0) return MRI_ENOTSUP;
        const int64_t npix = (int64_t)sh.nx * sh.ny;
        void* ws = B.ws;

        SolveItem& si = P.st.it[i];
        si.nx = sh.nx;
        si.ny = sh.ny;
        si.nb = sh.batch;
        si.nblk = L.nblk;
        si.block_begin = (int32_t)blocks;
        si.ksplit = L.nplanes;
        si.npix = npix;
        si.x0 = B.x0;
        si.rho = at<float2>(ws, L.rho);
        si.rho0 = at<float2>(ws, L.rho0);
        si.xnew = at<float2>(ws, L.xnew);
        si.b = at<float2>(ws, L.b);
        si.r = at<float2>(ws, L.r);
        si.p = at<float2>(ws, L.p);
        si.q = at<float2>(ws, L.q);
        si.fhd = at<float2>(ws, L.fhd);
        si.eta = at<float2>(ws, L.eta);
        si.mu = at<float2>(ws, L.mu);
        si.part = at<float2>(ws, L.part);
        si.red = at<double>(ws, L.red);
        si.sc = at<SolveScalars>(ws, L.sc);
        si.x_out = B.x_out;
        si.stats = B.stats;
        si.thr = (float)(prm.lambda / prm.beta);
        si.half_beta = (float)(0.5 * prm.beta);
        si.atol2 = prm.atol * prm.atol;
        si.rtol2 = prm.rtol * prm.rtol;
        si.warm = prm.cg_warm_start;
        si.cg_max = prm.cg_iters;
        si.admm_max = prm.admm_iters;
        si.slice_begin = slices;
        slices += sh.batch;
        blocks += (int64_t)L.nblk * sh.batch;
        P.max_cg = std::max(P.max_cg, (int)prm.cg_iters);

        NudftItem base;
        std::memset(&base, 0, sizeof(base));
        base.nx = sh.nx;
        base.ny = sh.ny;
        base.nc = sh.ncoils;
        base.nb = sh.batch;
        base.nk = sh.nk;
        base.traj = B.traj;
        base.traj_bs = sh.traj_batched ? 2 * sh.nk : 0;
        base.smaps = B.smaps;
        base.smaps_bs = sh.smaps_batched ? (int64_t)sh.ncoils * npix : 0;
        base.wimg = at<float2>(ws, L.wimg);
        base.part = si.part;
        base.ksplit = L.ksplit;
        base.kper = L.kper;
        bind_adj_tables(base, sh, at<char>(ws, L.part));
        base.active_stride = (int32_t)(sizeof(SolveScalars) / sizeof(int32_t));
        const int64_t ft = fwd_tiles(sh.nx, sh.ny, sh.ncoils, sh.nk, sh.batch);
        const int64_t at_ = adj_tiles(sh.nx, sh.ny, sh.ncoils, sh.batch, L.ksplit);
        const int64_t cw = fwd_wimg_elems(sh.nx, sh.ny, sh.ncoils, sh.batch);
        if (cw >= ((int64_t)1 << 31) || fwd_split_units(sh.nx, sh.ny, sh.ncoils, sh.batch) >= ((int64_t)1 << 31))
            return MRI_ENOTSUP;     // 32-bit indexing inside an item
        tiles_f += ft;
        tiles_a += at_;

        NudftItem a_fhd = base;
        a_fhd.data = const_cast<float2*>(B.y);
        a_fhd.active = nullptr;
        NudftItem f_init = base;
        f_init.img = prm.cg_warm_start ? si.rho : si.rho0;
        f_init.data = at<float2>(ws, L.dtmp);
        f_init.active = &si.sc[0].admm_active;
        NudftItem f_step = base;
        f_step.img = si.p;
        f_step.data = at<float2>(ws, L.dtmp);
        f_step.active = &si.sc[0].cg_active;
        append(P.afhd, a_fhd, at_, 0);
        append(P.finit, f_init, ft, cw);
        append(P.ainit, f_init, at_, 0);
        append(P.fstep, f_step, ft, cw);
        append(P.astep, f_step, at_, 0);
        if (precision == MRI_NUFFT) {
            P.nufft = true;
            if (nufft_layout(sh, solve_nufft_params(), &P.nl) != MRI_OK) return MRI_ENOTSUP;
            P.np = nufft_ptrs(P.nl, at<char>(ws, L.nufft));
            P.traj = B.traj;
            P.smaps = B.smaps;
            P.smaps_bs = base.smaps_bs;
            P.y = B.y;
            P.dtmp = at<float2>(ws, L.dtmp);
            P.part = si.part;
            P.src_init = f_init.img;
            P.src_step = si.p;
        }
    }
    if (blocks > (int64_t)1 << 30 || tiles_f > (int64_t)1 << 30 || tiles_a > (int64_t)1 << 30)
        return MRI_ENOTSUP;
    P.st.nitems = n;
    P.st.total_blocks = (int32_t)blocks;
    P.st.total_slices = slices;
    return MRI_OK;
}

#define PLAN_TRY(call)                         \
    do {                                       \
        hipError_t e_ = (call);                \
        if (e_ != hipSuccess) return e_;       \
    } while (0)

// F^H F applied to src: the adjoint's output lands in the partial-image
// plane(s) that k_adj_finish sums.
hipError_t enqueue_normal(const Plan& p, const NudftTable& f, const NudftTable& a, const float2* src,
                          hipStream_t s) {
    if (p.nufft) {
        PLAN_TRY(launch_nufft_forward(p.nl, p.np, src, p.smaps, p.smaps_bs, p.dtmp, s));
        return launch_nufft_adjoint(p.nl, p.np, p.dtmp, p.smaps, p.smaps_bs, p.part, s);
    }
    PLAN_TRY(launch_coil_weight(f, p.precision, s));
    PLAN_TRY(launch_nudft_forward(f, p.precision, s));
    return launch_nudft_adjoint(a, p.precision, s);
}

hipError_t enqueue_init(const Plan& p, hipStream_t s) {
    if (p.nufft) {
        PLAN_TRY(launch_nufft_prepare(p.nl, p.np, p.traj, s));      // the trajectory is fixed for the solve
        PLAN_TRY(launch_solve_init(p.st, s));
        PLAN_TRY(launch_nufft_adjoint(p.nl, p.np, p.y, p.smaps, p.smaps_bs, p.part, s));
    } else {
        PLAN_TRY(launch_adj_phases(p.afhd, s));                     // the trajectory is fixed for the solve
        PLAN_TRY(launch_solve_init(p.st, s));
        PLAN_TRY(launch_nudft_adjoint(p.afhd, p.precision, s));
    }
    PLAN_TRY(launch_adj_finish(p.st, kFinishFhd, s));
    return hipSuccess;
}

hipError_t enqueue_iteration(const Plan& p, hipStream_t s) {
    PLAN_TRY(launch_mu(p.st, s));
    PLAN_TRY(launch_rhs(p.st, s));
    PLAN_TRY(enqueue_normal(p, p.finit, p.ainit, p.src_init, s));
    PLAN_TRY(launch_adj_finish(p.st, kFinishCgInit, s));
    PLAN_TRY(launch_finalize(p.st, kFinCgInit, s));
    for (int j = 0; j < p.max_cg; ++j) {
        PLAN_TRY(enqueue_normal(p, p.fstep, p.astep, p.src_step, s));
        PLAN_TRY(launch_adj_finish(p.st, kFinishCgStep, s));
        PLAN_TRY(launch_finalize(p.st, kFinCgStep, s));
        PLAN_TRY(launch_cg_update(p.st, s));
        PLAN_TRY(launch_finalize(p.st, kFinCgUpdate, s));
        PLAN_TRY(launch_cg_dir(p.st, s));
    }
    PLAN_TRY(launch_dual(p.st, s));
    PLAN_TRY(launch_finalize(p.st, kFinDual, s));
    return hipSuccess;
}

hipError_t enqueue_final(const Plan& p, hipStream_t s) {
    return launch_solve_final(p.st, s);
}

}  // namespace mri
