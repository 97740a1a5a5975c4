// C ABI of libmriadmm (declared in include/mri_admm.h): argument checks,
// workspace planning, launch tables, and the ADMM / CG orchestration of
// Alg. 2 and Alg. 4 as a fixed sequence of kernels on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "solver.h"

namespace mri {
namespace {

thread_local std::string g_last_hip;

int hip_fail(hipError_t e) {
    g_last_hip = hipGetErrorString(e);
    return MRI_EHIP;
}

#define MRI_HIP(call)                              \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_fail(e_); \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

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
    if (p == MRI_BF16X3) return MRI_OK;
    return MRI_EINVAL;
}

int check_params(const mri_admm_params* p) {
    if (!p) return MRI_EINVAL;
    if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return MRI_EINVAL;
    if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return MRI_EINVAL;
    if (p->admm_iters < 0 || p->cg_iters < 0) return MRI_EINVAL;
    if (!(p->rtol >= 0.0) || !(p->atol >= 0.0)) return MRI_EINVAL;
    if (p->cg_warm_start != 0 && p->cg_warm_start != 1) return MRI_EINVAL;
    return check_precision(p->precision);
}

NudftItem base_item(const mri_shape& s, const float2* smaps, const double* traj) {
    NudftItem it;
    std::memset(&it, 0, sizeof(it));
    it.nx = s.nx;
    it.ny = s.ny;
    it.nc = s.ncoils;
    it.nb = s.batch;
    it.nk = s.nk;
    it.traj = traj;
    it.traj_bs = s.traj_batched ? 2 * s.nk : 0;
    it.smaps = smaps;
    it.smaps_bs = s.smaps_batched ? (int64_t)s.ncoils * s.nx * s.ny : 0;
    it.active_stride = 1;
    return it;
}

NudftTable single_table(const NudftItem& it, int64_t ntiles) {
    NudftTable t;
    std::memset(&t, 0, sizeof(t));
    t.nitems = 1;
    t.total_tiles = (int32_t)ntiles;
    t.it[0] = it;
    t.it[0].tile_begin = 0;
    t.it[0].ntiles = (int32_t)ntiles;
    return t;
}

size_t forward_ws(const mri_shape& s) {
    return align_up(sizeof(float2) * (size_t)fwd_wimg_elems(s.nx, s.ny, s.ncoils, s.batch));
}

size_t adjoint_ws(const mri_shape& s) {
    int32_t ks, kp;
    adj_split(s.nx, s.ny, s.ncoils, s.nk, s.batch, MRI_FP32, &ks, &kp);
    return align_up(sizeof(float2) * (size_t)s.nx * s.ny * s.batch * adj_partial_planes(s.ncoils, ks));
}

// ---- ADMM workspace ---------------------------------------------------------
struct AdmmLayout {
    size_t rho, rho0, xnew, b, r, p, q, fhd, eta, mu, dtmp, wimg, part, red, sc, total;
    int32_t ksplit, kper, nblk;
};

AdmmLayout admm_layout(const mri_shape& s, int precision) {
    AdmmLayout L;
    const int64_t npix = (int64_t)s.nx * s.ny;
    const size_t vec = align_up(sizeof(float2) * npix * s.batch);
    adj_split(s.nx, s.ny, s.ncoils, s.nk, s.batch, precision, &L.ksplit, &L.kper);
    L.nblk = (int32_t)ceil_div(npix, kVecThreads);
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
    L.dtmp = o; o += align_up(sizeof(float2) * (size_t)s.ncoils * s.nk * s.batch);
    L.wimg = o; o += forward_ws(s);
    L.part = o; o += adjoint_ws(s);
    L.red = o;  o += align_up(sizeof(double) * 2 * (size_t)L.nblk * s.batch);
    L.sc = o;   o += align_up(sizeof(SolveScalars) * (size_t)s.batch);
    L.total = o;
    return L;
}

template <class T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

}  // namespace
}  // namespace mri

using namespace mri;

extern "C" {

size_t mri_workspace_bytes(const mri_shape* shape, int op, const mri_admm_params* params) {
    if (check_shape(shape) != MRI_OK) return 0;
    switch (op) {
        case MRI_OP_FORWARD: return forward_ws(*shape);
        case MRI_OP_ADJOINT: return adjoint_ws(*shape);
        case MRI_OP_ADMM: return admm_layout(*shape, params ? params->precision : MRI_FP32).total;
        default: return 0;
    }
}

const char* mri_strerror(int code) {
    switch (code) {
        case MRI_OK: return "success";
        case MRI_EINVAL: return "invalid argument (null pointer, shape or parameter)";
        case MRI_ENOMEM: return "workspace too small or memory budget exceeded";
        case MRI_EHIP: return "HIP runtime error";
        case MRI_ENOTSUP: return "unsupported precision or shape";
        case MRI_ENUMERIC: return "non-finite value met during the solve";
        default: return "unknown error code";
    }
}

const char* mri_last_hip_error(void) { return g_last_hip.c_str(); }

int nudft_forward(const mri_shape* shape, const mri_c32* x, const mri_c32* smaps, const double* traj,
                  mri_c32* y, int precision, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if ((rc = check_precision(precision))) return rc;
    if (!x || !smaps || !traj || !y) return MRI_EINVAL;
    if (!ws || ws_bytes < forward_ws(*shape)) return MRI_ENOMEM;
    NudftItem it = base_item(*shape, reinterpret_cast<const float2*>(smaps), traj);
    it.img = reinterpret_cast<const float2*>(x);
    it.wimg = static_cast<float2*>(ws);
    it.data = reinterpret_cast<float2*>(y);
    const NudftTable t = single_table(it, fwd_tiles(shape->nx, shape->ny, shape->ncoils, shape->nk, shape->batch));
    hipStream_t s = static_cast<hipStream_t>(stream);
    MRI_HIP(launch_coil_weight(t, s));
    MRI_HIP(launch_nudft_forward(t, precision, s));
    return MRI_OK;
}

int nudft_adjoint(const mri_shape* shape, const mri_c32* y, const mri_c32* smaps, const double* traj,
                  mri_c32* x, int precision, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if ((rc = check_precision(precision))) return rc;
    if (!x || !smaps || !traj || !y) return MRI_EINVAL;
    const size_t need = adjoint_ws(*shape);
    if (!ws || ws_bytes < need) return MRI_ENOMEM;
    NudftItem it = base_item(*shape, reinterpret_cast<const float2*>(smaps), traj);
    it.data = const_cast<float2*>(reinterpret_cast<const float2*>(y));
    it.part = static_cast<float2*>(ws);
    adj_split(shape->nx, shape->ny, shape->ncoils, shape->nk, shape->batch, precision, &it.ksplit, &it.kper);
    const NudftTable t = single_table(it, adj_tiles_per_split(shape->nx, shape->ny, shape->batch) * it.ksplit);
    hipStream_t s = static_cast<hipStream_t>(stream);
    MRI_HIP(launch_nudft_adjoint(t, precision, s));
    MRI_HIP(launch_sum_partials(it.part, adj_partial_planes(shape->ncoils, it.ksplit),
                                (int64_t)shape->nx * shape->ny * shape->batch,
                                reinterpret_cast<float2*>(x), s));
    return MRI_OK;
}

int tv_forward(const mri_shape* shape, const mri_c32* x, mri_c32* g, void* stream) {
    if (!shape || !x || !g) return MRI_EINVAL;
    if (shape->nx < 1 || shape->ny < 1 || shape->batch < 1) return MRI_EINVAL;
    MRI_HIP(launch_tv_forward(shape->nx, shape->ny, shape->batch, reinterpret_cast<const float2*>(x),
                              reinterpret_cast<float2*>(g), static_cast<hipStream_t>(stream)));
    return MRI_OK;
}

int tv_adjoint(const mri_shape* shape, const mri_c32* g, mri_c32* x, void* stream) {
    if (!shape || !x || !g) return MRI_EINVAL;
    if (shape->nx < 1 || shape->ny < 1 || shape->batch < 1) return MRI_EINVAL;
    MRI_HIP(launch_tv_adjoint(shape->nx, shape->ny, shape->batch, reinterpret_cast<const float2*>(g),
                              reinterpret_cast<float2*>(x), static_cast<hipStream_t>(stream)));
    return MRI_OK;
}

int admm_solve(const mri_shape* shape, const mri_c32* smaps, const double* traj, const mri_c32* y,
               const mri_c32* x0, const mri_admm_params* params, mri_c32* x_out, mri_admm_stats* stats_dev,
               void* ws, size_t ws_bytes, void* stream) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if ((rc = check_params(params))) return rc;
    if (!smaps || !traj || !y || !x_out) return MRI_EINVAL;
    const mri_shape& sh = *shape;
    const AdmmLayout L = admm_layout(sh, params->precision);
    if (!ws || ws_bytes < L.total) return MRI_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int prec = params->precision;
    const int64_t npix = (int64_t)sh.nx * sh.ny;

    SolveTable st;
    std::memset(&st, 0, sizeof(st));
    st.nitems = 1;
    st.total_blocks = L.nblk * sh.batch;
    SolveItem& si = st.it[0];
    si.nx = sh.nx;
    si.ny = sh.ny;
    si.nb = sh.batch;
    si.nblk = L.nblk;
    si.block_begin = 0;
    si.ksplit = adj_partial_planes(sh.ncoils, L.ksplit);
    si.npix = npix;
    si.x0 = reinterpret_cast<const float2*>(x0);
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
    si.x_out = reinterpret_cast<float2*>(x_out);
    si.stats = stats_dev;
    si.thr = (float)(params->lambda / params->beta);
    si.half_beta = (float)(0.5 * params->beta);
    si.atol2 = params->atol * params->atol;
    si.rtol2 = params->rtol * params->rtol;
    si.warm = params->cg_warm_start;

    // NUDFT tables: F^H d (always), the CG start A rho (gated by admm_active),
    // and the CG step A d (gated by cg_active).
    const int32_t* admm_flag = &si.sc[0].admm_active;
    const int32_t* cg_flag = &si.sc[0].cg_active;
    const int32_t flag_stride = (int32_t)(sizeof(SolveScalars) / sizeof(int32_t));
    NudftItem base = base_item(sh, reinterpret_cast<const float2*>(smaps), traj);
    base.ksplit = L.ksplit;
    base.kper = L.kper;
    base.part = si.part;
    base.active_stride = flag_stride;
    base.wimg = at<float2>(ws, L.wimg);
    const int64_t ftiles = fwd_tiles(sh.nx, sh.ny, sh.ncoils, sh.nk, sh.batch);
    const int64_t atiles = adj_tiles_per_split(sh.nx, sh.ny, sh.batch) * L.ksplit;

    NudftItem a_fhd = base;
    a_fhd.data = const_cast<float2*>(reinterpret_cast<const float2*>(y));
    a_fhd.active = nullptr;
    NudftItem f_init = base;
    f_init.img = params->cg_warm_start ? si.rho : si.rho0;
    f_init.data = at<float2>(ws, L.dtmp);
    f_init.active = admm_flag;
    NudftItem a_init = f_init;
    NudftItem f_step = base;
    f_step.img = si.p;
    f_step.data = at<float2>(ws, L.dtmp);
    f_step.active = cg_flag;
    NudftItem a_step = f_step;
    const NudftTable T_afhd = single_table(a_fhd, atiles);
    const NudftTable T_finit = single_table(f_init, ftiles);
    const NudftTable T_ainit = single_table(a_init, atiles);
    const NudftTable T_fstep = single_table(f_step, ftiles);
    const NudftTable T_astep = single_table(a_step, atiles);

    MRI_HIP(launch_solve_init(st, s));
    if (params->admm_iters > 0) {
        MRI_HIP(launch_nudft_adjoint(T_afhd, prec, s));
        MRI_HIP(launch_adj_finish(st, kFinishFhd, s));
    }
    for (int m = 0; m < params->admm_iters; ++m) {
        MRI_HIP(launch_mu(st, s));
        MRI_HIP(launch_rhs(st, s));
        MRI_HIP(launch_coil_weight(T_finit, s));
        MRI_HIP(launch_nudft_forward(T_finit, prec, s));
        MRI_HIP(launch_nudft_adjoint(T_ainit, prec, s));
        MRI_HIP(launch_adj_finish(st, kFinishCgInit, s));
        for (int j = 0; j < params->cg_iters; ++j) {
            MRI_HIP(launch_coil_weight(T_fstep, s));
            MRI_HIP(launch_nudft_forward(T_fstep, prec, s));
            MRI_HIP(launch_nudft_adjoint(T_astep, prec, s));
            MRI_HIP(launch_adj_finish(st, kFinishCgStep, s));
            MRI_HIP(launch_cg_update(st, s));
            MRI_HIP(launch_cg_dir(st, s));
        }
        MRI_HIP(launch_dual(st, s));
    }
    MRI_HIP(launch_solve_final(st, s));
    return MRI_OK;
}

}  // extern "C"
