// C ABI of libmriadmm (declared in include/mri_admm.h): argument checks,
// workspace planning, launch tables, and the ADMM / CG orchestration of
// Alg. 2 and Alg. 4 as a fixed sequence of kernels on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "nufft.h"
#include "plan.h"

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

// Device scratch of nudft_forward_noalloc: the coil-weighted images live in
// this file-scope array instead of a caller workspace.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol); it uses the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Address of the current device's scratch array (nullptr on failure, with
// the HIP error in *err).
void* device_scratch(hipError_t* err) {
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
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

int mri_adjoint_split(const mri_shape* shape, int32_t* ksplit, int32_t* kper, int32_t* planes) {
    const int rc = check_shape(shape);
    if (rc) return rc;
    int32_t ks, kp;
    adj_split(shape->nx, shape->ny, shape->ncoils, shape->nk, shape->batch, MRI_FP32, &ks, &kp);
    if (ksplit) *ksplit = ks;
    if (kper) *kper = kp;
    if (planes) *planes = adj_partial_planes(shape->ncoils, ks);
    return MRI_OK;
}

size_t mri_nufft_workspace_bytes(const mri_shape* shape, const mri_nufft_params* params) {
    if (check_shape(shape) != MRI_OK || !params) return 0;
    NufftLayout L;
    if (nufft_layout(*shape, *params, &L) != MRI_OK) return 0;
    return L.total;
}

int nufft_prepare(const mri_shape* shape, const double* traj, const mri_nufft_params* params, void* ws,
                  size_t ws_bytes, void* stream) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if (!traj || !params) return MRI_EINVAL;
    NufftLayout L;
    if ((rc = nufft_layout(*shape, *params, &L))) return rc;
    if (!ws || ws_bytes < L.total) return MRI_ENOMEM;
    MRI_HIP(launch_nufft_prepare(L, nufft_ptrs(L, ws), traj, static_cast<hipStream_t>(stream)));
    return MRI_OK;
}

int nufft_forward(const mri_shape* shape, const mri_c32* x, const mri_c32* smaps, mri_c32* y,
                  const mri_nufft_params* params, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if (!x || !smaps || !y || !params) return MRI_EINVAL;
    NufftLayout L;
    if ((rc = nufft_layout(*shape, *params, &L))) return rc;
    if (!ws || ws_bytes < L.total) return MRI_ENOMEM;
    const int64_t sbs = shape->smaps_batched ? (int64_t)shape->ncoils * shape->nx * shape->ny : 0;
    MRI_HIP(launch_nufft_forward(L, nufft_ptrs(L, ws), reinterpret_cast<const float2*>(x),
                                 reinterpret_cast<const float2*>(smaps), sbs, reinterpret_cast<float2*>(y),
                                 static_cast<hipStream_t>(stream)));
    return MRI_OK;
}

int nufft_adjoint(const mri_shape* shape, const mri_c32* y, const mri_c32* smaps, mri_c32* x,
                  const mri_nufft_params* params, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if (!x || !smaps || !y || !params) return MRI_EINVAL;
    NufftLayout L;
    if ((rc = nufft_layout(*shape, *params, &L))) return rc;
    if (!ws || ws_bytes < L.total) return MRI_ENOMEM;
    const int64_t sbs = shape->smaps_batched ? (int64_t)shape->ncoils * shape->nx * shape->ny : 0;
    MRI_HIP(launch_nufft_adjoint(L, nufft_ptrs(L, ws), reinterpret_cast<const float2*>(y),
                                 reinterpret_cast<const float2*>(smaps), sbs, reinterpret_cast<float2*>(x),
                                 static_cast<hipStream_t>(stream)));
    return MRI_OK;
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
    if (fwd_wimg_elems(shape->nx, shape->ny, shape->ncoils, shape->batch) >= ((int64_t)1 << 31) ||
        fwd_split_units(shape->nx, shape->ny, shape->ncoils, shape->batch) >= ((int64_t)1 << 31))
        return MRI_ENOTSUP;
    if (!ws || ws_bytes < forward_ws(*shape)) return MRI_ENOMEM;
    NudftItem it = base_item(*shape, reinterpret_cast<const float2*>(smaps), traj);
    it.img = reinterpret_cast<const float2*>(x);
    it.wimg = static_cast<float2*>(ws);
    it.data = reinterpret_cast<float2*>(y);
    NudftTable t = single_table(it, fwd_tiles(shape->nx, shape->ny, shape->ncoils, shape->nk, shape->batch));
    t.cw_total = fwd_wimg_elems(shape->nx, shape->ny, shape->ncoils, shape->batch);
    hipStream_t s = static_cast<hipStream_t>(stream);
    MRI_HIP(launch_coil_weight(t, precision, s));
    MRI_HIP(launch_nudft_forward(t, precision, s));
    return MRI_OK;
}

int nudft_forward_noalloc(const mri_shape* shape, const mri_c32* x, const mri_c32* smaps, const double* traj,
                          mri_c32* y, int precision, void* stream) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if ((rc = check_precision(precision))) return rc;
    if (!x || !smaps || !traj || !y) return MRI_EINVAL;
    if (forward_ws(*shape) > kNoallocScratchBytes) return MRI_ENOMEM;
    hipError_t e = hipSuccess;
    void* ws = device_scratch(&e);
    if (!ws) return hip_fail(e);
    return nudft_forward(shape, x, smaps, traj, y, precision, ws, kNoallocScratchBytes, stream);
}

size_t mri_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

int nudft_adjoint_prepare(const mri_shape* shape, const double* traj, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if (!traj) return MRI_EINVAL;
    if (!ws || ws_bytes < adjoint_ws(*shape)) return MRI_ENOMEM;
    NudftItem it = base_item(*shape, nullptr, traj);
    bind_adj_tables(it, *shape, ws);
    const NudftTable t = single_table(it, 1);
    MRI_HIP(launch_adj_phases(t, static_cast<hipStream_t>(stream)));
    return MRI_OK;
}

int nudft_adjoint_prepared(const mri_shape* shape, const mri_c32* y, const mri_c32* smaps, const double* traj,
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
    bind_adj_tables(it, *shape, ws);
    const NudftTable t = single_table(it, adj_tiles(shape->nx, shape->ny, shape->ncoils, shape->batch, it.ksplit));
    hipStream_t s = static_cast<hipStream_t>(stream);
    MRI_HIP(launch_nudft_adjoint(t, precision, s));
    MRI_HIP(launch_sum_partials(it.part, adj_partial_planes(shape->ncoils, it.ksplit),
                                (int64_t)shape->nx * shape->ny * shape->batch,
                                reinterpret_cast<float2*>(x), s));
    return MRI_OK;
}

int nudft_adjoint(const mri_shape* shape, const mri_c32* y, const mri_c32* smaps, const double* traj,
                  mri_c32* x, int precision, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if ((rc = check_precision(precision))) return rc;
    if (!x || !smaps || !traj || !y) return MRI_EINVAL;
    if ((rc = nudft_adjoint_prepare(shape, traj, ws, ws_bytes, stream))) return rc;
    return nudft_adjoint_prepared(shape, y, smaps, traj, x, precision, ws, ws_bytes, stream);
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
    const AdmmLayout L = admm_layout(*shape, params->precision);
    if (!ws || ws_bytes < L.total) return MRI_ENOMEM;
    SolveBinding bind;
    bind.shape = *shape;
    bind.smaps = reinterpret_cast<const float2*>(smaps);
    bind.traj = traj;
    bind.y = reinterpret_cast<const float2*>(y);
    bind.x0 = reinterpret_cast<const float2*>(x0);
    bind.x_out = reinterpret_cast<float2*>(x_out);
    bind.stats = stats_dev;
    bind.params = *params;
    bind.ws = ws;
    Plan plan;
    if ((rc = build_plan(&bind, 1, params->precision, &plan))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    MRI_HIP(enqueue_init(plan, s));
    for (int m = 0; m < params->admm_iters; ++m) MRI_HIP(enqueue_iteration(plan, s));
    MRI_HIP(enqueue_final(plan, s));
    return MRI_OK;
}

}  // extern "C"
