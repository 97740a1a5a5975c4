// Request server: continuous batching of ADMM-TV reconstructions on one GPU.
//
// One device pool (allocated once), a FIFO of submitted requests, and up to
// kMaxItems running slots.  Each step admits what fits, runs one ADMM
// iteration for every slot as grouped launches replayed from a HIP graph
// (re-captured when the slot set changes), then retires finished slots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "plan.h"

namespace mri {
namespace {

// First-fit allocator over [0, size) with coalescing of free ranges.
class PoolAllocator {
public:
    explicit PoolAllocator(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = ws_align(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = ws_align(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;
};

// Byte layout of one request inside the pool.
struct ReqLayout {
    size_t smaps, traj, y, x0, out, stats, ws, total;
};

ReqLayout req_layout(const mri_shape& s, int precision, bool has_x0) {
    ReqLayout L;
    const size_t npix = (size_t)s.nx * s.ny;
    size_t o = 0;
    L.smaps = o; o += ws_align(sizeof(float2) * s.ncoils * npix);
    L.traj = o;  o += ws_align(sizeof(double) * 2 * (size_t)s.nk);
    L.y = o;     o += ws_align(sizeof(float2) * s.ncoils * (size_t)s.nk);
    L.x0 = o;    o += has_x0 ? ws_align(sizeof(float2) * npix) : 0;
    L.out = o;   o += ws_align(sizeof(float2) * npix);
    L.stats = o; o += ws_align(sizeof(mri_admm_stats));
    L.ws = o;    o += admm_layout(s, precision).total;
    L.total = o;
    return L;
}

struct Request {
    uint64_t id;
    mri_shape shape;
    mri_admm_params params;
    std::vector<mri_c32> smaps, y, x0;
    std::vector<double> traj;
};

struct Slot {
    bool used = false;
    uint64_t id = 0;
    size_t off = 0, bytes = 0;
    ReqLayout L{};
    SolveBinding bind{};
};

struct Result {
    std::vector<mri_c32> image;
    mri_admm_stats stats;
};

struct Server {
    int precision = MRI_FP32;
    int max_slots = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;               // created here (the caller passed none)
    char* pool = nullptr;
    PoolAllocator* alloc = nullptr;
    SolveScalars* host_sc = nullptr;       // pinned readback of per-slot scalars
    std::deque<Request> queue;
    Slot slots[kMaxItems];
    std::unordered_map<uint64_t, Result> done;
    uint64_t next_id = 1;
    hipGraphExec_t graph = nullptr;
    bool graph_valid = false;
    int64_t steps = 0, captures = 0;
    int32_t completed = 0, cancelled = 0;
    std::string last_error;
};

int hip_err(Server* S, hipError_t e) {
    S->last_error = hipGetErrorString(e);
    return MRI_EHIP;
}

#define SRV_HIP(S, call)                           \
    do {                                           \
        hipError_t e_ = (call);                    \
        if (e_ != hipSuccess) return hip_err(S, e_); \
    } while (0)

int active_bindings(Server* S, SolveBinding* out, int* idx) {
    int n = 0;
    for (int i = 0; i < S->max_slots; ++i)
        if (S->slots[i].used) {
            out[n] = S->slots[i].bind;
            idx[n] = i;
            ++n;
        }
    return n;
}

void free_slot(Server* S, int i) {
    Slot& sl = S->slots[i];
    S->alloc->release(sl.off, sl.bytes);
    sl = Slot();
    S->graph_valid = false;
}

// Admit queued requests in FIFO order while a slot and pool memory are free.
int admit(Server* S, SolveBinding* fresh, int* nfresh) {
    *nfresh = 0;
    while (!S->queue.empty()) {
        int free_i = -1;
        for (int i = 0; i < S->max_slots; ++i)
            if (!S->slots[i].used) {
                free_i = i;
                break;
            }
        if (free_i < 0) break;
        Request& r = S->queue.front();
        const ReqLayout L = req_layout(r.shape, S->precision, !r.x0.empty());
        size_t off;
        if (!S->alloc->alloc(L.total, &off)) break;   // strict FIFO: the head waits for memory
        Slot& sl = S->slots[free_i];
        sl.used = true;
        sl.id = r.id;
        sl.off = off;
        sl.bytes = L.total;
        sl.L = L;
        char* base = S->pool + off;
        SRV_HIP(S, hipMemcpyAsync(base + L.smaps, r.smaps.data(), r.smaps.size() * sizeof(mri_c32),
                                  hipMemcpyHostToDevice, S->stream));
        SRV_HIP(S, hipMemcpyAsync(base + L.traj, r.traj.data(), r.traj.size() * sizeof(double),
                                  hipMemcpyHostToDevice, S->stream));
        SRV_HIP(S, hipMemcpyAsync(base + L.y, r.y.data(), r.y.size() * sizeof(mri_c32),
                                  hipMemcpyHostToDevice, S->stream));
        if (!r.x0.empty())
            SRV_HIP(S, hipMemcpyAsync(base + L.x0, r.x0.data(), r.x0.size() * sizeof(mri_c32),
                                      hipMemcpyHostToDevice, S->stream));
        SRV_HIP(S, hipStreamSynchronize(S->stream));   // the host copies are released below
        SolveBinding& b = sl.bind;
        b.shape = r.shape;
        b.smaps = reinterpret_cast<const float2*>(base + L.smaps);
        b.traj = reinterpret_cast<const double*>(base + L.traj);
        b.y = reinterpret_cast<const float2*>(base + L.y);
        b.x0 = r.x0.empty() ? nullptr : reinterpret_cast<const float2*>(base + L.x0);
        b.x_out = reinterpret_cast<float2*>(base + L.out);
        b.stats = reinterpret_cast<mri_admm_stats*>(base + L.stats);
        b.params = r.params;
        b.ws = base + L.ws;
        fresh[(*nfresh)++] = b;
        S->queue.pop_front();
        S->graph_valid = false;
    }
    return MRI_OK;
}

int capture_iteration(Server* S) {
    SolveBinding b[kMaxItems];
    int idx[kMaxItems];
    const int n = active_bindings(S, b, idx);
    if (S->graph) {
        hipGraphExecDestroy(S->graph);
        S->graph = nullptr;
    }
    if (n == 0) {
        S->graph_valid = true;
        return MRI_OK;
    }
    Plan plan;
    int rc = build_plan(b, n, S->precision, &plan);
    if (rc) return rc;
    hipGraph_t g;
    SRV_HIP(S, hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal));
    const hipError_t e = enqueue_iteration(plan, S->stream);
    const hipError_t e2 = hipStreamEndCapture(S->stream, &g);
    if (e != hipSuccess) return hip_err(S, e);
    if (e2 != hipSuccess) return hip_err(S, e2);
    const hipError_t e3 = hipGraphInstantiate(&S->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e3 != hipSuccess) return hip_err(S, e3);
    S->graph_valid = true;
    S->captures += 1;
    return MRI_OK;
}

}  // namespace
}  // namespace mri

using namespace mri;

extern "C" {

size_t mri_server_request_bytes(const mri_shape* shape, int precision) {
    if (check_shape(shape) != MRI_OK || shape->batch != 1) return 0;
    return req_layout(*shape, precision, true).total;
}

int mri_server_create(size_t hbm_budget, int max_slots, int precision, void* stream, void** srv) {
    if (!srv || max_slots < 1 || max_slots > kMaxItems || hbm_budget < kWsAlign) return MRI_EINVAL;
    if (precision == MRI_NUFFT) return MRI_ENOTSUP;
    int rc = check_precision(precision);
    if (rc) return rc;
    Server* S = new (std::nothrow) Server();
    if (!S) return MRI_ENOMEM;
    S->precision = precision;
    S->max_slots = max_slots;
    hbm_budget = hbm_budget / kWsAlign * kWsAlign;
    if (hipMalloc(reinterpret_cast<void**>(&S->pool), hbm_budget) != hipSuccess) {
        (void)hipGetLastError();
        delete S;
        return MRI_ENOMEM;
    }
    // The caller's stream if it gave one; the legacy default stream cannot be
    // captured into a graph, so without one the server makes its own.
    S->stream = static_cast<hipStream_t>(stream);
    S->own_stream = S->stream == nullptr;
    if ((S->own_stream && hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) ||
        hipHostMalloc(reinterpret_cast<void**>(&S->host_sc), sizeof(SolveScalars) * kMaxItems,
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(S->pool);
        if (S->own_stream && S->stream) (void)hipStreamDestroy(S->stream);
        delete S;
        return MRI_EHIP;
    }
    S->alloc = new PoolAllocator(hbm_budget);
    *srv = S;
    return MRI_OK;
}

int mri_server_submit(void* srv, const mri_request* req, uint64_t* id) {
    Server* S = static_cast<Server*>(srv);
    if (!S || !req || !id) return MRI_EINVAL;
    int rc = check_shape(&req->shape);
    if (rc) return rc;
    if (req->shape.batch != 1 || req->shape.traj_batched || req->shape.smaps_batched) return MRI_EINVAL;
    if ((rc = check_params(&req->params))) return rc;
    if (req->params.precision != S->precision) return MRI_EINVAL;
    if (!req->smaps || !req->traj || !req->y) return MRI_EINVAL;
    const mri_shape& sh = req->shape;
    if (req_layout(sh, S->precision, req->x0 != nullptr).total > S->alloc->size()) return MRI_ENOMEM;
    Request r;
    r.id = S->next_id++;
    r.shape = sh;
    r.params = req->params;
    const size_t npix = (size_t)sh.nx * sh.ny;
    r.smaps.assign(req->smaps, req->smaps + sh.ncoils * npix);
    r.traj.assign(req->traj, req->traj + 2 * (size_t)sh.nk);
    r.y.assign(req->y, req->y + sh.ncoils * (size_t)sh.nk);
    if (req->x0) r.x0.assign(req->x0, req->x0 + npix);
    *id = r.id;
    S->queue.push_back(std::move(r));
    return MRI_OK;
}

int mri_server_step(void* srv, int* n_active) {
    Server* S = static_cast<Server*>(srv);
    if (!S) return MRI_EINVAL;
    if (n_active) *n_active = 0;
    SolveBinding fresh[kMaxItems];
    int nfresh = 0;
    int rc = admit(S, fresh, &nfresh);
    if (rc) return rc;
    if (nfresh > 0) {   // F^H y, initial image and scalars of the new slots
        Plan p;
        if ((rc = build_plan(fresh, nfresh, S->precision, &p))) return rc;
        SRV_HIP(S, enqueue_init(p, S->stream));
    }
    SolveBinding b[kMaxItems];
    int idx[kMaxItems];
    const int n = active_bindings(S, b, idx);
    if (n == 0) return MRI_OK;
    if (!S->graph_valid && (rc = capture_iteration(S))) return rc;
    SRV_HIP(S, hipGraphLaunch(S->graph, S->stream));
    for (int k = 0; k < n; ++k) {
        const AdmmLayout L = admm_layout(b[k].shape, S->precision);
        SRV_HIP(S, hipMemcpyAsync(&S->host_sc[k], static_cast<char*>(b[k].ws) + L.sc, sizeof(SolveScalars),
                                  hipMemcpyDeviceToHost, S->stream));
    }
    SRV_HIP(S, hipStreamSynchronize(S->stream));
    S->steps += 1;
    if (n_active) *n_active = n;

    // Retire slots whose stopping rule fired (iteration cap, tolerance or a
    // non-finite value): write x_out / stats, copy them to the host, free.
    SolveBinding fin[kMaxItems];
    int fin_idx[kMaxItems], nfin = 0;
    for (int k = 0; k < n; ++k)
        if (!S->host_sc[k].admm_active) {
            fin[nfin] = b[k];
            fin_idx[nfin++] = idx[k];
        }
    if (nfin > 0) {
        Plan p;
        if ((rc = build_plan(fin, nfin, S->precision, &p))) return rc;
        SRV_HIP(S, enqueue_final(p, S->stream));
        for (int k = 0; k < nfin; ++k) {
            Slot& sl = S->slots[fin_idx[k]];
            Result res;
            res.image.resize((size_t)sl.bind.shape.nx * sl.bind.shape.ny);
            SRV_HIP(S, hipMemcpyAsync(res.image.data(), sl.bind.x_out, res.image.size() * sizeof(mri_c32),
                                      hipMemcpyDeviceToHost, S->stream));
            SRV_HIP(S, hipMemcpyAsync(&res.stats, sl.bind.stats, sizeof(mri_admm_stats), hipMemcpyDeviceToHost,
                                      S->stream));
            SRV_HIP(S, hipStreamSynchronize(S->stream));
            S->done.emplace(sl.id, std::move(res));
            S->completed += 1;
            free_slot(S, fin_idx[k]);
        }
    }
    return MRI_OK;
}

int mri_server_poll(void* srv, uint64_t id, mri_c32* out_image, mri_admm_stats* stats, int* state) {
    Server* S = static_cast<Server*>(srv);
    if (!S || !state) return MRI_EINVAL;
    auto it = S->done.find(id);
    if (it != S->done.end()) {
        *state = MRI_REQ_DONE;
        if (out_image) {
            std::memcpy(out_image, it->second.image.data(), it->second.image.size() * sizeof(mri_c32));
            if (stats) *stats = it->second.stats;
            S->done.erase(it);
        }
        return MRI_OK;
    }
    for (int i = 0; i < S->max_slots; ++i)
        if (S->slots[i].used && S->slots[i].id == id) {
            *state = MRI_REQ_RUNNING;
            return MRI_OK;
        }
    for (const Request& r : S->queue)
        if (r.id == id) {
            *state = MRI_REQ_QUEUED;
            return MRI_OK;
        }
    *state = MRI_REQ_UNKNOWN;
    return MRI_OK;
}

int mri_server_cancel(void* srv, uint64_t id) {
    Server* S = static_cast<Server*>(srv);
    if (!S) return MRI_EINVAL;
    for (auto it = S->queue.begin(); it != S->queue.end(); ++it)
        if (it->id == id) {
            S->queue.erase(it);
            S->cancelled += 1;
            return MRI_OK;
        }
    for (int i = 0; i < S->max_slots; ++i)
        if (S->slots[i].used && S->slots[i].id == id) {
            // every step ends with the stream synchronised, so the slot is idle
            free_slot(S, i);
            S->cancelled += 1;
            return MRI_OK;
        }
    return S->done.erase(id) ? MRI_OK : MRI_EINVAL;
}

int mri_server_get_info(void* srv, mri_server_info* info) {
    Server* S = static_cast<Server*>(srv);
    if (!S || !info) return MRI_EINVAL;
    info->queued = (int32_t)S->queue.size();
    info->active = 0;
    for (int i = 0; i < S->max_slots; ++i) info->active += S->slots[i].used ? 1 : 0;
    info->completed = S->completed;
    info->cancelled = S->cancelled;
    info->steps = S->steps;
    info->graph_captures = S->captures;
    info->pool_bytes = S->alloc->size();
    info->pool_used = S->alloc->used();
    return MRI_OK;
}

int mri_server_destroy(void* srv) {
    Server* S = static_cast<Server*>(srv);
    if (!S) return MRI_EINVAL;
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    if (S->graph) (void)hipGraphExecDestroy(S->graph);
    if (S->pool) (void)hipFree(S->pool);
    if (S->host_sc) (void)hipHostFree(S->host_sc);
    if (S->own_stream && S->stream) (void)hipStreamDestroy(S->stream);
    delete S->alloc;
    delete S;
    return MRI_OK;
}

}  // extern "C"
