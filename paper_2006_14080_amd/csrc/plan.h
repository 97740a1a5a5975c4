// Launch plans for ADMM solves: one or more problems (each a batch of slices
// of one shape) bound to their workspaces, turned into the grouped launch
// tables of every kernel of Alg. 4.  admm_solve uses a plan of one problem;
// the request server (server.hip) a plan over its active slots.
#pragma once

#include "nufft.h"
#include "solver.h"

namespace mri {

constexpr size_t kWsAlign = 256;
inline size_t ws_align(size_t v) { return (v + kWsAlign - 1) / kWsAlign * kWsAlign; }

// Byte offsets of one solve's state inside its workspace.  With the NUFFT
// operator (MRI_NUFFT) `part` is one image per slice (the NUFFT adjoint's
// output) and `nufft` the operator's workspace; wimg and the dense adjoint's
// partial images and tables are absent.
struct AdmmLayout {
    size_t rho, rho0, xnew, b, r, p, q, fhd, eta, mu, dtmp, wimg, part, nufft, red, sc, total;
    int32_t ksplit, kper, nblk, nplanes;
};

// Argument checks shared by every entry point (MRI_OK or an MRI_E* code).
int check_shape(const mri_shape* s);
int check_precision(int p);        // the dense operators' forms (MRI_FP32, MRI_BF16X3, MRI_FP16X3)
int check_solve_precision(int p);  // those or MRI_NUFFT
int check_params(const mri_admm_params* p);

AdmmLayout admm_layout(const mri_shape& s, int precision);
size_t forward_ws(const mri_shape& s);
size_t adjoint_ws(const mri_shape& s);
// Point an item's adjoint phase tables into its adjoint workspace (part).
void bind_adj_tables(NudftItem& it, const mri_shape& s, void* part);

// One problem of a plan: inputs and outputs (device pointers) and workspace.
struct SolveBinding {
    mri_shape shape;
    const float2* smaps;
    const double* traj;
    const float2* y;
    const float2* x0;            // may be NULL
    float2* x_out;
    mri_admm_stats* stats;       // may be NULL
    mri_admm_params params;
    void* ws;                    // admm_layout(shape).total bytes
};

struct Plan {
    int precision;
    int max_cg;                  // CG step launches per ADMM iteration
    SolveTable st;
    NudftTable afhd;             // F^H y            (always runs)
    NudftTable finit, ainit;     // A rho at the CG start (gated by admm_active)
    NudftTable fstep, astep;     // A d per CG step      (gated by cg_active)
    // NUFFT operator (precision MRI_NUFFT, one problem): its layout and
    // workspace, the trajectory it is planned from, and the arrays each
    // application reads and writes.
    bool nufft;
    NufftLayout nl;
    NufftPtrs np;
    const double* traj;
    const float2* smaps;
    int64_t smaps_bs;
    const float2* y;             // k-space data
    float2* dtmp;                // forward output of an application of A
    float2* part;                // adjoint output (one image per slice)
    const float2* src_init;      // image A is applied to at the CG start (rho or rho0)
    const float2* src_step;      // CG direction
};

// Build the tables for n <= kMaxItems bindings (all of one precision).
int build_plan(const SolveBinding* b, int n, int precision, Plan* out);

hipError_t enqueue_init(const Plan& p, hipStream_t s);       // rho, eta, scalars; F^H y
hipError_t enqueue_iteration(const Plan& p, hipStream_t s);  // one ADMM iteration (eq. (6)-(8))
hipError_t enqueue_final(const Plan& p, hipStream_t s);      // x_out, stats

}  // namespace mri
