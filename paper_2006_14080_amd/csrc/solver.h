// ADMM / CG state and the vector-kernel launch interface (internal).
#pragma once

#include "internal.h"

namespace mri {

// Per-slice solver scalars, resident in device memory for the whole solve.
// Every decision of Alg. 2 and Alg. 4 (tolerances, breakdown, iteration
// counts) is taken on the device from these, so a solve never waits on the host.
struct SolveScalars {
    double tau;          // r^H r of the current CG residual
    double alpha_cg;     // tau / Re(d^H A d) of the current CG step
    double beta_cg;      // tau' / tau
    double pap;          // Re(d^H A d)
    double alpha_admm;   // ||rho' - rho||^2 / ||rho||^2
    int32_t admm_active; // 1 while ADMM iterates (cleared by the stopping rule)
    int32_t cg_active;   // 1 while the current CG solve iterates (implies admm_active)
    int32_t admm_iters;
    int32_t cg_steps;
    int32_t status;      // MRI_OK or MRI_ENUMERIC
    int32_t cg_it;       // CG steps taken in the current ADMM iteration
    int32_t pad;
};

// One solve (nb slices of one shape) as seen by the vector kernels.
struct SolveItem {
    int32_t nx, ny, nb, nblk;       // nblk: vector blocks (tiles) per slice
    int32_t block_begin;            // first block of this item in a grouped launch
    int32_t ksplit;                 // partial images per slice from the adjoint
    int64_t npix;
    const float2* x0;               // [nb][npix] or NULL
    float2 *rho, *rho0, *xnew, *b, *r, *p, *q, *fhd, *part;   // [nb][npix] ([ksplit][nb][npix] for part)
    float2 *eta, *mu;               // [nb][2][npix]
    double* red;                    // [nb][2][nblk] reduction partials
    SolveScalars* sc;               // [nb]
    float2* x_out;                  // [nb][npix]
    mri_admm_stats* stats;          // [nb] or NULL
    float thr;                      // lambda / beta
    float half_beta;                // beta / 2
    double atol2, rtol2;
    int32_t warm;
    int32_t cg_max;                 // CG steps per ADMM iteration (Alg. 2 max_iterations)
    int32_t admm_max;               // ADMM iterations (Alg. 4 max_iterations)
    int32_t slice_begin;            // first slice of this item in a grouped launch
};

struct SolveTable {
    int32_t nitems;
    int32_t total_blocks;
    int32_t total_slices;
    SolveItem it[kMaxItems];
};

// Vector-kernel tiles: a block of kVecThreads threads covers kTileX columns x
// kTileY rows of one slice; each thread one column and kVecRows rows.
constexpr int kVecThreads = 256;
constexpr int kTileX = 64;
constexpr int kVecRows = 4;
constexpr int kTileY = (kVecThreads / kTileX) * kVecRows;   // 16
__host__ __device__ inline int vec_tiles(int nx, int ny) {
    return ((nx + kTileX - 1) / kTileX) * ((ny + kTileY - 1) / kTileY);
}

enum FinishMode { kFinishFhd = 0, kFinishCgInit = 1, kFinishCgStep = 2 };
enum FinalizeMode { kFinCgInit = 0, kFinCgStep = 1, kFinCgUpdate = 2, kFinDual = 3 };

hipError_t launch_solve_init(const SolveTable& t, hipStream_t s);
hipError_t launch_mu(const SolveTable& t, hipStream_t s);
hipError_t launch_rhs(const SolveTable& t, hipStream_t s);
hipError_t launch_adj_finish(const SolveTable& t, int mode, hipStream_t s);
hipError_t launch_cg_update(const SolveTable& t, hipStream_t s);
hipError_t launch_cg_dir(const SolveTable& t, hipStream_t s);
hipError_t launch_dual(const SolveTable& t, hipStream_t s);
hipError_t launch_finalize(const SolveTable& t, int mode, hipStream_t s);
hipError_t launch_solve_final(const SolveTable& t, hipStream_t s);

hipError_t launch_sum_partials(const float2* part, int ksplit, int64_t n, float2* out, hipStream_t s);
hipError_t launch_tv_forward(int nx, int ny, int nb, const float2* x, float2* g, hipStream_t s);
hipError_t launch_tv_adjoint(int nx, int ny, int nb, const float2* g, float2* x, hipStream_t s);

}  // namespace mri
