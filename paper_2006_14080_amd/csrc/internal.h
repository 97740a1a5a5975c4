// Internal interfaces of libmriadmm shared between the kernel files and the
// host runtime.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mri_admm.h"

namespace mri {

constexpr int kMaxItems = 16;     // problems per grouped launch

// ---------------------------------------------------------------------------
// NUDFT launch tables.  One "item" is a problem of one shape with nb slices;
// a grouped launch covers up to kMaxItems items, each owning a contiguous
// range of tiles.  Tables travel by value as kernel arguments, so a launch
// needs no host-to-device copy and a captured graph keeps them.
// ---------------------------------------------------------------------------
struct NudftItem {
    int32_t nx, ny, nc, nb;
    int64_t nk;
    const double* traj;  int64_t traj_bs;    // doubles per slice, 0 = shared
    const float2* smaps; int64_t smaps_bs;   // complex per slice, 0 = shared
    const float2* img;                       // [nb][ny][nx]   forward input
    float2* wimg;                            // [nb][nc][ny][pitch] coil-weighted image (forward workspace)
    float2* data;                            // [nb][nc][nk]   forward output / adjoint input
    float2* part;                            // [ksplit * coil groups][nb][ny][nx] adjoint partial images
    const int32_t* active;                   // per-slice run flag (nullable): slice b runs iff
                                             // active[b * active_stride] != 0
    int32_t active_stride;
    int32_t ksplit;                          // adjoint: sample-range splits
    int32_t kper;                            // adjoint: samples per split (multiple of 8)
    // Adjoint phase tables (k_adj_phases, once per trajectory): exp(+i w_x,k x)
    // [nk][nx] and exp(+i w_y,k y) [nk][ny] (centred offsets), per slice when
    // the trajectory is per slice (stride 0 = shared).
    float2* ephx;  int64_t ephx_bs;
    float2* ephy;  int64_t ephy_bs;
    int32_t tile_begin;                      // first tile of this item
    int32_t ntiles;
    int64_t cw_begin;                        // first coil-weighting element of this item
};

struct NudftTable {
    int32_t nitems;
    int32_t total_tiles;
    int64_t cw_total;                        // coil-weighting elements over all items
    NudftItem it[kMaxItems];
};
static_assert(sizeof(NudftTable) <= 4096, "a NudftTable is passed as a kernel argument");

// Forward tiling: 64 samples per workgroup, rows = all y in chunks of 256.
constexpr int kFwdCols = 64;
// Adjoint tiling: 128 x columns, 32 y rows, all coils (in groups of 8) per tile.
constexpr int kAdjCols = 128;
constexpr int kAdjRows = 32;
constexpr int kAdjCoilGroup = 8;
constexpr int kKStep = 8;          // complex K values per pipeline stage

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t fwd_tiles(int nx, int ny, int nc, int64_t nk, int nb);
// Elements of the coil-weighted image the forward reads (rows padded to a K-step).
int64_t fwd_wimg_elems(int nx, int ny, int nc, int nb);
// Adjoint tiles (workgroups) per sample split: nb x 128-column x 32-row blocks.
int64_t adj_tiles_per_split(int nx, int ny, int nb);
// Workgroups of one adjoint launch for a problem: pixel tiles x coil groups x sample splits.
int64_t adj_tiles(int nx, int ny, int nc, int nb, int ksplit);
// Row tiles per wave of the forward (by ny) and of the adjoint (by coil count).
__host__ __device__ inline int fwd_nt(int ny) {
    const int npass = (ny + 255) / 256;
    const int nt = (ny + 64 * npass - 1) / (64 * npass);
    return nt < 2 ? 2 : nt;
}
// Rows of the forward's pre-split operand: whole passes of 2 * fwd_nt * 32.
__host__ __device__ inline int fwd_padded_rows(int ny) {
    const int prows = 2 * fwd_nt(ny) * 32;
    return (ny + prows - 1) / prows * prows;
}
// (slice, coil, K-step, row) units of the split (16-bit) pre-pass: the hi and
// lo chunks of both lane halves, 16 bytes each.
constexpr int kSplitUnitBytes = 64;
__host__ __device__ inline int64_t fwd_split_units(int nx, int ny, int nc, int nb) {
    return (int64_t)nb * nc * ((nx + kKStep - 1) / kKStep) * fwd_padded_rows(ny);
}
// Split-FP16 form: inverse row scales, float [nb][nc][padded rows], stored
// right after the units (16-byte aligned).
__host__ __device__ inline int64_t fwd_rowscale_floats(int ny, int nc, int nb) {
    return (int64_t)nb * nc * fwd_padded_rows(ny);
}
__host__ __device__ inline float* fwd_rowscale(float2* wimg, int nx, int ny, int nc, int nb) {
    return reinterpret_cast<float*>(reinterpret_cast<char*>(wimg) + kSplitUnitBytes * fwd_split_units(nx, ny, nc, nb));
}
// Row tiles per wave of the adjoint: coils run in even groups of 2 * adj_nt.
__host__ __device__ inline int adj_nt(int nc) {
    const int ngroups = (nc + kAdjCoilGroup - 1) / kAdjCoilGroup;
    const int gsz = (nc + ngroups - 1) / ngroups;
    const int nt = (gsz + 1) / 2;
    return nt < 2 ? 2 : nt;
}
// Partial images the adjoint writes per slice: one per (sample split, coil group).
// Coil groups of the adjoint (one per workgroup and partial image).
__host__ __device__ inline int adj_coil_groups(int nc) { return (nc + 2 * adj_nt(nc) - 1) / (2 * adj_nt(nc)); }
__host__ __device__ inline int adj_partial_planes(int nc, int ksplit) { return ksplit * adj_coil_groups(nc); }
// Adjoint workspace: the partial images [planes][nb][ny][nx], then (split-FP16
// form) one int32 scale exponent per (slice, coil, sample split).
__host__ __device__ inline int64_t adj_partial_elems(int nx, int ny, int nc, int nb, int ksplit) {
    return (int64_t)adj_partial_planes(nc, ksplit) * nb * nx * ny;
}
__host__ __device__ inline int32_t* adj_scale_exp(float2* part, int nx, int ny, int nc, int nb, int ksplit) {
    return reinterpret_cast<int32_t*>(part + adj_partial_elems(nx, ny, nc, nb, ksplit));
}
// Complex elements of the adjoint's phase tables (nbt trajectories).
__host__ __device__ inline int64_t adj_table_elems(int nx, int ny, int64_t nk, int nbt) {
    return (int64_t)nbt * nk * ((int64_t)nx + ny);
}
// Choose the sample-range split of the adjoint for one problem.
void adj_split(int nx, int ny, int nc, int64_t nk, int nb, int precision,
               int32_t* ksplit, int32_t* kper);

// Pre-pass of the forward for every item of t: wimg = smaps (.) img (FP32
// rows, or split operand chunks for MRI_BF16X3 / MRI_FP16X3).
hipError_t launch_coil_weight(const NudftTable& t, int precision, hipStream_t s);
hipError_t launch_nudft_forward(const NudftTable& t, int precision, hipStream_t s);
hipError_t launch_nudft_adjoint(const NudftTable& t, int precision, hipStream_t s);
// Fill the adjoint phase tables of every item of t (ephx, ephy).
hipError_t launch_adj_phases(const NudftTable& t, hipStream_t s);

}  // namespace mri
