// NUFFT approximation of the multi-coil NUDFT (internal): Kaiser-Bessel
// gridding on an oversampled power-of-two grid, a radix-2 FFT, and
// deapodisation.  Workspace layout and launchers shared by the C ABI.
#pragma once

#include "internal.h"

namespace mri {

constexpr int kNufftBin = 16;          // grid points per bin side (spreading tiles)
constexpr int kNufftMaxGrid = 4096;    // largest grid side (one FFT signal in LDS)
constexpr int kNufftMaxWidth = 10;     // W + 1 <= 16 keeps a footprint within two bins per axis

// Geometry of one NUFFT shape (host and device).
struct NufftGeom {
    int32_t nx, ny, nc, nb, nbt;       // nbt: trajectories (1 shared or nb per slice)
    int64_t nk;
    int32_t w;                         // kernel width W in grid points (W + 1 weights per axis)
    int32_t gx, gy, lgx, lgy;          // grid sides (powers of two) and their logs
    int32_t nbx, nby;                  // bins per axis
    double betax, betay;               // Kaiser-Bessel shape per axis
    int64_t nkeys, nkeys_pow2;         // bin entries (4 per sample) and the sort length
};

// Byte offsets inside an NUFFT workspace.
struct NufftLayout {
    NufftGeom g;
    size_t wx, wy, mx, my, dx, dy, twx, twy, keys, bins, grid, total;
};

// MRI_OK and the layout, or an error for unsupported parameters.
int nufft_layout(const mri_shape& s, const mri_nufft_params& p, NufftLayout* out);

// Device pointers of a workspace.
struct NufftPtrs {
    float *wx, *wy;          // [nbt][nk][W+1] kernel weights of each sample's grid neighbours
    int32_t *mx, *my;        // [nbt][nk] first neighbour (grid index, mod G)
    float *dx, *dy;          // [nx], [ny] 1 / Psi at the pixel offsets (deapodisation)
    float2 *twx, *twy;       // [G/2] exp(-2 pi i m / G)
    uint64_t* keys;          // [nkeys_pow2] (bin << 32 | sample), sorted
    int32_t* bins;           // [nbt * nbins + 1] first entry of each bin
    float2* grid;            // [nb][nc][gy][gx]
};
NufftPtrs nufft_ptrs(const NufftLayout& L, void* ws);

hipError_t launch_nufft_prepare(const NufftLayout& L, const NufftPtrs& P, const double* traj, hipStream_t s);
hipError_t launch_nufft_forward(const NufftLayout& L, const NufftPtrs& P, const float2* x, const float2* smaps,
                                int64_t smaps_bs, float2* y, hipStream_t s);
hipError_t launch_nufft_adjoint(const NufftLayout& L, const NufftPtrs& P, const float2* y, const float2* smaps,
                                int64_t smaps_bs, float2* x, hipStream_t s);

}  // namespace mri
