// NUFFT approximation of the multi-coil NUDFT: the O(N log N) operator of
// the paper's comparison systems (Sec. VII, Table II), behind the same
// interface as the dense operators.
//
// Forward, per slice b and coil g (t = w G / (2 pi) a sample's position in
// grid units per axis, m its W + 1 nearest grid points, psi the Kaiser-Bessel
// kernel and Psi its Fourier transform):
//   v = s_g (.) x_b / Psi            (deapodised, zero-padded into the G grid)
//   U = FFT_G(v)                     (exp(-2 pi i m x / G), rows then columns)
//   y[b][g][k] = sum_m psi_x(t_x - m_x) psi_y(t_y - m_y) U[m_y][m_x]
// Adjoint: the exact conjugate transpose, grid points gathering the samples
// whose kernel reaches them (deterministic: each point sums its samples in
// sample order), the inverse FFT (exp(+2 pi i m x / G), unnormalised),
// crop, 1 / Psi, and sum_g conj(s_g).
//
// Preparation (once per trajectory): every sample's first grid neighbour and
// its W + 1 weights per axis (FP64 kernel evaluation, stored in FP32), the
// deapodisation, FFT twiddles, and for the spreading a list of (bin, sample)
// entries sorted by bin and sample (bitonic sort of unique 64-bit keys), so
// that each 16 x 16 tile of grid points reads exactly the samples that reach
// it, in sample order.
#include <cmath>
#include <cstring>

#include "device.h"
#include "nufft.h"

namespace mri {
namespace {

constexpr int kT = 256;                               // threads per block of the element-wise kernels
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr uint64_t kNoKey = ~(uint64_t)0;

// I0(z), the modified Bessel function of the first kind of order zero, from
// its power series sum_j (z^2 / 4)^j / (j!)^2 (all terms positive; converges
// to FP64 precision within 60 terms for z <= 40).
__device__ double bessel_i0(double z) {
    const double q = 0.25 * z * z;
    double term = 1.0, sum = 1.0;
    for (int j = 1; j < 60; ++j) {
        term *= q / ((double)j * (double)j);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

// The kernel psi(u) = I0(beta sqrt(1 - (2u/W)^2)) on |u| <= W/2, else 0.
__device__ double kb_psi(double u, int w, double beta) {
    const double r = 2.0 * u / (double)w;
    const double z = 1.0 - r * r;
    return z < 0.0 ? 0.0 : bessel_i0(beta * sqrt(z));
}

// Its Fourier transform Psi(f) = int psi(u) exp(2 pi i u f) du
//   = W sinh(sqrt(beta^2 - (pi W f)^2)) / sqrt(beta^2 - (pi W f)^2).
__device__ double kb_Psi(double f, int w, double beta) {
    const double pw = 3.14159265358979323846 * (double)w * f;
    const double a = beta * beta - pw * pw;
    if (a > 0.0) {
        const double r = sqrt(a);
        return (double)w * sinh(r) / r;
    }
    const double r = sqrt(-a);
    return r > 0.0 ? (double)w * sin(r) / r : (double)w;
}

// Per sample and axis: first neighbour m0 = ceil(t - W/2) (stored mod G) and
// the weights psi(t - m0 - i), i = 0..W; four (bin, sample) keys per sample
// (the up to 2 x 2 bins its footprint touches; repeats become kNoKey).
__global__ __launch_bounds__(kT) void k_nufft_samples(const NufftGeom g, const double* __restrict__ traj,
                                                      float* __restrict__ wx, float* __restrict__ wy,
                                                      int32_t* __restrict__ mx, int32_t* __restrict__ my,
                                                      uint64_t* __restrict__ keys) {
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= g.nkeys_pow2 / 4 && e >= (int64_t)g.nbt * g.nk) return;
    if (e >= (int64_t)g.nbt * g.nk) {                    // padding of the sort
        for (int q = 0; q < 4; ++q)
            if (4 * e + q < g.nkeys_pow2) keys[4 * e + q] = kNoKey;
        return;
    }
    const int bt = (int)(e / g.nk);
    const int64_t k = e - (int64_t)bt * g.nk;
    const int w = g.w;
    int m0x, m0y;
    {
        const double t = traj[2 * e] * (double)g.gx / kTwoPi;
        const double m0 = ceil(t - 0.5 * w);
        for (int i = 0; i <= w; ++i) wx[e * (w + 1) + i] = (float)kb_psi(t - (m0 + i), w, g.betax);
        m0x = (int)(((int64_t)m0 % g.gx + g.gx) % g.gx);
    }
    {
        const double t = traj[2 * e + 1] * (double)g.gy / kTwoPi;
        const double m0 = ceil(t - 0.5 * w);
        for (int i = 0; i <= w; ++i) wy[e * (w + 1) + i] = (float)kb_psi(t - (m0 + i), w, g.betay);
        m0y = (int)(((int64_t)m0 % g.gy + g.gy) % g.gy);
    }
    mx[e] = m0x;
    my[e] = m0y;
    const int bx0 = m0x / kNufftBin, bx1 = ((m0x + w) & (g.gx - 1)) / kNufftBin;
    const int by0 = m0y / kNufftBin, by1 = ((m0y + w) & (g.gy - 1)) / kNufftBin;
    const int64_t nbins = (int64_t)g.nbx * g.nby;
    const int bxs[2] = {bx0, bx1}, bys[2] = {by0, by1};
    for (int q = 0; q < 4; ++q) {
        const int bx = bxs[q & 1], by = bys[q >> 1];
        const bool repeat = ((q & 1) && bx1 == bx0) || ((q >> 1) && by1 == by0);
        const uint64_t bin = (uint64_t)(bt * nbins + (int64_t)by * g.nbx + bx);
        keys[4 * e + q] = repeat ? kNoKey : (bin << 32) | (uint64_t)k;
    }
}

// 1 / Psi at the centred pixel offsets of both axes.
__global__ __launch_bounds__(kT) void k_nufft_deapod(const NufftGeom g, float* __restrict__ dx, float* __restrict__ dy) {
    const int i = blockIdx.x * kT + threadIdx.x;
    if (i < g.nx) dx[i] = (float)(1.0 / kb_Psi((double)(i - g.nx / 2) / g.gx, g.w, g.betax));
    if (i < g.ny) dy[i] = (float)(1.0 / kb_Psi((double)(i - g.ny / 2) / g.gy, g.w, g.betay));
}

// Twiddles exp(-2 pi i m / G), m < G/2, evaluated in FP64.
__global__ __launch_bounds__(kT) void k_nufft_twiddles(const NufftGeom g, float2* __restrict__ twx,
                                                       float2* __restrict__ twy) {
    const int m = blockIdx.x * kT + threadIdx.x;
    if (m < g.gx / 2) {
        double s, c;
        sincospi(2.0 * m / g.gx, &s, &c);
        twx[m] = make_float2((float)c, (float)-s);
    }
    if (m < g.gy / 2) {
        double s, c;
        sincospi(2.0 * m / g.gy, &s, &c);
        twy[m] = make_float2((float)c, (float)-s);
    }
}

// One compare-exchange pass of a bitonic sort (ascending) over n = 2^p keys.
__global__ __launch_bounds__(kT) void k_bitonic(uint64_t* __restrict__ a, int64_t n, int64_t j, int64_t k) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const int64_t l = i ^ j;
    if (l <= i) return;
    const uint64_t x = a[i], y = a[l];
    const bool up = (i & k) == 0;
    if ((x > y) == up) {
        a[i] = y;
        a[l] = x;
    }
}

// First sorted entry of every bin (binary search), plus the count of all
// entries in the last slot.
__global__ __launch_bounds__(kT) void k_nufft_bin_starts(const uint64_t* __restrict__ keys, int64_t n,
                                                         int64_t nb_total, int32_t* __restrict__ bins) {
    const int64_t b = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (b > nb_total) return;
    const uint64_t target = (uint64_t)b << 32;
    int64_t lo = 0, hi = n;                               // first index with keys[i] >= target
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    bins[b] = (int32_t)lo;
}

// Forward step 1: the deapodised, coil-weighted image in the G grid
// (every grid element written: zeros outside the image).
__global__ __launch_bounds__(kT) void k_nufft_pre(const NufftGeom g, const float2* __restrict__ x,
                                                  const float2* __restrict__ smaps, int64_t smaps_bs,
                                                  const float* __restrict__ dx, const float* __restrict__ dy,
                                                  float2* __restrict__ grid) {
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int64_t gsz = (int64_t)g.gx * g.gy;
    if (e >= gsz * g.nc * g.nb) return;
    const int64_t bg = e / gsz;
    const int rem = (int)(e - bg * gsz);
    const int gyi = rem >> g.lgx, gxi = rem & (g.gx - 1);
    const int b = (int)(bg / g.nc), c = (int)(bg - (int64_t)b * g.nc);
    const int ox = gxi < g.gx / 2 ? gxi : gxi - g.gx;     // pixel offsets of this grid point
    const int oy = gyi < g.gy / 2 ? gyi : gyi - g.gy;
    const int j = ox + g.nx / 2, i = oy + g.ny / 2;
    float2 v = make_float2(0.f, 0.f);
    if (j >= 0 && j < g.nx && i >= 0 && i < g.ny) {
        const int64_t p = (int64_t)i * g.nx + j;
        const float2 s = smaps[b * smaps_bs + (int64_t)c * g.nx * g.ny + p];
        v = cscale(cmul(s, x[(int64_t)b * g.nx * g.ny + p]), dx[j] * dy[i]);
    }
    grid[e] = v;
}

// Radix-2 Stockham FFT of `per` signals of length G = 2^lg per block in LDS.
// Signal s, element i sits at (s / plane_sig) * plane_stride + (s % plane_sig)
// * sig_stride + i * elem_stride; rows (elem_stride 1) load element-major per
// signal, columns (sig_stride 1) signal-major, so a wave's loads are
// contiguous either way.  inverse: exp(+2 pi i m x / G) (conjugate twiddles).
__global__ __launch_bounds__(kT) void k_fft(float2* __restrict__ data, int lg, int per, int64_t plane_sig,
                                            int64_t plane_stride, int64_t sig_stride, int64_t elem_stride,
                                            const float2* __restrict__ tw, int inverse) {
    extern __shared__ __attribute__((aligned(16))) float2 lds[];
    const int n = 1 << lg, half = n >> 1;
    const int cnt = per * n;
    float2* buf0 = lds;
    float2* buf1 = lds + cnt;
    const int64_t s0 = (int64_t)blockIdx.x * per;
    const bool cols = sig_stride == 1 && elem_stride != 1;
    auto addr = [&](int c, int i) -> int64_t {
        const int64_t s = s0 + c;
        return (s / plane_sig) * plane_stride + (s % plane_sig) * sig_stride + (int64_t)i * elem_stride;
    };
    for (int q = threadIdx.x; q < cnt; q += kT) {
        const int c = cols ? q % per : q / n, i = cols ? q / per : q % n;
        buf0[c * n + i] = data[addr(c, i)];
    }
    __syncthreads();
    float2* src = buf0;
    float2* dst = buf1;
    for (int ll = 0; ll < lg; ++ll) {
        const int len = 1 << ll;
        for (int q = threadIdx.x; q < per * half; q += kT) {
            const int c = q >> (lg - 1), j = q & (half - 1);
            const int k = j & (len - 1);
            float2 w = tw[k << (lg - 1 - ll)];
            if (inverse) w.y = -w.y;
            const float2 a = src[c * n + j];
            const float2 b = cmul(src[c * n + j + half], w);
            const int d = ((j >> ll) << (ll + 1)) + k;
            dst[c * n + d] = cadd(a, b);
            dst[c * n + d + len] = csub(a, b);
        }
        __syncthreads();
        float2* t = src;
        src = dst;
        dst = t;
    }
    for (int q = threadIdx.x; q < cnt; q += kT) {
        const int c = cols ? q % per : q / n, i = cols ? q / per : q % n;
        data[addr(c, i)] = src[c * n + i];
    }
}

// Forward step 3: each sample gathers its (W+1) x (W+1) grid neighbours, for
// every coil (neighbours in a fixed order).
__global__ __launch_bounds__(kT) void k_nufft_interp(const NufftGeom g, const float* __restrict__ wx,
                                                     const float* __restrict__ wy, const int32_t* __restrict__ mx,
                                                     const int32_t* __restrict__ my, const float2* __restrict__ grid,
                                                     float2* __restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= (int64_t)g.nb * g.nk) return;
    const int b = (int)(e / g.nk);
    const int64_t k = e - (int64_t)b * g.nk;
    const int64_t se = (g.nbt > 1 ? (int64_t)b * g.nk : 0) + k;   // sample of the slice's trajectory
    const int w = g.w;
    float fx[kNufftMaxWidth + 1], fy[kNufftMaxWidth + 1];
    for (int i = 0; i <= w; ++i) {
        fx[i] = wx[se * (w + 1) + i];
        fy[i] = wy[se * (w + 1) + i];
    }
    const int x0 = mx[se], y0 = my[se];
    const int64_t gsz = (int64_t)g.gx * g.gy;
    for (int c = 0; c < g.nc; ++c) {
        const float2* gr = grid + ((int64_t)b * g.nc + c) * gsz;
        float2 acc = make_float2(0.f, 0.f);
        for (int iy = 0; iy <= w; ++iy) {
            const float2* row = gr + (int64_t)((y0 + iy) & (g.gy - 1)) * g.gx;
            float2 r = make_float2(0.f, 0.f);
            for (int ix = 0; ix <= w; ++ix) r = cadd(r, cscale(row[(x0 + ix) & (g.gx - 1)], fx[ix]));
            acc = cadd(acc, cscale(r, fy[iy]));
        }
        y[((int64_t)b * g.nc + c) * g.nk + k] = acc;
    }
}

// Adjoint step 1: one block per (16 x 16 bin, slice, group of up to 8
// coils); each thread owns one grid point and sums, in sample order, the
// samples of the bin's list whose kernel reaches it.  Every grid element is
// written by exactly one block (zero where no sample reaches).
constexpr int kSpreadChunk = 64;
constexpr int kSpreadCoils = 8;
__global__ __launch_bounds__(kT) void k_nufft_spread(const NufftGeom g, const float* __restrict__ wx,
                                                     const float* __restrict__ wy, const int32_t* __restrict__ mx,
                                                     const int32_t* __restrict__ my, const uint64_t* __restrict__ keys,
                                                     const int32_t* __restrict__ bins, const float2* __restrict__ y,
                                                     float2* __restrict__ grid) {
    __shared__ float sw_x[kSpreadChunk][kNufftMaxWidth + 1];
    __shared__ float sw_y[kSpreadChunk][kNufftMaxWidth + 1];
    __shared__ int32_t s_mx[kSpreadChunk], s_my[kSpreadChunk];
    __shared__ float2 s_d[kSpreadChunk][kSpreadCoils];
    const int nbins = g.nbx * g.nby;
    const int bin = blockIdx.x;
    const int ncg = (g.nc + kSpreadCoils - 1) / kSpreadCoils;
    const int b = blockIdx.y / ncg, cg = blockIdx.y - b * ncg;
    const int c0 = cg * kSpreadCoils, ncoil = min(kSpreadCoils, g.nc - c0);
    const int bt = g.nbt > 1 ? b : 0;
    const int64_t tb = (int64_t)bt * g.nk;                 // this trajectory's first sample
    const int32_t beg = bins[(int64_t)bt * nbins + bin], end = bins[(int64_t)bt * nbins + bin + 1];
    const int gxi = (bin % g.nbx) * kNufftBin + (threadIdx.x & (kNufftBin - 1));
    const int gyi = (bin / g.nbx) * kNufftBin + (threadIdx.x / kNufftBin);
    const int w = g.w;
    float2 acc[kSpreadCoils];
#pragma unroll
    for (int c = 0; c < kSpreadCoils; ++c) acc[c] = make_float2(0.f, 0.f);
    for (int e0 = beg; e0 < end; e0 += kSpreadChunk) {
        const int n = min(kSpreadChunk, end - e0);
        __syncthreads();
        for (int q = threadIdx.x; q < n * (w + 1); q += kT) {
            const int s = q / (w + 1), i = q - s * (w + 1);
            const int64_t k = (int64_t)(keys[e0 + s] & 0xffffffffu);
            sw_x[s][i] = wx[(tb + k) * (w + 1) + i];
            sw_y[s][i] = wy[(tb + k) * (w + 1) + i];
        }
        for (int q = threadIdx.x; q < n * kSpreadCoils; q += kT) {
            const int s = q / kSpreadCoils, c = q - s * kSpreadCoils;
            const int64_t k = (int64_t)(keys[e0 + s] & 0xffffffffu);
            if (c == 0) {
                s_mx[s] = mx[tb + k];
                s_my[s] = my[tb + k];
            }
            s_d[s][c] = c < ncoil ? y[((int64_t)b * g.nc + c0 + c) * g.nk + k] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        for (int s = 0; s < n; ++s) {
            const int ox = (gxi - s_mx[s]) & (g.gx - 1);
            const int oy = (gyi - s_my[s]) & (g.gy - 1);
            if (ox <= w && oy <= w) {
                const float wt = sw_x[s][ox] * sw_y[s][oy];
#pragma unroll
                for (int c = 0; c < kSpreadCoils; ++c) acc[c] = cadd(acc[c], cscale(s_d[s][c], wt));
            }
        }
    }
    const int64_t gsz = (int64_t)g.gx * g.gy;
#pragma unroll
    for (int c = 0; c < kSpreadCoils; ++c)      // constant indices keep acc in registers
        if (c < ncoil) grid[((int64_t)b * g.nc + c0 + c) * gsz + (int64_t)gyi * g.gx + gxi] = acc[c];
}

// Adjoint step 3: crop, deapodise and combine the coils in a fixed order.
__global__ __launch_bounds__(kT) void k_nufft_post(const NufftGeom g, const float2* __restrict__ grid,
                                                   const float2* __restrict__ smaps, int64_t smaps_bs,
                                                   const float* __restrict__ dx, const float* __restrict__ dy,
                                                   float2* __restrict__ x) {
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int64_t npix = (int64_t)g.nx * g.ny;
    if (e >= npix * g.nb) return;
    const int b = (int)(e / npix);
    const int64_t p = e - (int64_t)b * npix;
    const int i = (int)(p / g.nx), j = (int)(p - (int64_t)i * g.nx);
    const int gxi = (j - g.nx / 2) & (g.gx - 1), gyi = (i - g.ny / 2) & (g.gy - 1);
    const int64_t gsz = (int64_t)g.gx * g.gy;
    float2 acc = make_float2(0.f, 0.f);
    for (int c = 0; c < g.nc; ++c) {
        const float2 v = grid[((int64_t)b * g.nc + c) * gsz + (int64_t)gyi * g.gx + gxi];
        acc = cadd(acc, cmulc(smaps[b * smaps_bs + (int64_t)c * npix + p], v));
    }
    x[e] = cscale(acc, dx[j] * dy[i]);
}

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

int grid_side(int n, double sigma) {
    int gs = kNufftBin;
    while (gs < sigma * n) gs *= 2;
    return gs;
}

double kb_beta(int w, double sigma) {
    const double a = (double)w * w * (sigma - 0.5) * (sigma - 0.5) / (sigma * sigma) - 0.8;
    return 3.14159265358979323846 * std::sqrt(a > 0.0 ? a : 0.0);
}

hipError_t fft2(const NufftGeom& g, const NufftPtrs& P, int inverse, hipStream_t s) {
    const int64_t planes = (int64_t)g.nc * g.nb;
    const int64_t gsz = (int64_t)g.gx * g.gy;
    // rows: signals of length gx, element stride 1
    int per = std::max(1, 2048 / g.gx);
    if (per > g.gy) per = g.gy;
    size_t lds = 2 * sizeof(float2) * (size_t)per * g.gx;
    hipLaunchKernelGGL(k_fft, dim3((unsigned)(planes * g.gy / per)), dim3(kT), lds, s, P.grid, g.lgx, per,
                       (int64_t)g.gy, gsz, (int64_t)g.gx, (int64_t)1, P.twx, inverse);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // columns: signals of length gy, element stride gx, neighbouring columns adjacent
    per = std::max(1, std::min(16, 2048 / g.gy));
    if (per > g.gx) per = g.gx;
    lds = 2 * sizeof(float2) * (size_t)per * g.gy;
    hipLaunchKernelGGL(k_fft, dim3((unsigned)(planes * g.gx / per)), dim3(kT), lds, s, P.grid, g.lgy, per,
                       (int64_t)g.gx, gsz, (int64_t)1, (int64_t)g.gx, P.twy, inverse);
    return hipGetLastError();
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

int nufft_layout(const mri_shape& s, const mri_nufft_params& p, NufftLayout* out) {
    NufftLayout& L = *out;
    std::memset(&L, 0, sizeof(L));
    if (p.width < 2 || p.width > kNufftMaxWidth) return MRI_EINVAL;
    if (!(p.sigma >= 1.25 && p.sigma <= 4.0)) return MRI_EINVAL;
    NufftGeom& g = L.g;
    g.nx = s.nx;
    g.ny = s.ny;
    g.nc = s.ncoils;
    g.nb = s.batch;
    g.nbt = s.traj_batched ? s.batch : 1;
    g.nk = s.nk;
    g.w = p.width;
    g.gx = grid_side(s.nx, p.sigma);
    g.gy = grid_side(s.ny, p.sigma);
    if (g.gx > kNufftMaxGrid || g.gy > kNufftMaxGrid) return MRI_ENOTSUP;
    g.lgx = ilog2(g.gx);
    g.lgy = ilog2(g.gy);
    g.nbx = g.gx / kNufftBin;
    g.nby = g.gy / kNufftBin;
    g.betax = kb_beta(p.width, (double)g.gx / s.nx);
    g.betay = kb_beta(p.width, (double)g.gy / s.ny);
    g.nkeys = 4 * (int64_t)g.nbt * g.nk;
    g.nkeys_pow2 = 1;
    while (g.nkeys_pow2 < g.nkeys) g.nkeys_pow2 *= 2;
    const int64_t nbins = (int64_t)g.nbt * g.nbx * g.nby;
    if (g.nk >= ((int64_t)1 << 31) || nbins >= ((int64_t)1 << 31) || g.nkeys_pow2 >= ((int64_t)1 << 31))
        return MRI_ENOTSUP;
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const int64_t ns = (int64_t)g.nbt * g.nk;
    size_t o = 0;
    L.wx = o;   o += al(sizeof(float) * ns * (g.w + 1));
    L.wy = o;   o += al(sizeof(float) * ns * (g.w + 1));
    L.mx = o;   o += al(sizeof(int32_t) * ns);
    L.my = o;   o += al(sizeof(int32_t) * ns);
    L.dx = o;   o += al(sizeof(float) * g.nx);
    L.dy = o;   o += al(sizeof(float) * g.ny);
    L.twx = o;  o += al(sizeof(float2) * (g.gx / 2));
    L.twy = o;  o += al(sizeof(float2) * (g.gy / 2));
    L.keys = o; o += al(sizeof(uint64_t) * g.nkeys_pow2);
    L.bins = o; o += al(sizeof(int32_t) * (nbins + 1));
    L.grid = o; o += al(sizeof(float2) * (size_t)g.gx * g.gy * g.nc * g.nb);
    L.total = o;
    return MRI_OK;
}

NufftPtrs nufft_ptrs(const NufftLayout& L, void* ws) {
    char* b = static_cast<char*>(ws);
    NufftPtrs P;
    P.wx = reinterpret_cast<float*>(b + L.wx);
    P.wy = reinterpret_cast<float*>(b + L.wy);
    P.mx = reinterpret_cast<int32_t*>(b + L.mx);
    P.my = reinterpret_cast<int32_t*>(b + L.my);
    P.dx = reinterpret_cast<float*>(b + L.dx);
    P.dy = reinterpret_cast<float*>(b + L.dy);
    P.twx = reinterpret_cast<float2*>(b + L.twx);
    P.twy = reinterpret_cast<float2*>(b + L.twy);
    P.keys = reinterpret_cast<uint64_t*>(b + L.keys);
    P.bins = reinterpret_cast<int32_t*>(b + L.bins);
    P.grid = reinterpret_cast<float2*>(b + L.grid);
    return P;
}

hipError_t launch_nufft_prepare(const NufftLayout& L, const NufftPtrs& P, const double* traj, hipStream_t s) {
    const NufftGeom& g = L.g;
    const int64_t threads = std::max<int64_t>((int64_t)g.nbt * g.nk, g.nkeys_pow2 / 4);
    hipLaunchKernelGGL(k_nufft_samples, dim3(blocks(threads)), dim3(kT), 0, s, g, traj, P.wx, P.wy, P.mx, P.my,
                       P.keys);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nufft_deapod, dim3(blocks(std::max(g.nx, g.ny))), dim3(kT), 0, s, g, P.dx, P.dy);
    hipLaunchKernelGGL(k_nufft_twiddles, dim3(blocks(std::max(g.gx, g.gy) / 2)), dim3(kT), 0, s, g, P.twx, P.twy);
    const int64_t n = g.nkeys_pow2;
    for (int64_t k = 2; k <= n; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(k_bitonic, dim3(blocks(n)), dim3(kT), 0, s, P.keys, n, j, k);
    const int64_t nbins = (int64_t)g.nbt * g.nbx * g.nby;
    hipLaunchKernelGGL(k_nufft_bin_starts, dim3(blocks(nbins + 1)), dim3(kT), 0, s, P.keys, n, nbins, P.bins);
    return hipGetLastError();
}

hipError_t launch_nufft_forward(const NufftLayout& L, const NufftPtrs& P, const float2* x, const float2* smaps,
                                int64_t smaps_bs, float2* y, hipStream_t s) {
    const NufftGeom& g = L.g;
    const int64_t ngrid = (int64_t)g.gx * g.gy * g.nc * g.nb;
    hipLaunchKernelGGL(k_nufft_pre, dim3(blocks(ngrid)), dim3(kT), 0, s, g, x, smaps, smaps_bs, P.dx, P.dy, P.grid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = fft2(g, P, 0, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_nufft_interp, dim3(blocks((int64_t)g.nb * g.nk)), dim3(kT), 0, s, g, P.wx, P.wy, P.mx,
                       P.my, P.grid, y);
    return hipGetLastError();
}

hipError_t launch_nufft_adjoint(const NufftLayout& L, const NufftPtrs& P, const float2* y, const float2* smaps,
                                int64_t smaps_bs, float2* x, hipStream_t s) {
    const NufftGeom& g = L.g;
    const int ncg = (g.nc + kSpreadCoils - 1) / kSpreadCoils;
    hipLaunchKernelGGL(k_nufft_spread, dim3((unsigned)(g.nbx * g.nby), (unsigned)(g.nb * ncg)), dim3(kT), 0, s, g,
                       P.wx, P.wy, P.mx, P.my, P.keys, P.bins, y, P.grid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = fft2(g, P, 1, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_nufft_post, dim3(blocks((int64_t)g.nx * g.ny * g.nb)), dim3(kT), 0, s, g, P.grid, smaps,
                       smaps_bs, P.dx, P.dy, x);
    return hipGetLastError();
}

}  // namespace mri
