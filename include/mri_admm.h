/*
 * mri_admm.h -- C ABI of libmriadmm, an MI355X (gfx950) implementation of
 * compressed-sensing ADMM reconstruction of multi-coil non-Cartesian MRI with
 * the non-uniform DFT written as dense complex matrix products
 * (Lu et al., "Accelerating MRI Reconstruction on TPUs", arXiv:2006.14080).
 *
 * Notation follows the paper: image rho (here x), coil sensitivities s,
 * trajectory k, k-space data d (here y), regularisation lambda, augmented
 * Lagrangian penalty beta (eq. (5)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layout.  All arrays are dense, C-contiguous, little-endian:
 *   image   [B][ny][nx]          mri_c32, x (column) fastest
 *   smaps   [B or 1][nc][ny][nx] mri_c32
 *   traj    [B or 1][nk][2]      double, radians per pixel; column 0 pairs
 *                                with x, column 1 with y
 *   data    [B][nc][nk]          mri_c32, coil-major
 *   grad    [B][2][ny][nx]       mri_c32, [0] = x-difference, [1] = y-difference
 * Pixel (i, j) sits at the centred integer offsets y = i - ny/2, x = j - nx/2
 * (integer division), so the Cartesian case equals the centred FFT.
 *
 * Ownership.  Every array argument is a caller-owned DEVICE pointer, 8-byte
 * aligned; the library never retains one after the call returns.  The caller
 * allocates the workspace (size from mri_workspace_bytes); the library never
 * allocates device memory on these paths.
 *
 * Streams.  `stream` is a hipStream_t (NULL = default stream).  Every call
 * only enqueues work on it and returns; outputs are valid once the stream
 * reaches that point.  Calls are thread-safe when each thread uses its own
 * stream and its own workspace.
 *
 * Errors.  Entry points return 0 (MRI_OK) or a negative MRI_E* code and
 * enqueue nothing on error.  Outputs are unspecified after an error.
 * No C++ exception crosses this interface.
 */
#ifndef MRI_ADMM_H
#define MRI_ADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* complex64, the layout of torch.complex64 / std::complex<float>. */
typedef struct { float re, im; } mri_c32;

/* Problem shape.  batch >= 1 independent slices of one shape.
 * traj_batched / smaps_batched = 0: one array shared by every slice;
 * = 1: one array per slice.  nx != ny is allowed. */
typedef struct {
    int32_t nx, ny, ncoils;
    int64_t nk;
    int32_t batch;
    int32_t traj_batched, smaps_batched;
} mri_shape;

/* Arithmetic of the NUDFT matrix products. */
enum {
    MRI_FP32 = 0,   /* FP32 MFMA products, FP32 accumulation */
    MRI_BF16X3 = 1, /* split-BF16 compensated products (hi*hi + hi*lo + lo*hi)
                       on BF16 MFMA, FP32 accumulation (Sec. II-A); about 16
                       bits per operand */
    MRI_FP16X3 = 2, /* the same split products with fp16 parts on FP16 MFMA
                       (same rate): about 22 bits per operand; operands are
                       scaled by exact powers of two into fp16's range */
    MRI_NUFFT = 3   /* admm_solve only: F applied by the NUFFT operator
                       (nufft_*, width 6, oversampling 2, FP32) instead of
                       the dense NUDFT; one problem per call (any batch) */
};

enum {
    MRI_OK = 0,
    MRI_EINVAL = -1,    /* NULL pointer, bad shape or parameter */
    MRI_ENOMEM = -2,    /* workspace too small / budget exceeded */
    MRI_EHIP = -3,      /* HIP runtime error (see mri_strerror / mri_last_hip_error) */
    MRI_ENOTSUP = -4,   /* unsupported precision or shape */
    MRI_ENUMERIC = -5   /* non-finite value met during a solve (reported in stats) */
};

/* Operation selector for mri_workspace_bytes. */
enum { MRI_OP_FORWARD = 0, MRI_OP_ADJOINT = 1, MRI_OP_ADMM = 2 };

/* Largest supported sizes (one GPU's share). */
#define MRI_MAX_DIM 2048      /* nx, ny */
#define MRI_MAX_COILS 64
#define MRI_MAX_BATCH 4096

/*
 * nudft_forward -- y = F(x), eq. (1)-(2):
 *   y[b][g][k] = sum_{i,j} s[g][i][j] x[b][i][j] exp(-i (w0_k x_j + w1_k y_i)).
 * The phase matrix is never stored: it is generated tile by tile from the
 * trajectory (argument reduced in FP64, Alg. 1), and the product is the
 * separable form of Alg. 1, T = E_x (s (.) x)^T followed by a row sum
 * against E_y.
 *   x [B][ny][nx], smaps, traj as above, y [B][nc][nk] (written).
 *   precision: MRI_FP32, MRI_BF16X3 or MRI_FP16X3.
 *   ws/ws_bytes: workspace of at least mri_workspace_bytes(shape,
 *   MRI_OP_FORWARD, NULL) bytes; it receives the coil-weighted images
 *   s (.) x (rows padded to a multiple of 8 pixels): 8 B per coil pixel,
 *   in FP32 or, in the split forms, already split into 16-bit high and low
 *   parts in the matrix cores' operand order (MRI_FP16X3 adds one float
 *   scale per row).
 * Errors: MRI_EINVAL, MRI_ENOTSUP, MRI_ENOMEM, MRI_EHIP.
 */
int nudft_forward(const mri_shape* shape, const mri_c32* x, const mri_c32* smaps,
                  const double* traj, mri_c32* y, int precision,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * nudft_forward_noalloc -- nudft_forward for callers that cannot allocate
 * device memory or pass a workspace (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The same kernels and
 * results (bit for bit) as nudft_forward; the coil-weighted images go to a
 * library-owned device scratch array of mri_noalloc_scratch_bytes() bytes
 * (64 MiB, held on each GPU the library runs on until the process ends)
 * instead of a workspace.  Nothing is allocated and nothing needs clearing:
 * every scratch byte the kernels read is written earlier in the same call.
 * All calls on one GPU share that GPU's array: calls that overlap on one GPU
 * (different streams or threads without ordering) race and give undefined
 * results.  The first call on a device looks up the array's address there.
 * Errors: as nudft_forward; MRI_ENOMEM when the shape needs more than the
 * scratch (mri_workspace_bytes(shape, MRI_OP_FORWARD, NULL) > 64 MiB).
 */
int nudft_forward_noalloc(const mri_shape* shape, const mri_c32* x, const mri_c32* smaps,
                          const double* traj, mri_c32* y, int precision, void* stream);
size_t mri_noalloc_scratch_bytes(void);

/*
 * nudft_adjoint -- x = F^H(y): the adjoint of eq. (1) with the conjugate coil
 * combine, which is the "inverse DFT" of Alg. 3 and the F^H of eq. (12)-(13):
 *   x[b][i][j] = sum_g conj(s[g][i][j]) sum_k exp(+i (w0_k x_j + w1_k y_i)) y[b][g][k].
 * No density compensation.  The sample sum is split over workgroups and the
 * partial images are added in a fixed order, so results are bitwise
 * reproducible run to run.
 *   y [B][nc][nk], x [B][ny][nx] (written).  Workspace: MRI_OP_ADJOINT; it
 *   holds the partial images and the phase tables exp(+i w_k x), exp(+i w_k y)
 *   of the trajectory, (nx + ny) * nk * 8 bytes per trajectory (Alg. 1 forms
 *   the same factors), rebuilt by every call.  Equivalent to
 *   nudft_adjoint_prepare followed by nudft_adjoint_prepared.
 * Errors: as nudft_forward.
 */
int nudft_adjoint(const mri_shape* shape, const mri_c32* y, const mri_c32* smaps,
                  const double* traj, mri_c32* x, int precision,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * nudft_adjoint_prepare -- fill the phase tables of nudft_adjoint for one
 * shape and trajectory into an MRI_OP_ADJOINT workspace (the values are those
 * of Alg. 1's phase factors, with the FP64 argument reduction).
 * nudft_adjoint_prepared -- nudft_adjoint using the tables already in ws,
 * for callers that apply the adjoint repeatedly with a fixed trajectory (as
 * admm_solve does inside): results are bit-identical to nudft_adjoint.  The
 * tables must come from nudft_adjoint_prepare (or nudft_adjoint) with the
 * same shape, trajectory contents and workspace, and be complete on the
 * stream (same stream, or synchronised); otherwise the result is undefined.
 * Only the partial-image part of ws is written, so prepared calls may follow
 * each other on one stream.
 * Errors: as nudft_forward (nudft_adjoint_prepare reads only shape, traj, ws).
 */
int nudft_adjoint_prepare(const mri_shape* shape, const double* traj,
                          void* ws, size_t ws_bytes, void* stream);
int nudft_adjoint_prepared(const mri_shape* shape, const mri_c32* y, const mri_c32* smaps,
                           const double* traj, mri_c32* x, int precision,
                           void* ws, size_t ws_bytes, void* stream);

/*
 * tv_forward -- g = Theta(x), the finite-difference sparsifying transform
 * (Sec. III-A, Sec. IV-B): forward differences with periodic wrap,
 *   g[b][0][i][j] = x[b][i][(j+1) mod nx] - x[b][i][j]
 *   g[b][1][i][j] = x[b][(i+1) mod ny][j] - x[b][i][j].
 *   x [B][ny][nx], g [B][2][ny][nx] (written).  Only nx, ny, batch are read.
 * Errors: MRI_EINVAL, MRI_EHIP.
 */
int tv_forward(const mri_shape* shape, const mri_c32* x, mri_c32* g, void* stream);

/*
 * tv_adjoint -- x = Theta^H(g), the exact conjugate transpose of tv_forward:
 *   x[i][j] = g0[i][(j-1) mod nx] - g0[i][j] + g1[(i-1) mod ny][j] - g1[i][j].
 * Errors: MRI_EINVAL, MRI_EHIP.
 */
int tv_adjoint(const mri_shape* shape, const mri_c32* g, mri_c32* x, void* stream);

/* ADMM parameters (Table I names).  beta is the paper's augmented-Lagrangian
 * penalty (eq. (5)); the soft threshold of eq. (9) is lambda/beta and the
 * normal matrix of eq. (12) carries beta/2.  rtol = atol = 0 runs exactly
 * admm_iters x cg_iters steps (a step still stops early when its residual is
 * exactly zero or CG breaks down).  cg_warm_start = 1 starts each CG solve
 * from the current image, 0 from the initial image. */
typedef struct {
    double lambda, beta;
    int32_t admm_iters, cg_iters;
    double rtol, atol;
    int32_t precision, cg_warm_start;
} mri_admm_params;

/* Per-slice solve report, written to device memory at the end of admm_solve. */
typedef struct {
    int32_t admm_iters_run;  /* ADMM iterations executed */
    int32_t cg_steps_run;    /* CG steps executed, summed over ADMM iterations */
    double alpha;            /* last ||rho' - rho||^2 / ||rho||^2 (Alg. 4) */
    double tau;              /* last CG residual r^H r (Alg. 2) */
    int32_t status;          /* MRI_OK or MRI_ENUMERIC */
    int32_t pad;
} mri_admm_stats;

/*
 * admm_solve -- the whole of Alg. 4 (ADMM, eq. (6)-(13)) with the rho-update
 * solved by conjugate gradient (Alg. 2), per slice:
 *   F^H y once; rho = x0 (or 0), eta = 0; then per iteration
 *   mu = S_{lambda/beta}(Theta rho + eta)                  eq. (9)-(10)
 *   b = F^H y + (beta/2) Theta^H (mu - eta)                 eq. (13)
 *   solve (F^H F + (beta/2) Theta^H Theta) rho' = b by CG   eq. (11)-(12)
 *   eta += Theta rho' - mu;  alpha = ||rho' - rho||^2/||rho||^2   eq. (8)
 * stopping when the iteration cap is reached or alpha <= rtol^2.  CG starts
 * from r = b - A rho, stops after cg_iters steps, when r^H r <= atol^2, or
 * when d^H A d <= 0.  Vector arithmetic is FP32; dot products, norms and the
 * CG/ADMM scalars are FP64.  The complex soft threshold shrinks magnitudes.
 *   smaps, traj, y: inputs as above; x0 [B][ny][nx] or NULL (zeros);
 *   x_out [B][ny][nx] (written); stats_dev: device array of B mri_admm_stats
 *   or NULL.  Workspace: mri_workspace_bytes(shape, MRI_OP_ADMM, params).
 * Nothing is copied back to the host and the host never waits: all control
 * decisions (tolerances, breakdown) are taken on the device.
 * Errors: MRI_EINVAL (lambda < 0, beta <= 0, negative counts, bad shape),
 * MRI_ENOTSUP, MRI_ENOMEM, MRI_EHIP.
 */
int admm_solve(const mri_shape* shape, const mri_c32* smaps, const double* traj,
               const mri_c32* y, const mri_c32* x0, const mri_admm_params* params,
               mri_c32* x_out, mri_admm_stats* stats_dev,
               void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Request server: continuous batching of independent reconstructions.
 *
 * A server owns one device memory pool of `hbm_budget` bytes, allocated once
 * by mri_server_create (nothing is allocated on the device afterwards), and up
 * to `max_slots` (<= MRI_SERVER_MAX_SLOTS) concurrently running solves.
 * Submitted requests wait in a FIFO queue; every mri_server_step() first
 * admits queued requests in order while a slot is free and the pool can hold
 * the request's inputs, output and workspace, then runs ONE ADMM iteration
 * (Alg. 4 with its CG solve) for every active slot: each kernel of the
 * iteration is one grouped launch over all slots, so their work overlaps on
 * the device, and the iteration is replayed from a captured HIP graph that is
 * re-captured only when the set of active slots changes.  Each solve's ADMM
 * state stays resident in the pool.  After the iteration the step reads the
 * per-slot stopping flags, copies finished images to host memory and frees
 * their slots.  A slot's arithmetic does not depend on which other requests
 * share its launches, so a result is bit-for-bit the same alone and in a mix,
 * and equal to admm_solve on the same inputs.
 *
 * All mri_server_* calls on one server must come from one thread.  Input
 * arrays of mri_server_submit are HOST pointers and are copied before the
 * call returns.  Results are copied out to host memory by mri_server_poll.
 * --------------------------------------------------------------------------- */

#define MRI_SERVER_MAX_SLOTS 16

typedef struct {
    mri_shape shape;             /* batch must be 1; per-request traj/smaps */
    const mri_c32* smaps;        /* host [nc][ny][nx] */
    const double* traj;          /* host [nk][2] */
    const mri_c32* y;            /* host [nc][nk] */
    const mri_c32* x0;           /* host [ny][nx] or NULL */
    mri_admm_params params;      /* params.precision must equal the server's */
} mri_request;

typedef struct {
    int32_t queued, active, completed, cancelled;
    int64_t steps;               /* mri_server_step calls that ran an iteration */
    int64_t graph_captures;      /* iteration graphs captured */
    size_t pool_bytes, pool_used;
} mri_server_info;

enum { MRI_REQ_UNKNOWN = -1, MRI_REQ_QUEUED = 0, MRI_REQ_RUNNING = 1, MRI_REQ_DONE = 2 };

/* Create a server.  precision: MRI_FP32, MRI_BF16X3 or MRI_FP16X3 for all
 * its requests (MRI_NUFFT is not served: MRI_ENOTSUP).  stream: the hipStream_t every copy, launch and graph replay
 * of the server goes to (it must stay valid until mri_server_destroy and
 * must not be the legacy default stream, which cannot be captured); NULL =
 * the server creates and owns a non-blocking stream of its own.
 * Errors: MRI_EINVAL (max_slots out of range), MRI_ENOMEM (pool allocation
 * failed), MRI_EHIP. */
int mri_server_create(size_t hbm_budget, int max_slots, int precision, void* stream, void** srv);

/* Queue a request; *id receives its handle.  MRI_ENOMEM if the request alone
 * can never fit the pool; MRI_EINVAL for bad shape/params (batch != 1). */
int mri_server_submit(void* srv, const mri_request* req, uint64_t* id);

/* Bytes of pool one request occupies while it runs. */
size_t mri_server_request_bytes(const mri_shape* shape, int precision);

/* Admit, run one ADMM iteration for all active slots, retire finished ones.
 * Blocks until the iteration is done.  *n_active (nullable) receives the
 * number of slots that ran.  Returns 0 with *n_active = 0 when idle. */
int mri_server_step(void* srv, int* n_active);

/* State of a request (MRI_REQ_*).  When DONE and out_image is non-NULL the
 * host image [ny][nx] and (if non-NULL) the stats are copied out and the
 * result is released (a later poll reports MRI_REQ_UNKNOWN). */
int mri_server_poll(void* srv, uint64_t id, mri_c32* out_image, mri_admm_stats* stats, int* state);

/* Drop a queued or running request (its slot and memory are freed). */
int mri_server_cancel(void* srv, uint64_t id);

int mri_server_get_info(void* srv, mri_server_info* info);

/* Free the pool and all server resources. */
int mri_server_destroy(void* srv);

/* Workspace bytes needed by an operation (params may be NULL except for
 * MRI_OP_ADMM).  Returns 0 for an invalid shape. */
size_t mri_workspace_bytes(const mri_shape* shape, int op, const mri_admm_params* params);

/* ---------------------------------------------------------------------------
 * NUFFT operator: the O(N log N) approximation of F used by the paper's
 * comparison systems (Sec. VII, Table II), as an alternative to the dense
 * nudft_* operators, with the same shapes, layouts and conventions.
 *
 * Forward, per slice and coil: the coil-weighted image divided by the
 * kernel's Fourier transform (deapodisation) is zero-padded into a grid of
 * G = the smallest power of two >= sigma * n (at least 16) per axis, FFTed
 * (exp(-2 pi i m x / G)), and each sample interpolates its (W+1) x (W+1)
 * nearest grid points with the Kaiser-Bessel kernel
 *   psi(u) = I0(beta sqrt(1 - (2u/W)^2)),  |u| <= W/2,
 *   beta = pi sqrt(W^2 (s - 1/2)^2 / s^2 - 0.8),  s = G / n,
 * at the sample's grid position t = w G / (2 pi).  The adjoint is its exact
 * conjugate transpose (spreading, inverse FFT, crop, deapodisation, conj(s)
 * coil combine).  Relative error against the exact NUDFT: about 2e-6
 * (forward) and 5e-6 (adjoint) at W = 6, sigma = 2, and near ten times less
 * per extra point of width (W = 7: below 1e-6).  Spreading is deterministic:
 * every grid point sums the samples that reach it in sample order, so
 * results are bitwise reproducible run to run.
 *
 * A workspace of mri_nufft_workspace_bytes(shape, params) holds the plan
 * (per trajectory: each sample's neighbours and kernel weights, the samples
 * of every 16 x 16 grid tile sorted by index; deapodisation; FFT twiddles)
 * and the grid ([B][nc][Gy][Gx] complex64).  nufft_prepare builds the plan
 * from the trajectory (traj as for nudft_*, per slice when traj_batched);
 * nufft_forward / nufft_adjoint apply the operator with the plan already in
 * ws (same shape and params, prepared on the same stream or synchronised),
 * and overwrite only the grid, so they may follow each other.
 * --------------------------------------------------------------------------- */
typedef struct {
    int32_t width;        /* W, kernel width in grid points: 2 .. 10 (6 by default) */
    int32_t pad;
    double sigma;         /* oversampling: 1.25 .. 4 (2 by default); G <= 4096 */
} mri_nufft_params;

/* Workspace bytes of the NUFFT for a shape and parameters (0 when invalid or
 * unsupported). */
size_t mri_nufft_workspace_bytes(const mri_shape* shape, const mri_nufft_params* params);

/* Build the plan for shape / traj / params in ws.
 * Errors: MRI_EINVAL (null pointer, bad shape or params), MRI_ENOTSUP (grid
 * side above 4096 or too many samples), MRI_ENOMEM (ws too small), MRI_EHIP. */
int nufft_prepare(const mri_shape* shape, const double* traj, const mri_nufft_params* params,
                  void* ws, size_t ws_bytes, void* stream);

/* y ~ F(x): x [B][ny][nx], smaps [B or 1][nc][ny][nx], y [B][nc][nk]
 * (written).  Errors: as nufft_prepare. */
int nufft_forward(const mri_shape* shape, const mri_c32* x, const mri_c32* smaps, mri_c32* y,
                  const mri_nufft_params* params, void* ws, size_t ws_bytes, void* stream);

/* x ~ F^H(y), the exact adjoint of nufft_forward: y [B][nc][nk], x
 * [B][ny][nx] (written).  Errors: as nufft_prepare. */
int nufft_adjoint(const mri_shape* shape, const mri_c32* y, const mri_c32* smaps, mri_c32* x,
                  const mri_nufft_params* params, void* ws, size_t ws_bytes, void* stream);

/* Sample-range split of nudft_adjoint for a shape (the same for every
 * precision): *ksplit sample ranges of *kper samples each, and *planes
 * partial images per slice in the workspace, one per (sample range, coil
 * group of up to 8 coils), summed in a fixed order after the matrix
 * products.  Any output pointer may be NULL.  This fixes the adjoint's
 * summation order, and so its rounding, and the workspace's partial-image
 * bytes (*planes x batch x nx x ny x 8).
 * Errors: MRI_EINVAL for an invalid shape. */
int mri_adjoint_split(const mri_shape* shape, int32_t* ksplit, int32_t* kper, int32_t* planes);

/* Static description of an error code. */
const char* mri_strerror(int code);

/* Text of the last HIP error seen by this thread ("" if none). */
const char* mri_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MRI_ADMM_H */
