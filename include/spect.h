/*
 * spect.h -- C ABI of the MI355X (gfx950) rotation-based SPECT projector pair.
 *
 * Operator (Z. Li, Y. K. Dewaraja, J. A. Fessler, "Training End-to-End
 * Unrolled Iterative Neural Networks for SPECT Image Reconstruction"):
 *
 *   forward A (Sec. II-A, Alg. 1): for every view l, rotate the activity x and
 *     the attenuation map mu about z by theta_l (exact quarter turn, then three
 *     1-D linear-interpolation shears, zero outside the grid); form the
 *     accumulated attenuation factor of Eq. (1); weight; convolve every depth
 *     plane j with its PSF p(:,:,j,l) using replicate padding; sum over depth.
 *   back A' (Eq. (2), Alg. 2): the exact transpose of every one of those steps
 *     (transposed interpolation, the fold that is the adjoint of replicate
 *     padding), summed over views.
 *   EM (Sec. II-B, Eq. (7)-(8) with beta -> 0):
 *     x <- x * A'(y / (A x + r)) / A'1.
 *
 * Layouts (C order, float32, 0-based indices):
 *   volume      x[k][j][i]          nz x ny x nx   (i = x fastest, j = depth y)
 *   projection  v[l][k][i]          nview x nz x nx
 *   PSF         p[l][j][b][a]       nview x ny x pz x px (a along x fastest)
 * Plane j = ny-1 is nearest the detector.  Rotation centre c = (nx-1)/2.
 *
 * Memory ownership: the caller owns every device buffer (x, v, mu, psf, y, r,
 * sens, workspace).  A plan borrows mu, psf and the workspace; they must stay
 * valid and unmodified until spect_plan_destroy.  The library allocates only
 * the small host-side plan object; forward / back / em_step never allocate.
 * Outputs are overwritten, never accumulated.  Input and output buffers of one
 * call must not overlap (except x of spect_em_step, which is updated in place).
 *
 * Streams: every call enqueues work on the given HIP stream and returns without
 * synchronising.  A plan has one workspace, so at most one call per plan may
 * be in flight at a time; ordering across streams is the caller's business.
 *
 * Errors: argument, shape, alignment and workspace problems are reported
 * synchronously, before anything is enqueued (so they can be tested without a
 * GPU).  A failed launch returns SPECT_ERR_HIP.  Device faults surface at the
 * caller's next synchronisation.  No C++ exception crosses this ABI.
 */
#ifndef SPECT_H_
#define SPECT_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spect_plan_s* spect_plan;

typedef enum {
  SPECT_OK = 0,
  SPECT_ERR_NULL = 1,        /* a required pointer is NULL */
  SPECT_ERR_SHAPE = 2,       /* nx != ny, non-positive size, even PSF size */
  SPECT_ERR_VALUE = 3,       /* dy <= 0 or not finite, non-finite angle, bad flag */
  SPECT_ERR_WORKSPACE = 4,   /* workspace smaller than spect_workspace_bytes */
  SPECT_ERR_UNSUPPORTED = 5, /* size outside what this build supports */
  SPECT_ERR_HIP = 6,         /* a HIP runtime call or launch failed */
  SPECT_ERR_ALIGN = 7        /* device pointer not aligned as documented */
} spect_status;

/* convolution precision (spect_geom.conv_precision) */
#define SPECT_CONV_FP32 0  /* FP32 throughout (the reference-accuracy path) */
#define SPECT_CONV_BF16 1  /* PSF convolution and its adjoint as BF16 matrix-core
                              products with FP32 accumulation; rotation, attenuation,
                              depth sum, edge fold and EM stay FP32 */
#define SPECT_CONV_FP16 2  /* the same with FP16 operands: values of the weighted
                              volume and of projections handed to spect_back must
                              stay below 65504 in magnitude */
#define SPECT_CONV_BF16X3 3 /* each FP32 operand split as a BF16 leading part plus
                               a BF16 remainder (16 significant bits), each product
                               as three BF16 matrix-core products (hi*hi + hi*lo +
                               lo*hi) with FP32 accumulation: FP32-level accuracy on
                               the BF16 matrix cores */

/* flags */
#define SPECT_CACHE_MUBAR 0x1u  /* keep the attenuation factor of Eq. (1) for all
                                   views in the workspace (nview*nx*ny*nz floats),
                                   computed once at plan creation */
#define SPECT_ROT_BILINEAR 0x2u /* rotate activity and attenuation by 2-D bilinear
                                   interpolation with zero padding (the alternative
                                   Sec. II-A names beside the 3-pass shears): after
                                   the exact quarter turn, out(p) = bilinear sample at
                                   R(phi)^-1 (p - c) + c; spect_back applies its exact
                                   transpose.  Default: three 1-D shears. */
#define SPECT_PSF_SEPARABLE 0x4u /* the PSFs are separable (rank 1), p[b][a] = fz[b] fx[a]
                                    (an axis-aligned 2-D Gaussian fit is): d_psf then holds
                                    the factors, [nview][ny][pz + px] with the pz values of
                                    fz first, and the convolution runs as two 1-D passes
                                    (2 (px + pz) instead of 2 px pz FLOP per voxel).  FP32
                                    only: with another conv_precision, or a strip that does
                                    not fit the kernel's LDS, SPECT_ERR_UNSUPPORTED. */
#define SPECT_PSF_ALL_TAPS 0x8u /* never pair mirror-image PSF taps (see spect_plan_create);
                                   the plan then waits for nothing */
#define SPECT_PSF_SYMMETRIC_X 0x10u /* the caller states that every PSF row is its own
                                       mirror image in x, p[b][a] == p[b][px-1-a] (a centred
                                       Gaussian is): the FP32 4x4-block convolution pairs
                                       taps without checking on the device, and plan
                                       creation waits for nothing.  With a PSF that is not
                                       symmetric, the operator computed is that of the PSF
                                       p'[b][a] = p[b][min(a, px-1-a)].  Exclusive with
                                       SPECT_PSF_ALL_TAPS (else SPECT_ERR_VALUE). */
#define SPECT_TILING_4X4 0x20u  /* FP32 convolution on 4x4 matrix blocks when the shape
                                   fits them (else 16x16 blocks), instead of the plan's
                                   cost model */
#define SPECT_TILING_16X16 0x40u /* FP32 convolution as 16x16x4 Toeplitz blocks, instead of
                                    the plan's cost model.  Exclusive with SPECT_TILING_4X4
                                    (else SPECT_ERR_VALUE). */
#define SPECT_CONV_FFT 0x80u    /* PSF convolution through FP32 FFTs, as Sec. II-A computes it:
                                   the same operator (replicate padding, exact adjoint with
                                   the padding's fold), evaluated as circular convolutions of
                                   a size that holds the padded plane, with the depth sum
                                   taken on the spectra.  Any PSF (no symmetry needed).  The
                                   plan computes the PSF spectra once (nview*ny spectra of
                                   about (Lx/2) Lz complex values, Lx >= nx+px-1 and
                                   Lz >= nz+pz-1 the smallest even products of 2, 3, 5) and
                                   keeps them in the workspace.  FP32 only, not with
                                   SPECT_PSF_SEPARABLE; planes whose transform does not fit
                                   the kernels' LDS give SPECT_ERR_UNSUPPORTED.  Where the
                                   exact result is zero (bins outside the body's shadow),
                                   outputs carry rounding noise of either sign, of the order
                                   of 1e-7 times the largest output: clamp them before a use
                                   that needs nonnegative values (a Poisson rate). */
#define SPECT_PSF_SYMMETRIC_Z 0x100u /* the caller states that every PSF column is its own
                                        mirror image in z, p[b][a] == p[pz-1-b][a].  With
                                        SPECT_CONV_FFT and SPECT_PSF_SYMMETRIC_X too, on the
                                        transform sizes compiled in (spect_plan_describe
                                        reports fft_fixed other than 0), the plan keeps the
                                        spectra of the PSFs centred on the origin, which are
                                        then real (one float per bin instead of two: half the
                                        spectra's workspace and traffic, a real product per
                                        bin).  With a PSF that is not symmetric in both, the
                                        operator is that of its point-symmetric part
                                        (p[b][a] + p[pz-1-b][px-1-a]) / 2.  Ignored
                                        otherwise. */

/* Geometry of one plan (host struct, copied by spect_plan_create). */
typedef struct {
  int32_t nx, ny, nz;     /* volume size; nx == ny (rotation about z) */
  int32_t nview;          /* number of projection views */
  int32_t px, pz;         /* PSF size along x and z; both odd */
  double dy;              /* voxel size along y (same length unit as 1/mu), Eq. (1) */
  const double* angles;   /* host array of nview angles in radians, or NULL for
                             theta_l = 2 pi l / nview (Sec. II-A); read only
                             during spect_plan_create */
  uint32_t flags;         /* SPECT_CACHE_MUBAR | SPECT_ROT_BILINEAR | SPECT_PSF_SEPARABLE |
                             SPECT_PSF_ALL_TAPS | SPECT_PSF_SYMMETRIC_X | SPECT_TILING_4X4 |
                             SPECT_TILING_16X16 | SPECT_CONV_FFT | SPECT_PSF_SYMMETRIC_Z,
                             or 0; other bits give SPECT_ERR_VALUE */
  int32_t view_batch;     /* views processed per internal batch; 0 = all.
                             Smaller batches need less workspace. */
  int32_t conv_precision; /* SPECT_CONV_FP32 (0), SPECT_CONV_BF16, SPECT_CONV_FP16 or
                             SPECT_CONV_BF16X3;
                             other values give SPECT_ERR_VALUE */
} spect_geom;

/* Workspace bytes a plan with geometry g needs (host only, no GPU call).
 * Returns SPECT_ERR_* for an invalid geometry. */
spect_status spect_workspace_bytes(const spect_geom* g, size_t* bytes);

/* Create a plan.  d_mu: [nz][ny][nx] attenuation map (units of 1/dy),
 * d_psf: [nview][ny][pz][px] (with SPECT_PSF_SEPARABLE: [nview][ny][pz + px],
 * the z factor then the x factor), d_workspace: device memory of ws_bytes
 * (>= spect_workspace_bytes, 256-byte aligned).  All three are borrowed.
 * Enqueues the upload of the per-view shear tables (and, with
 * SPECT_CACHE_MUBAR, the attenuation-factor precomputation) on `stream`.
 * When the FP32 convolution runs on 4x4 blocks and neither SPECT_PSF_ALL_TAPS
 * nor SPECT_PSF_SYMMETRIC_X is set, it also checks on the device whether every
 * PSF row is its own mirror image in x (p[b][a] == p[b][px-1-a] exactly, as
 * for a centred Gaussian or any circularly symmetric response); if so the
 * convolution pairs taps a and px-1-a, adding the two input columns before
 * one product ((px + 1) / 2 products per row instead of px, the same operator
 * up to FP32 rounding).  That check waits for `stream`; the two flags skip it
 * (keep every tap, or pair on the caller's word). */
spect_status spect_plan_create(spect_plan* out, const spect_geom* g,
                               const float* d_mu, const float* d_psf,
                               void* d_workspace, size_t ws_bytes,
                               hipStream_t stream);

/* v = A x.  d_x: [nz][ny][nx], d_v: [nview][nz][nx] (overwritten).  Alg. 1. */
spect_status spect_forward(spect_plan plan, const float* d_x, float* d_v,
                           hipStream_t stream);

/* x = A' v.  d_v: [nview][nz][nx], d_x: [nz][ny][nx] (overwritten).
 * Exact transpose of spect_forward; Eq. (2), Alg. 2. */
spect_status spect_back(spect_plan plan, const float* d_v, float* d_x,
                        hipStream_t stream);

/* One ML-EM update in place (Eq. (7)-(8), beta -> 0):
 *   ybar = A x + r;  rho = y / ybar (0 where ybar <= 0);
 *   x <- x * A' rho / sens (0 where sens <= 0).
 * d_y: [nview][nz][nx] measured counts; d_r: background of the same shape or
 * NULL for zero; d_sens: A'1, [nz][ny][nx] (caller computes it once with
 * spect_back on a projection of ones). */
spect_status spect_em_step(spect_plan plan, float* d_x, const float* d_y,
                           const float* d_r, const float* d_sens,
                           hipStream_t stream);

/* One regularised EM update in place (Sec. II-B, Eq. (7)-(8)): with
 *   e = A'(y / (A x + r))  (the ratio 0 where A x + r <= 0),
 *   d = sens - beta * u,
 * x becomes the nonnegative root of beta x^2 + d x - x_old e = 0,
 *   x = (-d + sqrt(d^2 + 4 beta x_old e)) / (2 beta),
 * evaluated without cancellation when d > 0.  d_u: the regularisation
 * target [nz][ny][nx] (the paper's CNN output u_k); beta >= 0 and finite
 * (beta = 0 gives x_old e / sens, 0 where sens <= 0); otherwise
 * SPECT_ERR_VALUE.  Other arguments as for spect_em_step. */
spect_status spect_reg_em_step(spect_plan plan, float* d_x, const float* d_y,
                               const float* d_r, const float* d_sens, const float* d_u,
                               float beta, hipStream_t stream);

/* Vector-Jacobian product of one spect_em_step (Sec. II-B: the unrolled EM
 * iterations are trained by backpropagation, and the projector's adjoint is
 * what makes that exact).  For x+ = em_step(x, y) and an upstream gradient
 * g = dL/dx+ ([nz][ny][nx]) it writes
 *   d_gx = dL/dx  = g * b / sens + A'(gq)          [nz][ny][nx]
 *   d_gy = dL/dy  = t / ybar  (NULL to skip)       [nview][nz][nx]
 * with ybar = A x + r, rho = y / ybar, b = A' rho, t = A(g * x / sens) and
 * gq = -(t / ybar) * (y / ybar); the guarded branches (sens <= 0, ybar <= 0)
 * are constant and contribute zero.  The step's forward is recomputed from
 * d_x, so a caller that keeps only the iterates x_k gets gradients through
 * unrolled EM (four projector directions per step).  d_x, d_y, d_r
 * (nullable), d_sens as for spect_em_step; d_g must not overlap d_x, d_y,
 * d_r, d_sens or d_gy; d_gx may equal d_g and overlaps no other buffer. */
spect_status spect_em_step_vjp(spect_plan plan, const float* d_x, const float* d_y,
                               const float* d_r, const float* d_sens, const float* d_g,
                               float* d_gx, float* d_gy, hipStream_t stream);

/* v = A x without a plan and without allocating anything, for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The same operator and kernels as
 * spect_forward on a plan of geometry g (Alg. 1).  What a plan's workspace
 * would hold (rotation tables, computed on the device; the attenuation factors
 * of a view batch; weighted volumes; partial sums) lives in a static device
 * array of the library, 64 MiB per device, which spect_workspace_bytes(g)
 * must not exceed (else SPECT_ERR_WORKSPACE, before any device work; choose
 * g->view_batch to fit).  The array is shared by every call on a device and
 * keeps the last call's contents: calls that overlap on one device race.
 * Restrictions: g->angles must be NULL (default angles; else
 * SPECT_ERR_UNSUPPORTED); SPECT_CACHE_MUBAR is ignored; mirror-image taps are
 * paired only with SPECT_PSF_SYMMETRIC_X (no device check); with
 * SPECT_CONV_FFT the PSF spectra are computed in the array on every call
 * (they count in spect_workspace_bytes whatever the view batch).  d_mu
 * [nz][ny][nx], d_psf as for spect_plan_create, d_x [nz][ny][nx], d_v
 * [nview][nz][nx] (overwritten); all 4-byte aligned.  The first call on a
 * device looks up the array's address there (hipGetSymbolAddress). */
spect_status spect_forward_static(const spect_geom* g, const float* d_mu, const float* d_psf,
                                  const float* d_x, float* d_v, hipStream_t stream);

/* Release the host plan object (does not free borrowed device memory). */
spect_status spect_plan_destroy(spect_plan plan);

/* Human-readable text of a status code (static storage). */
const char* spect_status_string(spect_status s);

/* Test support: *d_out = sum_i (double)a[i] * (double)b[i] for float32 device
 * arrays of n elements, accumulated in FP64 in a fixed order (deterministic).
 * d_out is a device pointer to one double.  Used for adjoint-identity checks. */
spect_status spect_dot_f64(const float* d_a, const float* d_b, size_t n,
                           double* d_out, hipStream_t stream);

/* Per-kernel timing of one plan, for benchmarks.  spect_profile_start creates
 * a pool of 2*max_launches HIP events (host-side runtime objects, no device
 * memory); while it is active every kernel the plan launches is bracketed by
 * an event pair recorded on the caller's stream (launches beyond the pool are
 * not timed).  spect_profile_stop waits for the recorded events, writes one
 * entry per kernel name (at most max_out) to `out`, sets *n_out, releases the
 * pool and ends profiling.  Not for use while another call on the plan is
 * being enqueued from a different host thread. */
typedef struct {
  char name[32];          /* kernel name, e.g. "conv_fwd" */
  int32_t launches;       /* timed launches */
  double total_ms;        /* sum of the launch durations */
  double min_ms, max_ms;  /* shortest and longest launch */
} spect_kernel_time;

spect_status spect_profile_start(spect_plan plan, int32_t max_launches);
spect_status spect_profile_stop(spect_plan plan, spect_kernel_time* out, int32_t max_out,
                                int32_t* n_out);

/* Library version string. */
const char* spect_version(void);

/* The kernels a plan selected, as one line of key=value pairs written to buf
 * (NUL-terminated, truncated to len bytes): conv = fft | fp32-4x4 | fp32-16x16 |
 * fp32-direct (plain FP32 kernels, for PSFs taller than the matrix-core tiles
 * hold: pz >= 67) | separable | bf16 | fp16 | bf16x3, mirror = 1 when the FP32 4x4-block
 * convolution pairs mirror-image taps (see spect_plan_create), rotation =
 * 3pass | bilinear, view_batch, nchunk, rot_views (views per workgroup of
 * the forward rotation); with SPECT_CONV_FFT also fft_size = LxxLz (the
 * transform size) and fft_fixed (nonzero when kernels compiled for that size
 * run).  Host only. */
spect_status spect_plan_describe(spect_plan plan, char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* SPECT_H_ */
