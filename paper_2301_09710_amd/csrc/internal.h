// Internal declarations shared by the host code and the kernel files of
// libspect.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "spect.h"

namespace spect {

// Largest in-plane size for which two z-slices (n rows of stride n + 1
// floats), the scan segments and the per-view tables fit in the 160 KiB LDS
// of a gfx950 CU.
constexpr int kMaxLdsN = 136;
// Largest in-plane size: beyond kMaxLdsN the rotation kernels keep their
// working slices in global scratch (one per workgroup) instead of LDS.
constexpr int kMaxN = 256;
// Threads per workgroup of the rotation kernels.
constexpr int kRotThreads = 1024;
// Depth planes per workgroup (one partial sum each) of the forward convolution.
constexpr int kFwdJChunk = 16;
// Depth planes per workgroup of the adjoint convolution.
constexpr int kBackJChunk = 16;
// View groups (partial volumes) of the back rotation.
constexpr int kBackGroups = 16;
// Views a rotation workgroup processes for its slice.
constexpr int kRotViewsPerGroup = 8;
// Largest number of 4-deep k-steps of the MFMA convolution (pz <= 65).
constexpr int kMaxMfmaKSteps = 20;
// Largest number of depth chunks (forward partial sums) per tile and view.
constexpr int kMaxChunks = 16;
// LDS of one gfx950 compute unit.
constexpr size_t kLdsBytes = 163840;

// Tiling of the MFMA convolution (see conv_mfma.hip).
struct ConvShape {
  int nx, ny, nz, px, pz, ha, hb;
  int KS;               // k-steps per 16-row M-block: ceil((15 + pz) / 4)
  int WK, WI;           // waves of a workgroup along k and along i (WK * WI = 4)
  int tiles_k, tiles_i; // workgroup tiles of 16 WK x 32 WI output bins
  int RK, RI;           // staged region rows (k) and columns (i)
  int RSI, RSI_back;    // LDS row strides (forward, adjoint)
  int PL, Z;            // PSF row length in LDS and its zero offset (forward)
  int jc, nchunk;       // forward depth chunk
  int jc_back, nchunk_back;
};

// Tiling of the FP32 convolution on 4x4 matrix blocks (see conv_m4.hip).
struct M4Shape {
  int nx, ny, nz, px, pz, ha, hb;
  int ND4;              // steps per tap / 4: ceil((pz + 3) / 4)
  bool mirror;          // PSF rows symmetric in x: taps a and px-1-a share one product
  int BZ, BX;           // blocks of a wave along z and x (BZ * BX = 16)
  int WZ, WX;           // waves of a workgroup along z and x (WZ * WX = 8)
  int TH, TW;           // workgroup tile: 20 BZ WZ x 4 BX WX output bins
  int tiles_k, tiles_i; // workgroup tiles along z and x
  int RR, RC, RRS;      // region rows (z), columns (x), column stride in LDS
  int PL4;              // PSF column length in LDS
  int nchunk, nchunk_back;
  bool ok;              // the tiling fits the kernels' register and LDS budgets
};

// Tiling of the separable (rank-1) PSF convolution (see conv_sep.hip).
struct SepShape {
  int nx, ny, nz, px, pz, ha, hb;
  int NBx, NBz;         // tap counts rounded up to 4
  int nx8;              // nx rounded up to 8
  int ZS, nstrip;       // output rows (z) per workgroup strip, strips per plane
  int nchunk, nchunk_back;
  bool ok;              // the strips fit LDS and the forward's register-held outputs
};

// Tiling of the BF16 / FP16 convolution (see conv_lp.hip).
constexpr int kLpMaxWaves = 8;   // M-blocks (16 z each) per workgroup tile at most
struct LpShape {
  int nx, ny, nz, px, pz, ha, hb;
  int WKm, NN;            // M-blocks per tile; waves per workgroup (32 x bins each)
  int tiles_k, tiles_i;   // workgroup tiles of 16 WKm x 32 NN output bins
  int C7, ntq, NR;        // 8-row chunks per tap band, tap quads, region chunks
  int RR, RS, RC;         // region rows used, column stride (elements), columns used
  int dx, RCa;            // column shift aligning the region origin to 4; columns staged
  int QL;                 // PSF pair-table row length (words)
  int nchunk, nchunk_back;// depth chunks (forward, adjoint)
};

// Transform sizes and pass radices of the FFT convolution (see conv_fft.hip).
constexpr int kMaxFftPass = 12;
struct FftShape {
  int nx, ny, nz, px, pz, ha, hb;
  int Lx, Lz;             // transform sizes (even, factors 2, 3, 5) >= padded plane
  int Lh, H;              // Lx / 2, Lz / 2
  int stride;             // row stride of the LDS plane (complex elements)
  int nrx, nrz;           // passes along x and z
  int rx[kMaxFftPass], rz[kMaxFftPass];
  int NR, NS;             // regular spectrum slots, all slots (complex) per plane
  float r_lx, r_lh, r_lh1, r_nx;  // 1 / Lx, 1 / Lh, 1 / (Lh - 1), 1 / nx
  int nchunk, nchunk_back;
  int cfg;                // transform sizes fixed at compile time (conv_fft_fixed.hip), 0: none
  bool real;              // PSFs symmetric in x and z (flags), fixed sizes: real spectra
  bool ok;                // fits the kernels' registers and LDS
};
// The FFT convolution's kernels (launch_fft_fixed's `which`).
enum FftKernel { kFftSpectra = 0, kFftForward, kFftFinish, kFftBackPrep, kFftBack };

// Per-view geometry tables, on the device (inside the workspace).
//   quarter[l]             : m, number of quarter turns (0..3)
//   off[l][0][j], w[l][0][j]: passes 1 and 3 (along i, one entry per row j)
//   off[l][1][i], w[l][1][i]: pass 2 (along j, one entry per column i)
// A pass computes out[q] = w.x * in[q + off] + w.y * in[q + off + 1], zero
// outside [0, n); w.x = 1 - f and w.y = f of the fractional shift.
// Per-view rotation tables in the workspace.  Each of the 2n entries of a
// view holds two integers (off) and two floats (w):
//   3-pass shears: (offset, 0) and the two tap weights of a row (entries
//     [0, n), passes 1 and 3) or column (entries [n, 2n), pass 2);
//   bilinear: integer parts and fractions of the sample position's terms,
//     s = (c + cos (i - c) + sin (j - c), c - sin (i - c) + cos (j - c)),
//     split as a row term in j (entries [0, n)) plus a column term in i
//     (entries [n, 2n)).
// rot[l] = (cos phi, sin phi) of the residual angle.
struct Tables {
  const int32_t* quarter;
  const int32_t* off;     // nview x 2n x 2
  const float2* w;        // nview x 2n
  const float2* rot;      // nview
};

// Workspace layout (byte offsets from the workspace base, 256-B aligned).
struct Layout {
  size_t tables_quarter, tables_off, tables_w, tables_rot;
  size_t vol_batch;     // view_batch * N floats: W (forward) / U (back)
  size_t fwd_partial;   // nchunk * view_batch * nz * nx floats
  size_t back_partial;  // kBackGroups * N floats
  size_t mubar_cache;   // nview * N floats (only with SPECT_CACHE_MUBAR)
  size_t mubar_batch;   // view_batch * N floats (only without SPECT_CACHE_MUBAR)
  size_t em_proj;       // nview * nz * nx floats
  size_t em_vol;        // N floats
  size_t rot_scratch;   // working slices of the rotation kernels when nx > kMaxLdsN
  size_t em_proj2;      // nview * nz * nx floats (EM vector-Jacobian product)
  size_t em_vol2;       // N floats (EM vector-Jacobian product)
  size_t fft_tables;    // 2 Lx + Lz ints: transform index tables (SPECT_CONV_FFT)
  size_t fft_spectra;   // nview * ny * NS complex: PSF spectra (SPECT_CONV_FFT)
  size_t fft_part;      // nchunk * view_batch * NS complex: forward partial spectra
  size_t fft_vproj;     // view_batch * NS complex: projection spectra (adjoint)
  size_t total;
};

// Kernel identities for the optional per-launch timing.
enum KernelId {
  K_MUBAR = 0, K_ROT_FWD, K_CONV_FWD, K_FWD_REDUCE, K_CONV_BACK, K_ROT_BACK,
  K_BACK_REDUCE, K_EM_RATIO, K_EM_UPDATE, K_CONV_BACK_EDGES, K_EM_VJP, K_CONV_FWD_LP,
  K_CONV_BACK_LP, K_EM_REG_UPDATE, K_PSF_SPECTRA, K_CONV_FWD_FFT, K_FWD_FFT_FINISH,
  K_BACK_FFT_PREP, K_CONV_BACK_FFT, K_COUNT
};
extern const char* const kKernelNames[K_COUNT];

struct Profiler {
  int cap = 0, used = 0;
  hipEvent_t* ev = nullptr;   // 2 * cap events
  int* kid = nullptr;         // cap kernel ids
};

struct Plan {
  spect_geom g;         // angles pointer cleared after creation
  int view_batch;
  int rot_fwd_vg;       // views per workgroup of the line-pass forward rotation
  int nchunk;           // forward depth chunks
  const float* mu;
  const float* psf;
  char* ws;
  Layout lay;
  Tables tab;
  const float* mubar;   // cache or nullptr
  float* mubar_batch;   // per-batch attenuation factors when not cached
  float* rot_scratch;   // rotation working slices (nx > kMaxLdsN), else nullptr
  bool use_mfma;        // MFMA convolution path (else the direct kernels)
  bool bilinear;         // SPECT_ROT_BILINEAR
  ConvShape conv;
  M4Shape m4;           // FP32 convolution on 4x4 blocks, used when use_m4
  bool use_m4;
  bool separable;       // SPECT_PSF_SEPARABLE: psf holds the two 1-D factors per plane
  SepShape sep;
  int conv_precision;   // SPECT_CONV_FP32 / _BF16 / _FP16
  LpShape lp;           // tiling of the reduced-precision convolution
  bool use_fft;         // SPECT_CONV_FFT: convolution through the FFT
  FftShape fft;
  Profiler* prof;       // non-null while spect_profile_start is active
  // host copies of the tables (kept alive for the asynchronous upload)
  int32_t* h_quarter;
  int32_t* h_off;
  float2* h_w;
  float2* h_rot;
};

// Run `launch` (which enqueues one kernel on s), bracketed by profiling
// events when the plan's profiler is active.
template <class F>
hipError_t timed(const Plan& p, KernelId id, hipStream_t s, F&& launch) {
  Profiler* pr = p.prof;
  const bool rec = pr && pr->used < pr->cap;
  if (rec && hipEventRecord(pr->ev[2 * pr->used], s) != hipSuccess) return hipErrorUnknown;
  hipError_t e = launch();
  if (rec && e == hipSuccess) {
    if (hipEventRecord(pr->ev[2 * pr->used + 1], s) != hipSuccess) return hipErrorUnknown;
    pr->kid[pr->used++] = id;
  }
  return e;
}

spect_status compute_layout(const spect_geom& g, Layout* lay, int* view_batch, int* nchunk);
// Kernel selection and tiling of a plan over the workspace ws (no device work
// beyond occupancy queries; the tables, the attenuation cache and the mirror
// check are the caller's).
void configure_plan(Plan& p, const spect_geom& g, const Layout& lay, int view_batch, int nchunk,
                    const float* d_mu, const float* d_psf, char* ws);
// The forward projection of Alg. 1 on a configured plan with its tables in place.
spect_status forward_impl(const Plan& p, const float* x, float* v, hipStream_t s);

// ---- per-view rotation tables (host and device) ----
// Default angles theta_l = 2 pi l / nview split exactly as theta = M pi/2 + phi,
// phi in [-pi/4, pi/4): M = floor((8 l + nview) / (2 nview)), m = M mod 4.
__host__ __device__ inline void split_default_view(int l, int nview, int* m, double* phi) {
  const long long M = (8LL * l + nview) / (2LL * nview);
  *phi = (3.14159265358979323846 / 2.0) * (double)(4LL * l - M * nview) / (double)nview;
  *m = (int)(((M % 4) + 4) % 4);
}

// Integer part and fraction of v, the fraction in [0, 1) after rounding to float.
__host__ __device__ inline void split_pos(double v, int32_t* ip, float* frac) {
  double fl = ::floor(v);
  float f = (float)(v - fl);
  if (f >= 1.0f) { f = 0.0f; fl += 1.0; }
  *ip = (int32_t)fl;
  *frac = f;
}

// Entry (ps, r) of one view's tables for the residual angle phi (see Tables):
// off2[0..1] and w of row/column r of pass group ps.
__host__ __device__ inline void table_entry(int n, bool bilinear, double phi, int ps, int r,
                                            int32_t* off2, float2* w) {
  const double c = (n - 1) / 2.0;
  const double u = (double)r - c;
  if (bilinear) {
    const double s = ::sin(phi), co = ::cos(phi);
    // ps 0: row term (index j = r), ps 1: column term (index i = r)
    const double ti = ps == 0 ? s * u : c + co * u;
    const double tj = ps == 0 ? c + co * u : -s * u;
    float fi, fj;
    split_pos(ti, &off2[0], &fi);
    split_pos(tj, &off2[1], &fj);
    *w = make_float2(fi, fj);
  } else {
    // passes 1, 3: shift along i for row j = r; pass 2: shift along j for column i = r
    const double d = ps == 0 ? ::tan(phi / 2.0) * u : -::sin(phi) * u;
    const double fl = ::floor(d);
    const double f = d - fl;
    off2[0] = (int32_t)fl;
    off2[1] = 0;
    *w = make_float2((float)(1.0 - f), (float)f);
  }
}

bool conv_mfma_supported(const spect_geom& g);
ConvShape make_conv_shape(const spect_geom& g, int jc_fwd, int jc_back);
// Choose the depth chunking of the MFMA convolution for `views` views per
// launch from the device's CU count and the kernels' occupancy.
void tune_conv_chunks(ConvShape& cs, int views);
size_t conv_mfma_lds_bytes(const ConvShape& cs, bool back);
size_t conv_edges_lds_bytes(const ConvShape& cs);
M4Shape make_m4_shape(const spect_geom& g);
// Whether the 4x4-block tiling issues fewer matrix-core cycles than the 16x16 one.
bool m4_preferred(const M4Shape& s, const ConvShape& cs);
void tune_m4_chunks(M4Shape& s, int views);
// Sets p.m4.mirror: whether every PSF row equals its mirror image in x
// (checked on the device with the 4-byte scratch d_flag; waits for st).
hipError_t detect_m4_mirror(Plan& p, int* d_flag, hipStream_t st);
SepShape make_sep_shape(const spect_geom& g);
size_t sep_lds_bytes(const SepShape& s, bool back);
void tune_sep_chunks(SepShape& s, int views);
LpShape make_lp_shape(const spect_geom& g);
size_t lp_lds_bytes(const LpShape& s, bool split);
bool lp_supported(const spect_geom& g);
void tune_lp_chunks(LpShape& s, int views, int precision);
size_t rotation_lds_bytes(int n);
// Views per workgroup of the forward rotation for batches of nvb views:
// whole rounds of the resident workgroup slots, few views per workgroup.
int tune_rot_fwd_views(const spect_geom& g, int nvb);
size_t rotation_scratch_bytes(int n, int nz, int nview);

// ---- kernel launchers (return hipGetLastError() of the launch) ----
hipError_t launch_mubar(const Plan& p, float* out, int view0, int nviews, int out_view0,
                        hipStream_t s);
hipError_t launch_rot_fwd(const Plan& p, const float* x, const float* mb, int mb_off, float* W,
                          int view0, int nvb, hipStream_t s);
hipError_t launch_conv_fwd_mfma(const Plan& p, const float* W, float* partial, int view0, int nvb,
                                hipStream_t s);
hipError_t launch_conv_back_mfma(const Plan& p, const float* v, float* U, int view0, int nvb,
                                 hipStream_t s);
hipError_t launch_conv_m4(const Plan& p, bool back, const float* in, float* out, int view0,
                          int nvb, hipStream_t s);
hipError_t launch_conv_sep(const Plan& p, bool back, const float* in, float* out, int view0,
                           int nvb, hipStream_t s);
hipError_t launch_conv_back_edges(const Plan& p, const float* v, float* U, int view0, int nvb,
                                  hipStream_t s);
hipError_t launch_conv_fwd(const Plan& p, const float* W, float* partial, int view0, int nvb,
                           hipStream_t s);
hipError_t launch_fwd_reduce(const Plan& p, const float* partial, float* v, int view0, int nvb,
                             hipStream_t s);
hipError_t launch_conv_back(const Plan& p, const float* v, float* U, int view0, int nvb,
                            hipStream_t s);
hipError_t launch_rot_back(const Plan& p, const float* U, const float* mb, int mb_off,
                           float* partial, int view0, int nvb, bool accumulate, hipStream_t s);
hipError_t launch_back_reduce(const Plan& p, const float* partial, float* x, hipStream_t s);
hipError_t launch_em_ratio(const float* v, const float* y, const float* r, float* rho, size_t m,
                           hipStream_t s);
hipError_t launch_em_update(float* x, const float* e, const float* sens, size_t n, hipStream_t s);
hipError_t launch_conv_fwd_lp(const Plan& p, const float* W, float* partial, int view0, int nvb,
                              hipStream_t s);
hipError_t launch_conv_back_lp(const Plan& p, const float* v, float* U, int view0, int nvb,
                               hipStream_t s);
hipError_t launch_em_vjp_prep(const float* g, const float* x, const float* b, const float* sens,
                              float* gb, float* gx, size_t n, hipStream_t s);
hipError_t launch_em_vjp_ratio(float* t, const float* v, const float* y, const float* r, float* gy,
                               size_t m, hipStream_t s);
hipError_t launch_add(float* a, const float* b, size_t n, hipStream_t s);
hipError_t launch_em_reg_update(float* x, const float* e, const float* sens, const float* u,
                                float beta, size_t n, hipStream_t s);
FftShape make_fft_shape(const spect_geom& g);
// Which compile-time configuration holds these transform sizes (0: none).
int fft_fixed_config(const FftShape& s);
hipError_t launch_fft_fixed(const Plan& p, int which, const void* in, void* out, int view0, int nvb,
                            hipStream_t s);
void tune_fft_chunks(FftShape& s, int views);
hipError_t launch_fft_psf_spectra(const Plan& p, hipStream_t s);
hipError_t launch_conv_fwd_fft(const Plan& p, const float* W, int view0, int nvb, hipStream_t s);
hipError_t launch_fwd_fft_finish(const Plan& p, float* v, int view0, int nvb, hipStream_t s);
hipError_t launch_back_fft_prep(const Plan& p, const float* v, int view0, int nvb, hipStream_t s);
hipError_t launch_conv_back_fft(const Plan& p, float* U, int view0, int nvb, hipStream_t s);
hipError_t launch_dot_f64(const float* a, const float* b, size_t n, double* out, hipStream_t s);

}  // namespace spect
