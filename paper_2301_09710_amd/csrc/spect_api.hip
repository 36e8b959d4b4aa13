// C ABI of libspect: plan creation (host FP64 geometry tables, workspace
// layout, argument validation) and the entry points that chain the kernels.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "internal.h"

namespace spect {

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static spect_status validate(const spect_geom* g) {
  if (!g) return SPECT_ERR_NULL;
  if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nview < 1 || g->px < 1 || g->pz < 1)
    return SPECT_ERR_SHAPE;
  if (g->nx != g->ny) return SPECT_ERR_SHAPE;              // rotation about z needs a square slice
  if ((g->px & 1) == 0 || (g->pz & 1) == 0) return SPECT_ERR_SHAPE;  // centred odd kernels
  if (!(std::isfinite(g->dy) && g->dy > 0.0)) return SPECT_ERR_VALUE;
  if (g->flags & ~(SPECT_CACHE_MUBAR | SPECT_ROT_BILINEAR | SPECT_PSF_SEPARABLE |
                   SPECT_PSF_ALL_TAPS | SPECT_PSF_SYMMETRIC_X | SPECT_TILING_4X4 |
                   SPECT_TILING_16X16 | SPECT_CONV_FFT | SPECT_PSF_SYMMETRIC_Z))
    return SPECT_ERR_VALUE;
  if ((g->flags & SPECT_PSF_ALL_TAPS) && (g->flags & SPECT_PSF_SYMMETRIC_X)) return SPECT_ERR_VALUE;
  if ((g->flags & SPECT_TILING_4X4) && (g->flags & SPECT_TILING_16X16)) return SPECT_ERR_VALUE;
  if (g->view_batch < 0) return SPECT_ERR_VALUE;
  if (g->conv_precision != SPECT_CONV_FP32 && g->conv_precision != SPECT_CONV_BF16 &&
      g->conv_precision != SPECT_CONV_FP16 && g->conv_precision != SPECT_CONV_BF16X3)
    return SPECT_ERR_VALUE;
  if (g->angles)
    for (int l = 0; l < g->nview; ++l)
      if (!std::isfinite(g->angles[l])) return SPECT_ERR_VALUE;
  if (g->nx > kMaxN) return SPECT_ERR_UNSUPPORTED;
  // index arithmetic inside a plane / slice uses 32-bit ints
  if ((int64_t)g->nx * g->nz > (1 << 30) || (int64_t)g->px * g->pz > (1 << 20))
    return SPECT_ERR_UNSUPPORTED;
  if (g->flags & SPECT_CONV_FFT) {
    // the FFT form: FP32, general PSFs, planes whose transforms fit LDS
    if (g->conv_precision != SPECT_CONV_FP32 || (g->flags & SPECT_PSF_SEPARABLE) ||
        !make_fft_shape(*g).ok)
      return SPECT_ERR_UNSUPPORTED;
  }
  if (g->flags & SPECT_PSF_SEPARABLE) {
    // separable PSFs: FP32 1-D passes only
    if (g->conv_precision != SPECT_CONV_FP32 || !make_sep_shape(*g).ok) return SPECT_ERR_UNSUPPORTED;
  } else if (g->conv_precision != SPECT_CONV_FP32 &&
             !(lp_supported(*g) && conv_mfma_supported(*g))) {
    // the reduced-precision convolution needs its LDS tiles and the FP32 edge fold
    return SPECT_ERR_UNSUPPORTED;
  }
  return SPECT_OK;
}

spect_status compute_layout(const spect_geom& g, Layout* lay, int* view_batch, int* nchunk) {
  spect_status st = validate(&g);
  if (st != SPECT_OK) return st;
  const size_t n = (size_t)g.nx;
  const size_t N = n * g.ny * g.nz;
  const size_t M = (size_t)g.nview * g.nz * g.nx;
  const int vb = (g.view_batch > 0 && g.view_batch < g.nview) ? g.view_batch : g.nview;
  const int nc = (g.ny + kFwdJChunk - 1) / kFwdJChunk;   // same chunking for both conv paths
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t at = off; off += align256(bytes); return at; };
  lay->tables_quarter = take((size_t)g.nview * sizeof(int32_t));
  lay->tables_off = take((size_t)g.nview * 2 * n * 2 * sizeof(int32_t));
  lay->tables_w = take((size_t)g.nview * 2 * n * sizeof(float2));
  lay->tables_rot = take((size_t)g.nview * sizeof(float2));
  lay->vol_batch = take((size_t)vb * N * sizeof(float));
  const int maxc = nc > kMaxChunks ? nc : kMaxChunks;
  lay->fwd_partial = take((size_t)maxc * vb * g.nz * g.nx * sizeof(float));
  lay->back_partial = take((size_t)kBackGroups * N * sizeof(float));
  const bool cache = (g.flags & SPECT_CACHE_MUBAR) != 0;
  lay->mubar_cache = cache ? take((size_t)g.nview * N * sizeof(float)) : 0;
  lay->mubar_batch = cache ? 0 : take((size_t)vb * N * sizeof(float));

  lay->rot_scratch = take(rotation_scratch_bytes(g.nx, g.nz, g.nview));
  lay->em_proj = take(M * sizeof(float));
  lay->em_vol = take(N * sizeof(float));
  lay->em_proj2 = take(M * sizeof(float));
  lay->em_vol2 = take(N * sizeof(float));
  lay->fft_tables = lay->fft_spectra = lay->fft_part = lay->fft_vproj = 0;
  if (g.flags & SPECT_CONV_FFT) {
    const FftShape fs = make_fft_shape(g);
    const size_t ns = (size_t)fs.NS * sizeof(float2);
    lay->fft_tables = take((size_t)(2 * fs.Lx + fs.Lz) * sizeof(int));
    lay->fft_spectra = take((size_t)g.nview * g.ny * fs.NS * (fs.real ? sizeof(float) : sizeof(float2)));
    lay->fft_part = take((size_t)kMaxChunks * vb * ns);
    lay->fft_vproj = take((size_t)vb * ns);
  }
  lay->total = off;
  *view_batch = vb;
  *nchunk = nc;
  return SPECT_OK;
}

// theta = M pi/2 + phi, phi in [-pi/4, pi/4); integer rule for default angles.
static void split_view(const spect_geom& g, int l, int* m, double* phi) {
  if (!g.angles) {
    split_default_view(l, g.nview, m, phi);
    return;
  }
  const double th = g.angles[l];
  const long long M = (long long)std::floor(th / (M_PI / 2.0) + 0.5);
  *phi = th - (double)M * (M_PI / 2.0);
  *m = (int)(((M % 4) + 4) % 4);
}

static void fill_tables(const spect_geom& g, int32_t* q, int32_t* off, float2* w, float2* rot) {
  const int n = g.nx;
  const bool bil = (g.flags & SPECT_ROT_BILINEAR) != 0;
  for (int l = 0; l < g.nview; ++l) {
    int m;
    double phi;
    split_view(g, l, &m, &phi);
    q[l] = m;
    rot[l] = make_float2((float)std::cos(phi), (float)std::sin(phi));
    for (int r = 0; r < n; ++r)
      for (int ps = 0; ps < 2; ++ps) {
        const size_t e = ((size_t)l * 2 + ps) * n + r;
        table_entry(n, bil, phi, ps, r, &off[2 * e], &w[e]);
      }
  }
}

}  // namespace spect

namespace spect {
const char* const kKernelNames[K_COUNT] = {"mubar", "rot_fwd",  "conv_fwd",
                                           "fwd_reduce",  "conv_back", "rot_back",
                                           "back_reduce", "em_ratio", "em_update",
                                           "conv_back_edges", "em_vjp", "conv_fwd_lp",
                                           "conv_back_lp", "em_reg_update", "psf_spectra",
                                           "conv_fwd_fft", "fwd_fft_finish", "back_fft_prep",
                                           "conv_back_fft"};

static void profiler_free(Profiler* pr) {
  if (!pr) return;
  if (pr->ev)
    for (int i = 0; i < 2 * pr->cap; ++i)
      if (pr->ev[i]) (void)hipEventDestroy(pr->ev[i]);
  std::free(pr->ev);
  std::free(pr->kid);
  delete pr;
}
}  // namespace spect

namespace spect {

void configure_plan(Plan& p_, const spect_geom& g_, const Layout& lay, int vb, int nc,
                    const float* d_mu, const float* d_psf, char* ws) {
  Plan* p = &p_;
  const spect_geom* g = &g_;
  p->g = *g;
  p->g.angles = nullptr;
  p->view_batch = vb;
  p->nchunk = nc;
  p->mu = d_mu;
  p->psf = d_psf;
  p->ws = ws;
  p->lay = lay;
  p->prof = nullptr;
  p->bilinear = (g->flags & SPECT_ROT_BILINEAR) != 0;
  p->tab.quarter = reinterpret_cast<const int32_t*>(p->ws + lay.tables_quarter);
  p->tab.off = reinterpret_cast<const int32_t*>(p->ws + lay.tables_off);
  p->tab.w = reinterpret_cast<const float2*>(p->ws + lay.tables_w);
  p->tab.rot = reinterpret_cast<const float2*>(p->ws + lay.tables_rot);
  p->mubar = nullptr;
  p->mubar_batch = nullptr;
  p->rot_scratch = g->nx > kMaxLdsN ? reinterpret_cast<float*>(p->ws + lay.rot_scratch) : nullptr;
  p->rot_fwd_vg = tune_rot_fwd_views(*g, vb);
  p->use_mfma = conv_mfma_supported(*g);
  p->conv = make_conv_shape(*g, kFwdJChunk, kBackJChunk);
  p->m4 = make_m4_shape(*g);
  p->use_m4 = false;
  p->separable = (g->flags & SPECT_PSF_SEPARABLE) != 0;
  if (p->separable) {
    p->use_mfma = false;
    p->sep = make_sep_shape(*g);
    tune_sep_chunks(p->sep, g->nview);
    p->nchunk = p->sep.nchunk;
  } else if (p->use_mfma) {
    tune_conv_chunks(p->conv, g->nview);   // independent of view_batch: same sums
    p->nchunk = p->conv.nchunk;          // forward partial sums per view
    // SPECT_TILING_4X4 / SPECT_TILING_16X16 override the cost model
    bool m4 = m4_preferred(p->m4, p->conv);
    if (g->flags & SPECT_TILING_4X4) m4 = p->m4.ok;
    if (g->flags & SPECT_TILING_16X16) m4 = false;
    if (m4) {
      tune_m4_chunks(p->m4, g->nview);
      p->use_m4 = true;
      p->nchunk = p->m4.nchunk;
    }
  }
  p->conv_precision = g->conv_precision;
  if (p->conv_precision != SPECT_CONV_FP32) {
    p->lp = make_lp_shape(*g);
    tune_lp_chunks(p->lp, g->nview, p->conv_precision);
    p->nchunk = p->lp.nchunk;
  }
  p->use_fft = (g->flags & SPECT_CONV_FFT) != 0;
  if (p->use_fft) {
    p->use_mfma = p->use_m4 = false;
    p->fft = make_fft_shape(*g);
    tune_fft_chunks(p->fft, vb);
    p->nchunk = p->fft.nchunk;
  }
  if (!(g->flags & SPECT_CACHE_MUBAR))
    p->mubar_batch = reinterpret_cast<float*>(p->ws + lay.mubar_batch);
}

}  // namespace spect

using namespace spect;

// Attenuation factors of views [v0, v0 + nvb): the cache (computed at plan
// creation) or the batch buffer, filled here.  Returns the base pointer and
// the view offset to add to a batch-relative view index.
static hipError_t mubar_for_batch(const Plan& p, int v0, int nvb, hipStream_t s,
                                  const float** mb, int* off) {
  if (p.mubar) {
    *mb = p.mubar;
    *off = v0;
    return hipSuccess;
  }
  *mb = p.mubar_batch;
  *off = 0;
  return timed(p, K_MUBAR, s, [&] { return launch_mubar(p, p.mubar_batch, v0, nvb, v0, s); });
}

spect_status spect::forward_impl(const Plan& p, const float* x, float* v, hipStream_t s) {
  float* W = reinterpret_cast<float*>(p.ws + p.lay.vol_batch);
  float* part = reinterpret_cast<float*>(p.ws + p.lay.fwd_partial);
  for (int v0 = 0; v0 < p.g.nview; v0 += p.view_batch) {
    const int nvb = (p.g.nview - v0 < p.view_batch) ? p.g.nview - v0 : p.view_batch;
    const float* mb;
    int mb_off;
    if (mubar_for_batch(p, v0, nvb, s, &mb, &mb_off) != hipSuccess) return SPECT_ERR_HIP;
    if (timed(p, K_ROT_FWD, s, [&] { return launch_rot_fwd(p, x, mb, mb_off, W, v0, nvb, s); }) !=
        hipSuccess)
      return SPECT_ERR_HIP;
    if (p.use_fft) {
      if (timed(p, K_CONV_FWD_FFT, s, [&] { return launch_conv_fwd_fft(p, W, v0, nvb, s); }) !=
              hipSuccess ||
          timed(p, K_FWD_FFT_FINISH, s, [&] { return launch_fwd_fft_finish(p, v, v0, nvb, s); }) !=
              hipSuccess)
        return SPECT_ERR_HIP;
      continue;
    }
    const hipError_t ec =
        p.conv_precision != SPECT_CONV_FP32
            ? timed(p, K_CONV_FWD_LP, s, [&] { return launch_conv_fwd_lp(p, W, part, v0, nvb, s); })
            : timed(p, K_CONV_FWD, s, [&] {
                if (p.separable) return launch_conv_sep(p, false, W, part, v0, nvb, s);
                return p.use_mfma ? launch_conv_fwd_mfma(p, W, part, v0, nvb, s)
                                  : launch_conv_fwd(p, W, part, v0, nvb, s);
              });
    if (ec != hipSuccess) return SPECT_ERR_HIP;
    if (timed(p, K_FWD_REDUCE, s, [&] { return launch_fwd_reduce(p, part, v, v0, nvb, s); }) !=
        hipSuccess)
      return SPECT_ERR_HIP;
  }
  return SPECT_OK;
}

static spect_status back_impl(const Plan& p, const float* v, float* x, hipStream_t s) {
  float* U = reinterpret_cast<float*>(p.ws + p.lay.vol_batch);
  float* part = reinterpret_cast<float*>(p.ws + p.lay.back_partial);
  for (int v0 = 0; v0 < p.g.nview; v0 += p.view_batch) {
    const int nvb = (p.g.nview - v0 < p.view_batch) ? p.g.nview - v0 : p.view_batch;
    const hipError_t ec =
        p.use_fft
            ? (timed(p, K_BACK_FFT_PREP, s, [&] { return launch_back_fft_prep(p, v, v0, nvb, s); }) !=
                       hipSuccess
                   ? hipErrorUnknown
                   : timed(p, K_CONV_BACK_FFT, s, [&] { return launch_conv_back_fft(p, U, v0, nvb, s); }))
        : p.conv_precision != SPECT_CONV_FP32
            ? timed(p, K_CONV_BACK_LP, s, [&] { return launch_conv_back_lp(p, v, U, v0, nvb, s); })
            : timed(p, K_CONV_BACK, s, [&] {
                if (p.separable) return launch_conv_sep(p, true, v, U, v0, nvb, s);  // folds included
                return p.use_mfma ? launch_conv_back_mfma(p, v, U, v0, nvb, s)
                                  : launch_conv_back(p, v, U, v0, nvb, s);
              });
    if (ec != hipSuccess) return SPECT_ERR_HIP;
    if (p.use_mfma &&
        timed(p, K_CONV_BACK_EDGES, s,
              [&] { return launch_conv_back_edges(p, v, U, v0, nvb, s); }) != hipSuccess)
      return SPECT_ERR_HIP;
    const float* mb;
    int mb_off;
    if (mubar_for_batch(p, v0, nvb, s, &mb, &mb_off) != hipSuccess) return SPECT_ERR_HIP;
    if (timed(p, K_ROT_BACK, s, [&] {
          return launch_rot_back(p, U, mb, mb_off, part, v0, nvb, v0 > 0, s);
        }) != hipSuccess)
      return SPECT_ERR_HIP;
  }
  if (timed(p, K_BACK_REDUCE, s, [&] { return launch_back_reduce(p, part, x, s); }) != hipSuccess)
    return SPECT_ERR_HIP;
  return SPECT_OK;
}

extern "C" {

const char* spect_version(void) { return "libspect 0.1 (gfx950)"; }

spect_status spect_plan_describe(spect_plan plan, char* buf, size_t len) {
  if (!plan || !buf) return SPECT_ERR_NULL;
  if (len == 0) return SPECT_ERR_VALUE;
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  static const char* const kLp[] = {"fp32", "bf16", "fp16", "bf16x3"};
  const char* conv = p->use_fft ? "fft"
                     : p->separable ? "separable"
                     : p->conv_precision != SPECT_CONV_FP32 ? kLp[p->conv_precision & 3]
                     : p->use_m4    ? "fp32-4x4"
                     : p->use_mfma  ? "fp32-16x16"
                                    : "fp32-direct";
  const bool mirror = p->use_m4 && p->conv_precision == SPECT_CONV_FP32 && p->m4.mirror;
  int n = std::snprintf(buf, len, "conv=%s mirror=%d rotation=%s view_batch=%d nchunk=%d rot_views=%d",
                        conv, mirror ? 1 : 0, p->bilinear ? "bilinear" : "3pass", p->view_batch,
                        p->nchunk, p->rot_fwd_vg);
  if (p->use_fft && n > 0 && (size_t)n < len)
    std::snprintf(buf + n, len - n, " fft_size=%dx%d fft_fixed=%d fft_real=%d", p->fft.Lx,
                  p->fft.Lz, p->fft.cfg, p->fft.real ? 1 : 0);
  return SPECT_OK;
}

const char* spect_status_string(spect_status s) {
  switch (s) {
    case SPECT_OK: return "ok";
    case SPECT_ERR_NULL: return "null pointer argument";
    case SPECT_ERR_SHAPE: return "invalid shape (nx != ny, non-positive size or even PSF size)";
    case SPECT_ERR_VALUE: return "invalid value (dy, angles, flags or view_batch)";
    case SPECT_ERR_WORKSPACE: return "workspace too small";
    case SPECT_ERR_UNSUPPORTED: return "size not supported by this build";
    case SPECT_ERR_HIP: return "HIP runtime error";
    case SPECT_ERR_ALIGN: return "misaligned device pointer";
  }
  return "unknown status";
}

spect_status spect_workspace_bytes(const spect_geom* g, size_t* bytes) {
  if (!g || !bytes) return SPECT_ERR_NULL;
  Layout lay;
  int vb, nc;
  spect_status st = compute_layout(*g, &lay, &vb, &nc);
  if (st != SPECT_OK) return st;
  *bytes = lay.total;
  return SPECT_OK;
}

static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

spect_status spect_plan_create(spect_plan* out, const spect_geom* g, const float* d_mu,
                               const float* d_psf, void* d_workspace, size_t ws_bytes,
                               hipStream_t stream) {
  if (!out || !g || !d_mu || !d_psf || !d_workspace) return SPECT_ERR_NULL;
  *out = nullptr;
  Layout lay;
  int vb, nc;
  spect_status st = compute_layout(*g, &lay, &vb, &nc);
  if (st != SPECT_OK) return st;
  if (!aligned(d_workspace, 256) || !aligned(d_mu, 4) || !aligned(d_psf, 4)) return SPECT_ERR_ALIGN;
  if (ws_bytes < lay.total) return SPECT_ERR_WORKSPACE;

  Plan* p = new (std::nothrow) Plan();
  if (!p) return SPECT_ERR_HIP;
  configure_plan(*p, *g, lay, vb, nc, d_mu, d_psf, static_cast<char*>(d_workspace));
  const size_t n = (size_t)g->nx;
  p->h_quarter = static_cast<int32_t*>(std::malloc(g->nview * sizeof(int32_t)));
  p->h_off = static_cast<int32_t*>(std::malloc(g->nview * 2 * n * 2 * sizeof(int32_t)));
  p->h_w = static_cast<float2*>(std::malloc(g->nview * 2 * n * sizeof(float2)));
  p->h_rot = static_cast<float2*>(std::malloc(g->nview * sizeof(float2)));
  if (!p->h_quarter || !p->h_off || !p->h_w || !p->h_rot) {
    spect_plan_destroy(reinterpret_cast<spect_plan>(p));
    return SPECT_ERR_HIP;
  }
  fill_tables(*g, p->h_quarter, p->h_off, p->h_w, p->h_rot);
  hipError_t e = hipMemcpyAsync(p->ws + lay.tables_quarter, p->h_quarter,
                                g->nview * sizeof(int32_t), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->ws + lay.tables_off, p->h_off, g->nview * 2 * n * 2 * sizeof(int32_t),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->ws + lay.tables_w, p->h_w, g->nview * 2 * n * sizeof(float2),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->ws + lay.tables_rot, p->h_rot, g->nview * sizeof(float2),
                       hipMemcpyHostToDevice, stream);
  // PSF rows symmetric in x (a centred Gaussian, any circularly symmetric
  // response): the 4x4-block kernels pair taps a and px-1-a.  Checked exactly
  // on the device unless the caller states the symmetry (SPECT_PSF_SYMMETRIC_X)
  // or asks for every tap (SPECT_PSF_ALL_TAPS).
  if (e == hipSuccess && p->use_m4 && p->conv_precision == SPECT_CONV_FP32) {
    if (g->flags & SPECT_PSF_SYMMETRIC_X)
      p->m4.mirror = true;
    else if (!(g->flags & SPECT_PSF_ALL_TAPS))
      e = detect_m4_mirror(*p, reinterpret_cast<int*>(p->ws + lay.em_vol), stream);
  }
  if (e == hipSuccess && p->use_fft)
    e = timed(*p, K_PSF_SPECTRA, stream, [&] { return launch_fft_psf_spectra(*p, stream); });
  if (g->flags & SPECT_CACHE_MUBAR) {
    float* cache = reinterpret_cast<float*>(p->ws + lay.mubar_cache);
    if (e == hipSuccess)
      e = timed(*p, K_MUBAR, stream,
                [&] { return launch_mubar(*p, cache, 0, g->nview, 0, stream); });
    p->mubar = cache;
  }
  if (e != hipSuccess) {
    // make sure no queued copy still reads the host tables before freeing them
    (void)hipStreamSynchronize(stream);
    spect_plan_destroy(reinterpret_cast<spect_plan>(p));
    return SPECT_ERR_HIP;
  }
  *out = reinterpret_cast<spect_plan>(p);
  return SPECT_OK;
}

spect_status spect_plan_destroy(spect_plan plan) {
  if (!plan) return SPECT_ERR_NULL;
  Plan* p = reinterpret_cast<Plan*>(plan);
  profiler_free(p->prof);
  std::free(p->h_quarter);
  std::free(p->h_off);
  std::free(p->h_w);
  std::free(p->h_rot);
  delete p;
  return SPECT_OK;
}


spect_status spect_forward(spect_plan plan, const float* d_x, float* d_v, hipStream_t stream) {
  if (!plan || !d_x || !d_v) return SPECT_ERR_NULL;
  if (!aligned(d_x, 4) || !aligned(d_v, 4)) return SPECT_ERR_ALIGN;
  return forward_impl(*reinterpret_cast<Plan*>(plan), d_x, d_v, stream);
}

spect_status spect_back(spect_plan plan, const float* d_v, float* d_x, hipStream_t stream) {
  if (!plan || !d_v || !d_x) return SPECT_ERR_NULL;
  if (!aligned(d_x, 4) || !aligned(d_v, 4)) return SPECT_ERR_ALIGN;
  return back_impl(*reinterpret_cast<Plan*>(plan), d_v, d_x, stream);
}

spect_status spect_em_step(spect_plan plan, float* d_x, const float* d_y, const float* d_r,
                           const float* d_sens, hipStream_t stream) {
  if (!plan || !d_x || !d_y || !d_sens) return SPECT_ERR_NULL;
  if (!aligned(d_x, 4) || !aligned(d_y, 4) || !aligned(d_sens, 4) || (d_r && !aligned(d_r, 4)))
    return SPECT_ERR_ALIGN;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  const size_t N = (size_t)p.g.nx * p.g.ny * p.g.nz;
  const size_t M = (size_t)p.g.nview * p.g.nz * p.g.nx;
  float* ybar = reinterpret_cast<float*>(p.ws + p.lay.em_proj);
  float* e = reinterpret_cast<float*>(p.ws + p.lay.em_vol);
  spect_status st = forward_impl(p, d_x, ybar, stream);
  if (st != SPECT_OK) return st;
  if (timed(p, K_EM_RATIO, stream, [&] { return launch_em_ratio(ybar, d_y, d_r, ybar, M, stream); }) !=
      hipSuccess)
    return SPECT_ERR_HIP;
  st = back_impl(p, ybar, e, stream);
  if (st != SPECT_OK) return st;
  if (timed(p, K_EM_UPDATE, stream, [&] { return launch_em_update(d_x, e, d_sens, N, stream); }) !=
      hipSuccess)
    return SPECT_ERR_HIP;
  return SPECT_OK;
}

spect_status spect_reg_em_step(spect_plan plan, float* d_x, const float* d_y, const float* d_r,
                               const float* d_sens, const float* d_u, float beta,
                               hipStream_t stream) {
  if (!plan || !d_x || !d_y || !d_sens || !d_u) return SPECT_ERR_NULL;
  if (!(std::isfinite(beta) && beta >= 0.0f)) return SPECT_ERR_VALUE;
  if (!aligned(d_x, 4) || !aligned(d_y, 4) || !aligned(d_sens, 4) || !aligned(d_u, 4) ||
      (d_r && !aligned(d_r, 4)))
    return SPECT_ERR_ALIGN;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  const size_t N = (size_t)p.g.nx * p.g.ny * p.g.nz;
  const size_t M = (size_t)p.g.nview * p.g.nz * p.g.nx;
  float* ybar = reinterpret_cast<float*>(p.ws + p.lay.em_proj);
  float* e = reinterpret_cast<float*>(p.ws + p.lay.em_vol);
  spect_status st = forward_impl(p, d_x, ybar, stream);
  if (st != SPECT_OK) return st;
  if (timed(p, K_EM_RATIO, stream, [&] { return launch_em_ratio(ybar, d_y, d_r, ybar, M, stream); }) !=
      hipSuccess)
    return SPECT_ERR_HIP;
  if ((st = back_impl(p, ybar, e, stream)) != SPECT_OK) return st;
  if (timed(p, K_EM_REG_UPDATE, stream, [&] {
        return launch_em_reg_update(d_x, e, d_sens, d_u, beta, N, stream);
      }) != hipSuccess)
    return SPECT_ERR_HIP;
  return SPECT_OK;
}

spect_status spect_em_step_vjp(spect_plan plan, const float* d_x, const float* d_y,
                               const float* d_r, const float* d_sens, const float* d_g,
                               float* d_gx, float* d_gy, hipStream_t stream) {
  if (!plan || !d_x || !d_y || !d_sens || !d_g || !d_gx) return SPECT_ERR_NULL;
  if (!aligned(d_x, 4) || !aligned(d_y, 4) || !aligned(d_sens, 4) || !aligned(d_g, 4) ||
      !aligned(d_gx, 4) || (d_r && !aligned(d_r, 4)) || (d_gy && !aligned(d_gy, 4)))
    return SPECT_ERR_ALIGN;
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  const size_t N = (size_t)p.g.nx * p.g.ny * p.g.nz;
  const size_t M = (size_t)p.g.nview * p.g.nz * p.g.nx;
  float* v = reinterpret_cast<float*>(p.ws + p.lay.em_proj);     // A x
  float* t = reinterpret_cast<float*>(p.ws + p.lay.em_proj2);    // rho, then A gb, then gq
  float* b = reinterpret_cast<float*>(p.ws + p.lay.em_vol);      // A' rho
  float* w = reinterpret_cast<float*>(p.ws + p.lay.em_vol2);     // gb, then A' gq
  // recompute the forward of the step (nothing is kept between calls)
  spect_status st = forward_impl(p, d_x, v, stream);
  if (st != SPECT_OK) return st;
  if (timed(p, K_EM_RATIO, stream, [&] { return launch_em_ratio(v, d_y, d_r, t, M, stream); }) !=
      hipSuccess)
    return SPECT_ERR_HIP;
  if ((st = back_impl(p, t, b, stream)) != SPECT_OK) return st;
  if (timed(p, K_EM_VJP, stream, [&] {
        return launch_em_vjp_prep(d_g, d_x, b, d_sens, w, d_gx, N, stream);
      }) != hipSuccess)
    return SPECT_ERR_HIP;
  if ((st = forward_impl(p, w, t, stream)) != SPECT_OK) return st;
  if (timed(p, K_EM_VJP, stream, [&] {
        return launch_em_vjp_ratio(t, v, d_y, d_r, d_gy, M, stream);
      }) != hipSuccess)
    return SPECT_ERR_HIP;
  if ((st = back_impl(p, t, w, stream)) != SPECT_OK) return st;
  if (timed(p, K_EM_VJP, stream, [&] { return launch_add(d_gx, w, N, stream); }) != hipSuccess)
    return SPECT_ERR_HIP;
  return SPECT_OK;
}

spect_status spect_profile_start(spect_plan plan, int32_t max_launches) {
  if (!plan) return SPECT_ERR_NULL;
  if (max_launches < 1 || max_launches > (1 << 20)) return SPECT_ERR_VALUE;
  Plan* p = reinterpret_cast<Plan*>(plan);
  profiler_free(p->prof);
  p->prof = nullptr;
  Profiler* pr = new (std::nothrow) Profiler();
  if (!pr) return SPECT_ERR_HIP;
  pr->cap = max_launches;
  pr->ev = static_cast<hipEvent_t*>(std::calloc(2 * (size_t)max_launches, sizeof(hipEvent_t)));
  pr->kid = static_cast<int*>(std::calloc((size_t)max_launches, sizeof(int)));
  if (!pr->ev || !pr->kid) {
    profiler_free(pr);
    return SPECT_ERR_HIP;
  }
  for (int i = 0; i < 2 * max_launches; ++i)
    if (hipEventCreate(&pr->ev[i]) != hipSuccess) {
      profiler_free(pr);
      return SPECT_ERR_HIP;
    }
  p->prof = pr;
  return SPECT_OK;
}

spect_status spect_profile_stop(spect_plan plan, spect_kernel_time* out, int32_t max_out,
                                int32_t* n_out) {
  if (!plan || !n_out || (max_out > 0 && !out)) return SPECT_ERR_NULL;
  Plan* p = reinterpret_cast<Plan*>(plan);
  Profiler* pr = p->prof;
  *n_out = 0;
  if (!pr) return SPECT_OK;
  p->prof = nullptr;
  spect_kernel_time acc[K_COUNT];
  std::memset(acc, 0, sizeof(acc));
  spect_status st = SPECT_OK;
  for (int r = 0; r < pr->used; ++r) {
    if (hipEventSynchronize(pr->ev[2 * r + 1]) != hipSuccess) { st = SPECT_ERR_HIP; break; }
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, pr->ev[2 * r], pr->ev[2 * r + 1]) != hipSuccess) {
      st = SPECT_ERR_HIP;
      break;
    }
    spect_kernel_time& a = acc[pr->kid[r]];
    if (a.launches == 0 || ms < a.min_ms) a.min_ms = ms;
    if (a.launches == 0 || ms > a.max_ms) a.max_ms = ms;
    a.launches += 1;
    a.total_ms += ms;
  }
  int n = 0;
  for (int k = 0; k < K_COUNT && st == SPECT_OK; ++k) {
    if (acc[k].launches == 0) continue;
    if (n < max_out) {
      out[n] = acc[k];
      std::strncpy(out[n].name, kKernelNames[k], sizeof(out[n].name) - 1);
      out[n].name[sizeof(out[n].name) - 1] = 0;
    }
    ++n;
  }
  *n_out = n < max_out ? n : max_out;
  profiler_free(pr);
  return st;
}

spect_status spect_dot_f64(const float* d_a, const float* d_b, size_t n, double* d_out,
                           hipStream_t stream) {
  if (!d_a || !d_b || !d_out) return SPECT_ERR_NULL;
  if (!aligned(d_a, 4) || !aligned(d_b, 4) || !aligned(d_out, 8)) return SPECT_ERR_ALIGN;
  return launch_dot_f64(d_a, d_b, n, d_out, stream) == hipSuccess ? SPECT_OK : SPECT_ERR_HIP;
}

}  // extern "C"
