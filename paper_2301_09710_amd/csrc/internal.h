// Internal declarations shared by the host code and the kernel files of
// libspect.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/spect.h"

namespace spect {

// Largest in-plane size for which one z-slice (two padded n x (n+1) float
// buffers) fits in the 160 KiB LDS of a gfx950 compute unit.
constexpr int kMaxLdsN = 140;
// Threads per workgroup of the rotation kernels.
constexpr int kRotThreads = 1024;
// Depth planes per partial sum of the forward convolution.
constexpr int kFwdJChunk = 8;
// View groups (partial volumes) of the back rotation.
constexpr int kBackGroups = 16;

// Per-view geometry tables, on the device (inside the workspace).
//   quarter[l]             : m, number of quarter turns (0..3)
//   off[l][0][j], w[l][0][j]: passes 1 and 3 (along i, one entry per row j)
//   off[l][1][i], w[l][1][i]: pass 2 (along j, one entry per column i)
// A pass computes out[q] = w.x * in[q + off] + w.y * in[q + off + 1], zero
// outside [0, n); w.x = 1 - f and w.y = f of the fractional shift.
struct Tables {
  const int32_t* quarter;
  const int32_t* off;
  const float2* w;
};

// Workspace layout (byte offsets from the workspace base, 256-B aligned).
struct Layout {
  size_t tables_quarter, tables_off, tables_w;
  size_t vol_batch;     // view_batch * N floats: W (forward) / U (back)
  size_t fwd_partial;   // nchunk * view_batch * nz * nx floats
  size_t back_partial;  // kBackGroups * N floats
  size_t mubar_cache;   // nview * N floats (only with SPECT_CACHE_MUBAR)
  size_t em_proj;       // nview * nz * nx floats
  size_t em_vol;        // N floats
  size_t total;
};

struct Plan {
  spect_geom g;         // angles pointer cleared after creation
  int view_batch;
  int nchunk;           // forward depth chunks
  const float* mu;
  const float* psf;
  char* ws;
  Layout lay;
  Tables tab;
  const float* mubar;   // cache or nullptr
  // host copies of the tables (kept alive for the asynchronous upload)
  int32_t* h_quarter;
  int32_t* h_off;
  float2* h_w;
};

spect_status compute_layout(const spect_geom& g, Layout* lay, int* view_batch, int* nchunk);

// ---- kernel launchers (return hipGetLastError() of the launch) ----
hipError_t launch_mubar_cache(const Plan& p, float* out, hipStream_t s);
hipError_t launch_rot_fwd(const Plan& p, const float* x, float* W, int view0, int nvb,
                          hipStream_t s);
hipError_t launch_conv_fwd(const Plan& p, const float* W, float* partial, int view0, int nvb,
                           hipStream_t s);
hipError_t launch_fwd_reduce(const Plan& p, const float* partial, float* v, int view0, int nvb,
                             hipStream_t s);
hipError_t launch_conv_back(const Plan& p, const float* v, float* U, int view0, int nvb,
                            hipStream_t s);
hipError_t launch_rot_back(const Plan& p, const float* U, float* partial, int view0, int nvb,
                           bool accumulate, hipStream_t s);
hipError_t launch_back_reduce(const Plan& p, const float* partial, float* x, hipStream_t s);
hipError_t launch_em_ratio(const float* v, const float* y, const float* r, float* rho, size_t m,
                           hipStream_t s);
hipError_t launch_em_update(float* x, const float* e, const float* sens, size_t n, hipStream_t s);
hipError_t launch_dot_f64(const float* a, const float* b, size_t n, double* out, hipStream_t s);

}  // namespace spect
