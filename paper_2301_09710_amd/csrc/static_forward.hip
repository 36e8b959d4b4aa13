// spect_forward_static: the forward projection of Alg. 1 (Sec. II-A) for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  It takes the
// geometry instead of a plan and keeps everything a plan's workspace would
// hold -- the per-view rotation tables, the attenuation factors of a view
// batch, the weighted volumes and the per-chunk partial sums -- in `scratch`,
// a file-scope device array of kScratchBytes.  Nothing is allocated: the
// tables are computed on the device (the same FP64 formulas as a plan's host
// tables), and the kernels are the plan's.
//
// `scratch` is one array per device, shared by every call on that device, and
// it keeps the last call's contents; no kernel here needs it to start at zero
// (every region is written before it is read within a call).  Calls that
// overlap on one device race on it.
#include <mutex>

#include "internal.h"

namespace spect {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

// Device address of `scratch` on each device (its host-side name is only a
// stand-in), looked up once per device with that device current.
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on_current_device(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Rotation tables of the default angles theta_l = 2 pi l / nview, one
// workgroup per view (see Tables and table_entry).
__global__ void fill_tables_kernel(int n, int nview, int bilinear, int32_t* __restrict__ quarter,
                                   int32_t* __restrict__ off, float2* __restrict__ w,
                                   float2* __restrict__ rot) {
  const int l = blockIdx.x;
  if (l >= nview) return;
  int m;
  double phi;
  split_default_view(l, nview, &m, &phi);
  if (threadIdx.x == 0) {
    quarter[l] = m;
    rot[l] = make_float2((float)::cos(phi), (float)::sin(phi));
  }
  for (int t = threadIdx.x; t < 2 * n; t += blockDim.x) {
    const int ps = t / n, r = t - ps * n;
    const size_t e = ((size_t)l * 2 + ps) * n + r;
    table_entry(n, bilinear != 0, phi, ps, r, &off[2 * e], &w[e]);
  }
}

}  // namespace
}  // namespace spect

using namespace spect;

extern "C" spect_status spect_forward_static(const spect_geom* g, const float* d_mu,
                                             const float* d_psf, const float* d_x, float* d_v,
                                             hipStream_t stream) {
  if (!g || !d_mu || !d_psf || !d_x || !d_v) return SPECT_ERR_NULL;
  if (g->angles) return SPECT_ERR_UNSUPPORTED;     // the tables are made on the device
  spect_geom gs = *g;
  gs.flags &= ~SPECT_CACHE_MUBAR;                   // nothing outlives the call
  Layout lay;
  int vb = 0, nc = 0;
  spect_status st = compute_layout(gs, &lay, &vb, &nc);
  if (st != SPECT_OK) return st;
  if (lay.total > kScratchBytes) return SPECT_ERR_WORKSPACE;
  const uintptr_t a4 = (uintptr_t)d_mu | (uintptr_t)d_psf | (uintptr_t)d_x | (uintptr_t)d_v;
  if (a4 % 4) return SPECT_ERR_ALIGN;
  char* ws = nullptr;
  if (scratch_on_current_device(&ws) != hipSuccess) return SPECT_ERR_HIP;
  Plan p{};
  configure_plan(p, gs, lay, vb, nc, d_mu, d_psf, ws);
  // pairing of mirror-image taps only on the caller's word: the device check
  // would have to wait for the stream
  p.m4.mirror = p.use_m4 && p.conv_precision == SPECT_CONV_FP32 &&
                (gs.flags & SPECT_PSF_SYMMETRIC_X) != 0;
  hipLaunchKernelGGL(fill_tables_kernel, dim3((unsigned)gs.nview), dim3(256), 0, stream, gs.nx,
                     gs.nview, p.bilinear ? 1 : 0,
                     reinterpret_cast<int32_t*>(ws + lay.tables_quarter),
                     reinterpret_cast<int32_t*>(ws + lay.tables_off),
                     reinterpret_cast<float2*>(ws + lay.tables_w),
                     reinterpret_cast<float2*>(ws + lay.tables_rot));
  if (hipGetLastError() != hipSuccess) return SPECT_ERR_HIP;
  if (p.use_fft && launch_fft_psf_spectra(p, stream) != hipSuccess) return SPECT_ERR_HIP;
  return forward_impl(p, d_x, d_v, stream);
}
