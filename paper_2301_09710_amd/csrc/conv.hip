// PSF convolution kernels (Sec. II-A): every depth plane j of the rotated,
// attenuated volume is convolved with p(:,:,j,l) using replicate padding and
// the planes are summed (forward, Alg. 1); the back projector applies the
// exact transpose, including the fold that is the adjoint of replicate
// padding (Alg. 2).
//
//   forward  c[i,k] = sum_{a,b} p[a,b] w[clamp(i-a+ha), clamp(k-b+hb)]
//   back     u[i',k'] = sum_{a,b} p[a,b] sum{ v[i,k] : clamp(i-a+ha) = i',
//                                                 clamp(k-b+hb) = k' }
//
// For an interior output the back sum has one term per tap; on an edge row
// (i' = 0 or nx-1) or column it sums a run of v along that axis.
#include "internal.h"

namespace spect {
namespace {

__device__ __forceinline__ int clampi(int q, int lo, int hi) { return q < lo ? lo : (q > hi ? hi : q); }

// grid (ceil(nx*nz/256), nchunk, nvb): one output bin per thread, one chunk
// of kFwdJChunk depth planes per grid row; partial[c][lb][k][i].
__global__ __launch_bounds__(256) void conv_fwd_direct(const float* __restrict__ W,
                                                       const float* __restrict__ psf,
                                                       float* __restrict__ partial, int nx, int ny,
                                                       int nz, int px, int pz, int view0, int nvb) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= nx * nz) return;
  const int k = p / nx, i = p - k * nx;
  const int c = blockIdx.y, lb = blockIdx.z, l = view0 + lb;
  const int j0 = c * kFwdJChunk, j1 = min(ny, j0 + kFwdJChunk);
  const int ha = (px - 1) / 2, hb = (pz - 1) / 2;
  float acc = 0.0f;
  for (int j = j0; j < j1; ++j) {
    const float* pj = psf + ((size_t)l * ny + j) * pz * px;
    for (int b = 0; b < pz; ++b) {
      const int kc = clampi(k - b + hb, 0, nz - 1);
      const float* row = W + (((size_t)lb * nz + kc) * ny + j) * nx;
      const float* pb = pj + b * px;
      for (int a = 0; a < px; ++a) acc += pb[a] * row[clampi(i - a + ha, 0, nx - 1)];
    }
  }
  partial[((size_t)c * nvb + lb) * nx * nz + p] = acc;
}

__global__ void fwd_reduce_kernel(const float* __restrict__ partial, float* __restrict__ v,
                                  int plane, int nvb, int nchunk, int view0) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)nvb * plane;
  if (q >= total) return;
  float s = 0.0f;
  for (int c = 0; c < nchunk; ++c) s += partial[(size_t)c * total + q];
  v[(size_t)view0 * plane + q] = s;
}

// grid (ceil(nx*nz/256), ny, nvb): U[lb][k'][j][i'] = (conv^T v_l)(i', k') for plane j.
__global__ __launch_bounds__(256) void conv_back_direct(const float* __restrict__ v,
                                                        const float* __restrict__ psf,
                                                        float* __restrict__ U, int nx, int ny,
                                                        int nz, int px, int pz, int view0) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= nx * nz) return;
  const int kq = p / nx, iq = p - kq * nx;
  const int j = blockIdx.y, lb = blockIdx.z, l = view0 + lb;
  const int ha = (px - 1) / 2, hb = (pz - 1) / 2;
  const float* vl = v + (size_t)l * nz * nx;
  const float* pj = psf + ((size_t)l * ny + j) * pz * px;
  float acc = 0.0f;
  for (int b = 0; b < pz; ++b) {
    int klo = (kq == 0) ? 0 : kq + b - hb;
    int khi = (kq == nz - 1) ? nz - 1 : kq + b - hb;
    klo = max(klo, 0);
    khi = min(khi, nz - 1);
    if (klo > khi) continue;
    for (int a = 0; a < px; ++a) {
      int ilo = (iq == 0) ? 0 : iq + a - ha;
      int ihi = (iq == nx - 1) ? nx - 1 : iq + a - ha;
      ilo = max(ilo, 0);
      ihi = min(ihi, nx - 1);
      if (ilo > ihi) continue;
      float s = 0.0f;
      for (int kk = klo; kk <= khi; ++kk)
        for (int ii = ilo; ii <= ihi; ++ii) s += vl[kk * nx + ii];
      acc += pj[b * px + a] * s;
    }
  }
  U[(((size_t)lb * nz + kq) * ny + j) * nx + iq] = acc;
}

}  // namespace

hipError_t launch_conv_fwd(const Plan& p, const float* W, float* partial, int view0, int nvb,
                           hipStream_t s) {
  const spect_geom& g = p.g;
  dim3 grid((unsigned)((g.nx * g.nz + 255) / 256), (unsigned)p.nchunk, (unsigned)nvb);
  hipLaunchKernelGGL(conv_fwd_direct, grid, dim3(256), 0, s, W, p.psf, partial, g.nx, g.ny, g.nz,
                     g.px, g.pz, view0, nvb);
  return hipGetLastError();
}

hipError_t launch_fwd_reduce(const Plan& p, const float* partial, float* v, int view0, int nvb,
                             hipStream_t s) {
  const int plane = p.g.nx * p.g.nz;
  size_t total = (size_t)nvb * plane;
  hipLaunchKernelGGL(fwd_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     partial, v, plane, nvb, p.nchunk, view0);
  return hipGetLastError();
}

hipError_t launch_conv_back(const Plan& p, const float* v, float* U, int view0, int nvb,
                            hipStream_t s) {
  const spect_geom& g = p.g;
  dim3 grid((unsigned)((g.nx * g.nz + 255) / 256), (unsigned)g.ny, (unsigned)nvb);
  hipLaunchKernelGGL(conv_back_direct, grid, dim3(256), 0, s, v, p.psf, U, g.nx, g.ny, g.nz, g.px,
                     g.pz, view0);
  return hipGetLastError();
}

}  // namespace spect
