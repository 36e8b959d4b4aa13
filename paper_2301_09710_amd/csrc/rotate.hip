// Rotation kernels: rotate activity and attenuation slices by theta_l,
// form the attenuation factor of Eq. (1) and weight (forward), and the exact
// transpose of those steps accumulated over views (back).  Sec. II-A.
//
// One workgroup handles one z-slice (an n x n plane, n = nx = ny) of one
// view.  The slice lives in LDS as rows j of stride S = n + 1 floats (the +1
// keeps the column passes and the quarter-turn scatter free of bank
// conflicts).  Every pass of the 3-pass rotation is a 1-D two-tap gather
// along rows or columns; a pass reads the whole slice into registers, waits,
// and writes it back, so a slice needs one buffer.  The quarter turn P_m is
// applied while the slice is copied from HBM into LDS (coalesced global
// reads, permuted LDS writes); its transpose is applied on the way out.
#include "internal.h"

namespace spect {
namespace {

constexpr int NT = kRotThreads;
constexpr int RMAX = (kMaxLdsN * kMaxLdsN + NT - 1) / NT;

// Position (di, dj) that pixel (i, j) takes under P_m, the gather
// out(p) = in(R(m*90deg)^-1 (p - c) + c) with R acting on (i, j).
__device__ __forceinline__ void quarter_dst(int m, int n, int i, int j, int& di, int& dj) {
  if (m == 0) { di = i; dj = j; }
  else if (m == 1) { di = n - 1 - j; dj = i; }
  else if (m == 2) { di = n - 1 - i; dj = n - 1 - j; }
  else { di = j; dj = n - 1 - i; }
}

__device__ __forceinline__ float ld(const float* line, int q, int n, int stride) {
  return (q >= 0 && q < n) ? line[q * stride] : 0.0f;
}

// Copy a global [j][i] slice into LDS rows, applying P_m.
__device__ void load_quarter(float* buf, const float* __restrict__ src, int n, int S, int m) {
  for (int p = threadIdx.x; p < n * n; p += NT) {
    int j = p / n, i = p - j * n;
    int di, dj;
    quarter_dst(m, n, i, j, di, dj);
    buf[dj * S + di] = src[p];
  }
}

// One gather pass along i for every row j (passes 1 and 3), or its transpose.
//   forward:   out[j][i]  = w.x in[j][i + o] + w.y in[j][i + o + 1]
//   transpose: out[j][q]  = w.x g[j][q - o] + w.y g[j][q - o - 1]
template <bool kTranspose>
__device__ void pass_rows(float* buf, int n, int S, const int* off, const float2* w) {
  float tmp[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    int p = threadIdx.x + r * NT;
    float val = 0.0f;
    if (p < n * n) {
      int j = p / n, i = p - j * n;
      int o = off[j];
      float2 ww = w[j];
      const float* row = buf + j * S;
      if (!kTranspose) val = ww.x * ld(row, i + o, n, 1) + ww.y * ld(row, i + o + 1, n, 1);
      else             val = ww.x * ld(row, i - o, n, 1) + ww.y * ld(row, i - o - 1, n, 1);
    }
    tmp[r] = val;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    int p = threadIdx.x + r * NT;
    if (p < n * n) { int j = p / n, i = p - j * n; buf[j * S + i] = tmp[r]; }
  }
  __syncthreads();
}

// One gather pass along j for every column i (pass 2), or its transpose.
template <bool kTranspose>
__device__ void pass_cols(float* buf, int n, int S, const int* off, const float2* w) {
  float tmp[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    int p = threadIdx.x + r * NT;
    float val = 0.0f;
    if (p < n * n) {
      int j = p / n, i = p - j * n;
      int o = off[i];
      float2 ww = w[i];
      const float* col = buf + i;
      if (!kTranspose) val = ww.x * ld(col, j + o, n, S) + ww.y * ld(col, j + o + 1, n, S);
      else             val = ww.x * ld(col, j - o, n, S) + ww.y * ld(col, j - o - 1, n, S);
    }
    tmp[r] = val;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    int p = threadIdx.x + r * NT;
    if (p < n * n) { int j = p / n, i = p - j * n; buf[j * S + i] = tmp[r]; }
  }
  __syncthreads();
}

// Eq. (1) in place on a rotated attenuation slice: running suffix sum along j
// (detector beyond j = n-1), kept in FP64.
__device__ void mubar_scan(float* buf, int n, int S, double dy) {
  if (threadIdx.x < n) {
    const int i = threadIdx.x;
    double run = 0.0;
    for (int j = n - 1; j >= 0; --j) {
      float mu = buf[j * S + i];
      buf[j * S + i] = (float)exp(-dy * (0.5 * (double)mu + run));
      run += (double)mu;
    }
  }
  __syncthreads();
}

__device__ void load_tables(const Tables& tab, int l, int n, int* s_off, float2* s_w) {
  for (int t = threadIdx.x; t < 2 * n; t += NT) {
    s_off[t] = tab.off[(size_t)l * 2 * n + t];
    s_w[t] = tab.w[(size_t)l * 2 * n + t];
  }
}

// Rotated attenuation factor of view l, slice k, into buf.
__device__ void mubar_slice(float* buf, const float* __restrict__ mu, const float* __restrict__ cache,
                            int l, int k, int n, int nz, int S, int m, const int* s_off,
                            const float2* s_w, double dy) {
  const size_t nn = (size_t)n * n;
  if (cache) {
    const float* src = cache + ((size_t)l * nz + k) * nn;
    for (int p = threadIdx.x; p < n * n; p += NT) {
      int j = p / n, i = p - j * n;
      buf[j * S + i] = src[p];
    }
    __syncthreads();
    return;
  }
  load_quarter(buf, mu + (size_t)k * nn, n, S, m);
  __syncthreads();
  pass_rows<false>(buf, n, S, s_off, s_w);
  pass_cols<false>(buf, n, S, s_off + n, s_w + n);
  pass_rows<false>(buf, n, S, s_off, s_w);
  mubar_scan(buf, n, S, dy);
}

struct Smem {
  float* A;
  float* B;
  int* off;
  float2* w;
};

__device__ Smem carve(int n) {
  extern __shared__ float smem[];
  const int S = n + 1;
  Smem s;
  s.A = smem;
  s.B = smem + n * S;
  s.off = reinterpret_cast<int*>(s.B + n * S);
  s.w = reinterpret_cast<float2*>(s.off + 2 * n);
  return s;
}

size_t smem_bytes(int n) { return (size_t)2 * n * (n + 1) * 4 + (size_t)2 * n * 4 + (size_t)2 * n * 8; }

__global__ __launch_bounds__(NT) void mubar_cache_kernel(const float* __restrict__ mu,
                                                         float* __restrict__ out, int n, int nz,
                                                         Tables tab, double dy) {
  Smem s = carve(n);
  const int k = blockIdx.x, l = blockIdx.y, S = n + 1;
  load_tables(tab, l, n, s.off, s.w);
  __syncthreads();
  mubar_slice(s.A, mu, nullptr, l, k, n, nz, S, tab.quarter[l], s.off, s.w, dy);
  float* dst = out + ((size_t)l * nz + k) * n * n;
  for (int p = threadIdx.x; p < n * n; p += NT) {
    int j = p / n, i = p - j * n;
    dst[p] = s.A[j * S + i];
  }
}

// Forward: W[lb][k] = (R_l x)[k] * mubar_l[k]   (lb = l - view0)
__global__ __launch_bounds__(NT) void rot_fwd_kernel(const float* __restrict__ x,
                                                     const float* __restrict__ mu,
                                                     const float* __restrict__ cache,
                                                     float* __restrict__ W, int n, int nz,
                                                     int view0, Tables tab, double dy) {
  Smem s = carve(n);
  const int k = blockIdx.x, lb = blockIdx.y, l = view0 + lb, S = n + 1;
  const int m = tab.quarter[l];
  load_tables(tab, l, n, s.off, s.w);
  __syncthreads();
  mubar_slice(s.A, mu, cache, l, k, n, nz, S, m, s.off, s.w, dy);
  load_quarter(s.B, x + (size_t)k * n * n, n, S, m);
  __syncthreads();
  pass_rows<false>(s.B, n, S, s.off, s.w);
  pass_cols<false>(s.B, n, S, s.off + n, s.w + n);
  // pass 3 fused with the weight and the store
  float* dst = W + ((size_t)lb * nz + k) * n * n;
  for (int p = threadIdx.x; p < n * n; p += NT) {
    int j = p / n, i = p - j * n;
    int o = s.off[j];
    float2 ww = s.w[j];
    const float* row = s.B + j * S;
    float val = ww.x * ld(row, i + o, n, 1) + ww.y * ld(row, i + o + 1, n, 1);
    dst[p] = val * s.A[j * S + i];
  }
}

// Back: partial[g][k] (+)= sum over views lb = g, g+G, ... of
//        P_m^T S1^T S2^T S3^T (U[lb][k] * mubar_l[k])
__global__ __launch_bounds__(NT) void rot_back_kernel(const float* __restrict__ U,
                                                      const float* __restrict__ mu,
                                                      const float* __restrict__ cache,
                                                      float* __restrict__ partial, int n, int nz,
                                                      int view0, int nvb, int accumulate,
                                                      Tables tab, double dy) {
  Smem s = carve(n);
  const int k = blockIdx.x, g = blockIdx.y, S = n + 1;
  const size_t nn = (size_t)n * n;
  float acc[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) acc[r] = 0.0f;
  for (int lb = g; lb < nvb; lb += kBackGroups) {
    const int l = view0 + lb;
    const int m = tab.quarter[l];
    load_tables(tab, l, n, s.off, s.w);
    __syncthreads();
    mubar_slice(s.A, mu, cache, l, k, n, nz, S, m, s.off, s.w, dy);
    const float* src = U + ((size_t)lb * nz + k) * nn;
    for (int p = threadIdx.x; p < n * n; p += NT) {
      int j = p / n, i = p - j * n;
      s.B[j * S + i] = src[p] * s.A[j * S + i];
    }
    __syncthreads();
    pass_rows<true>(s.B, n, S, s.off, s.w);           // pass 3 transpose
    pass_cols<true>(s.B, n, S, s.off + n, s.w + n);   // pass 2 transpose
    pass_rows<true>(s.B, n, S, s.off, s.w);           // pass 1 transpose
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {                  // P_m transpose (gather back)
      int p = threadIdx.x + r * NT;
      if (p < n * n) {
        int j = p / n, i = p - j * n, di, dj;
        quarter_dst(m, n, i, j, di, dj);
        acc[r] += s.B[dj * S + di];
      }
    }
    __syncthreads();
  }
  float* dst = partial + ((size_t)g * nz + k) * nn;
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    int p = threadIdx.x + r * NT;
    if (p < n * n) dst[p] = accumulate ? dst[p] + acc[r] : acc[r];
  }
}

__global__ void back_reduce_kernel(const float* __restrict__ partial, float* __restrict__ x,
                                   size_t N) {
  size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  float s = 0.0f;
  for (int g = 0; g < kBackGroups; ++g) s += partial[(size_t)g * N + p];
  x[p] = s;
}

}  // namespace

static hipError_t set_smem(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_mubar_cache(const Plan& p, float* out, hipStream_t s) {
  const int n = p.g.nx;
  size_t sm = smem_bytes(n);
  hipError_t e = set_smem((const void*)mubar_cache_kernel, sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mubar_cache_kernel, dim3(p.g.nz, p.g.nview), dim3(NT), sm, s, p.mu, out, n,
                     p.g.nz, p.tab, p.g.dy);
  return hipGetLastError();
}

hipError_t launch_rot_fwd(const Plan& p, const float* x, float* W, int view0, int nvb,
                          hipStream_t s) {
  const int n = p.g.nx;
  size_t sm = smem_bytes(n);
  hipError_t e = set_smem((const void*)rot_fwd_kernel, sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rot_fwd_kernel, dim3(p.g.nz, nvb), dim3(NT), sm, s, x, p.mu, p.mubar, W, n,
                     p.g.nz, view0, p.tab, p.g.dy);
  return hipGetLastError();
}

hipError_t launch_rot_back(const Plan& p, const float* U, float* partial, int view0, int nvb,
                           bool accumulate, hipStream_t s) {
  const int n = p.g.nx;
  size_t sm = smem_bytes(n);
  hipError_t e = set_smem((const void*)rot_back_kernel, sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rot_back_kernel, dim3(p.g.nz, kBackGroups), dim3(NT), sm, s, U, p.mu,
                     p.mubar, partial, n, p.g.nz, view0, nvb, accumulate ? 1 : 0, p.tab, p.g.dy);
  return hipGetLastError();
}

hipError_t launch_back_reduce(const Plan& p, const float* partial, float* x, hipStream_t s) {
  size_t N = (size_t)p.g.nx * p.g.ny * p.g.nz;
  hipLaunchKernelGGL(back_reduce_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                     partial, x, N);
  return hipGetLastError();
}

}  // namespace spect
