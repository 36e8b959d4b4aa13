// Rotation kernels (Sec. II-A): rotate activity and attenuation slices by
// theta_l with an exact quarter turn and three 1-D linear-interpolation
// shears, form the attenuation factor of Eq. (1), weight; and the exact
// transpose of those steps accumulated over views (Alg. 2).
//
// Design: one workgroup owns one z-slice (n x n, n = nx = ny) held in LDS as
// rows j of stride S floats and loops over several views.  The three
// passes are evaluated as one fused gather per output pixel: pass 3 needs two
// pass-2 values, each needing two pass-1 values, each needing two pixels of
// the quarter-turned slice -- at most 8 LDS reads and 14 two-tap blends,
// with the pass semantics kept exactly (every intermediate sample outside
// [0, n) is zero, as in a pass over the whole slice).  A wave owns 8 x 8 pixel
// tiles and the LDS row stride S is 8 (mod 16) floats: the gathers of a
// rotated tile then spread over the 64 LDS banks for every angle (a wave
// covering one row would read along a sheared line, which some angle maps
// onto one bank).  The quarter turn is an
// affine remapping of the LDS address, so the slice is staged once per
// workgroup, unrotated, whatever the view.  The transpose uses the same
// tables with the taps mirrored (out[q] = w.x in[q - o] + w.y in[q - o - 1]),
// applies the passes in reverse order and the inverse quarter turn last.
#include "internal.h"

namespace spect {
namespace {

constexpr int NT = kRotThreads;
constexpr int NWAVE = NT / 64;
constexpr int TPR_MAX = (kMaxLdsN + 7) / 8;                 // 8x8 tiles per row
constexpr int RMAX = (TPR_MAX * TPR_MAX + NWAVE - 1) / NWAVE; // tiles (pixels) per lane

// LDS row stride of a slice: >= n and = 8 (mod 16).
__host__ __device__ __forceinline__ int slice_stride(int n) { return n + ((8 - n % 16) + 16) % 16; }

// Pixel of lane `lane`, iteration r: 8x8 tile (w + NWAVE r) of the slice.
__device__ __forceinline__ bool tile_pixel(int n, int r, int& i, int& j) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tpr = (n + 7) >> 3;
  const int tile = w + NWAVE * r;
  const int tj = tile / tpr, ti = tile - tj * tpr;
  i = 8 * ti + (lane & 7);
  j = 8 * tj + (lane >> 3);
  return tj < tpr && i < n && j < n;
}

// Position (di, dj) that pixel (i, j) takes under P_m, the gather
// out(p) = in(R(m*90deg)^-1 (p - c) + c) with R acting on (i, j).
__device__ __forceinline__ void quarter_dst(int m, int n, int i, int j, int& di, int& dj) {
  if (m == 0) { di = i; dj = j; }
  else if (m == 1) { di = n - 1 - j; dj = i; }
  else if (m == 2) { di = n - 1 - i; dj = n - 1 - j; }
  else { di = j; dj = n - 1 - i; }
}

// LDS address of f0(i, j) = (P_m x)(i, j) when the unrotated slice is stored
// as X[j][i] with row stride S:  addr = base + ci * i + cj * j.
struct QAddr { int base, ci, cj; };
__device__ __forceinline__ QAddr quarter_addr(int m, int n, int S) {
  // m=0: X[j][i]; m=1: X[n-1-i][j]; m=2: X[n-1-j][n-1-i]; m=3: X[i][n-1-j]
  if (m == 0) return {0, 1, S};
  if (m == 1) return {(n - 1) * S, -S, 1};
  if (m == 2) return {(n - 1) * S + (n - 1), -1, -S};
  return {n - 1, S, -1};
}

struct ViewTab {          // per-view tables in LDS
  int* o13;  float2* w13; // passes 1 and 3, indexed by row j
  int* o2;   float2* w2;  // pass 2, indexed by column i
};

__device__ __forceinline__ bool inside(int q, int n) { return (unsigned)q < (unsigned)n; }

// Forward: value of (S3 S2 S1 P_m x)(i, j) from the unrotated slice X.
__device__ __forceinline__ float rotated_pixel(const float* X, int n, const QAddr& qa,
                                               const ViewTab& t, int i, int j) {
  float f3 = 0.0f;
  const int o3 = t.o13[j];
  const float2 w3 = t.w13[j];
#pragma unroll
  for (int t3 = 0; t3 < 2; ++t3) {
    const int i2 = i + o3 + t3;
    if (!inside(i2, n)) continue;
    const int o2 = t.o2[i2];
    const float2 w2 = t.w2[i2];
    float f2 = 0.0f;
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2) {
      const int j1 = j + o2 + t2;
      if (!inside(j1, n)) continue;
      const int o1 = t.o13[j1];
      const float2 w1 = t.w13[j1];
      const int ia = i2 + o1, ib = i2 + o1 + 1;
      const float a = inside(ia, n) ? X[qa.base + qa.ci * ia + qa.cj * j1] : 0.0f;
      const float b = inside(ib, n) ? X[qa.base + qa.ci * ib + qa.cj * j1] : 0.0f;
      const float f1 = w1.x * a + w1.y * b;
      f2 += (t2 == 0 ? w2.x : w2.y) * f1;
    }
    f3 += (t3 == 0 ? w3.x : w3.y) * f2;
  }
  return f3;
}

// Transpose: value of (S1^T S2^T S3^T g)(q, r) from g stored as G[r][q].
__device__ __forceinline__ float rotated_T_pixel(const float* G, int n, int S, const ViewTab& t,
                                                 int q, int r) {
  // pass-1 transpose along i for row r
  const int o1 = t.o13[r];
  const float2 w1 = t.w13[r];
  float h1 = 0.0f;
#pragma unroll
  for (int t1 = 0; t1 < 2; ++t1) {
    const int q2 = q - o1 - t1;
    if (!inside(q2, n)) continue;
    // pass-2 transpose along j for column q2
    const int o2 = t.o2[q2];
    const float2 w2 = t.w2[q2];
    float h2 = 0.0f;
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2) {
      const int r3 = r - o2 - t2;
      if (!inside(r3, n)) continue;
      // pass-3 transpose along i for row r3
      const int o3 = t.o13[r3];
      const float2 w3 = t.w13[r3];
      const int qa = q2 - o3, qb = q2 - o3 - 1;
      const float a = inside(qa, n) ? G[r3 * S + qa] : 0.0f;
      const float b = inside(qb, n) ? G[r3 * S + qb] : 0.0f;
      const float h3 = w3.x * a + w3.y * b;
      h2 += (t2 == 0 ? w2.x : w2.y) * h3;
    }
    h1 += (t1 == 0 ? w1.x : w1.y) * h2;
  }
  return h1;
}

// LDS carve-up: slice buffers of n*S floats, then the tables of one view.
__device__ __forceinline__ ViewTab carve_tab(float* after, int n) {
  ViewTab t;
  t.o13 = reinterpret_cast<int*>(after);
  t.o2 = t.o13 + n;
  t.w13 = reinterpret_cast<float2*>(t.o2 + n);   // 8-byte aligned: 2n ints precede
  t.w2 = t.w13 + n;
  return t;
}

__device__ __forceinline__ void load_tab(const Tables& tab, int l, int n, const ViewTab& t) {
  const int32_t* off = tab.off + (size_t)l * 2 * n;
  const float2* w = tab.w + (size_t)l * 2 * n;
  for (int e = threadIdx.x; e < 2 * n; e += NT) {
    t.o13[e] = off[e];   // o13 and o2 are contiguous: [0, n) pass 1/3, [n, 2n) pass 2
    t.w13[e] = w[e];
  }
}

__device__ __forceinline__ void stage_slice(float* X, const float* __restrict__ src, int n, int S) {
  for (int p = threadIdx.x; p < n * n; p += NT) {
    const int j = p / n, i = p - j * n;
    X[j * S + i] = src[p];
  }
}

// ---------------------------------------------------------------- Eq. (1)
// grid (nz, ceil(nviews / VG)): for slice k and views [v0 + g*VG, ...):
// out[(l - out_view0)][k] = mubar of view l.  LDS: mu slice, rotated buffer, tables.
__global__ __launch_bounds__(NT) void mubar_kernel(const float* __restrict__ mu,
                                                   float* __restrict__ out, int n, int nz,
                                                   int view0, int nviews, int VG, int out_view0,
                                                   Tables tab, double dy) {
  extern __shared__ float smem[];
  const int S = slice_stride(n);
  float* X = smem;
  float* Y = smem + n * S;
  ViewTab t = carve_tab(Y + n * S, n);
  const int k = blockIdx.x;
  const size_t nn = (size_t)n * n;
  stage_slice(X, mu + (size_t)k * nn, n, S);
  const int lb0 = blockIdx.y * VG, lb1 = min(nviews, lb0 + VG);
  for (int lb = lb0; lb < lb1; ++lb) {
    const int l = view0 + lb;
    __syncthreads();                                   // X staged / previous view done
    load_tab(tab, l, n, t);
    __syncthreads();
    const QAddr qa = quarter_addr(tab.quarter[l], n, S);
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      int i, j;
      if (tile_pixel(n, r, i, j)) Y[j * S + i] = rotated_pixel(X, n, qa, t, i, j);
    }
    __syncthreads();
    // suffix scan along j for every column i (detector beyond j = n-1), FP64
    if (threadIdx.x < n) {
      const int i = threadIdx.x;
      double run = 0.0;
      for (int j = n - 1; j >= 0; --j) {
        const float m = Y[j * S + i];
        Y[j * S + i] = (float)exp(-dy * (0.5 * (double)m + run));
        run += (double)m;
      }
    }
    __syncthreads();
    float* dst = out + ((size_t)(l - out_view0) * nz + k) * nn;
    for (int p = threadIdx.x; p < n * n; p += NT) {
      const int j = p / n, i = p - j * n;
      dst[p] = Y[j * S + i];
    }
  }
}

// ---------------------------------------------------------------- forward
// grid (nz, ceil(nvb / VG)): W[lb][k] = (R_l x)[k] * mubar_l[k] for the views
// lb of this group; mubar of view lb is at mb + (lb + mb_off) * N.
__global__ __launch_bounds__(NT) void rot_fwd_kernel(const float* __restrict__ x,
                                                     const float* __restrict__ mb, int mb_off,
                                                     float* __restrict__ W, int n, int nz,
                                                     int view0, int nvb, int VG, Tables tab) {
  extern __shared__ float smem[];
  const int S = slice_stride(n);
  float* X = smem;
  ViewTab t = carve_tab(X + n * S, n);
  const int k = blockIdx.x;
  const size_t nn = (size_t)n * n, N = nn * nz;
  stage_slice(X, x + (size_t)k * nn, n, S);
  const int lb0 = blockIdx.y * VG, lb1 = min(nvb, lb0 + VG);
  for (int lb = lb0; lb < lb1; ++lb) {
    const int l = view0 + lb;
    const float* mbs = mb + (size_t)(lb + mb_off) * N + (size_t)k * nn;
    float att[RMAX];                       // attenuation factors, loaded ahead of the gathers
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      int i, j;
      att[r] = tile_pixel(n, r, i, j) ? mbs[j * n + i] : 0.0f;
    }
    __syncthreads();
    load_tab(tab, l, n, t);
    __syncthreads();
    const QAddr qa = quarter_addr(tab.quarter[l], n, S);
    float* dst = W + (size_t)lb * N + (size_t)k * nn;
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      int i, j;
      if (tile_pixel(n, r, i, j)) dst[j * n + i] = rotated_pixel(X, n, qa, t, i, j) * att[r];
    }
  }
}

// ---------------------------------------------------------------- back
// grid (nz, G): partial[g][k] (+)= sum over views lb = g, g+G, ... of
//   P_m^T S1^T S2^T S3^T (U[lb][k] * mubar_l[k]).
__global__ __launch_bounds__(NT) void rot_back_kernel(const float* __restrict__ U,
                                                      const float* __restrict__ mb, int mb_off,
                                                      float* __restrict__ partial, int n, int nz,
                                                      int view0, int nvb, int G, int accumulate,
                                                      Tables tab) {
  extern __shared__ float smem[];
  const int S = slice_stride(n);
  float* Gs = smem;
  ViewTab t = carve_tab(Gs + n * S, n);
  const int k = blockIdx.x, g = blockIdx.y;
  const size_t nn = (size_t)n * n, N = nn * nz;
  float acc[RMAX];
#pragma unroll
  for (int r = 0; r < RMAX; ++r) acc[r] = 0.0f;
  for (int lb = g; lb < nvb; lb += G) {
    const int l = view0 + lb;
    const int m = tab.quarter[l];
    __syncthreads();                                   // previous view's readers done
    load_tab(tab, l, n, t);
    const float* src = U + (size_t)lb * N + (size_t)k * nn;
    const float* mbs = mb + (size_t)(lb + mb_off) * N + (size_t)k * nn;
    for (int p = threadIdx.x; p < n * n; p += NT) {
      const int j = p / n, i = p - j * n;
      Gs[j * S + i] = src[p] * mbs[p];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      int i, j;
      if (tile_pixel(n, r, i, j)) {
        int di, dj;
        quarter_dst(m, n, i, j, di, dj);                 // P_m^T: x(i, j) = h(P_m position)
        acc[r] += rotated_T_pixel(Gs, n, S, t, di, dj);
      }
    }
  }
  float* dst = partial + (size_t)g * N + (size_t)k * nn;
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    int i, j;
    if (tile_pixel(n, r, i, j)) dst[j * n + i] = accumulate ? dst[j * n + i] + acc[r] : acc[r];
  }
}

__global__ void back_reduce_kernel(const float* __restrict__ partial, float* __restrict__ x,
                                   size_t N, int G) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  float s = 0.0f;
  for (int g = 0; g < G; ++g) s += partial[(size_t)g * N + p];
  x[p] = s;
}

size_t tab_bytes(int n) { return (size_t)2 * n * 4 + (size_t)2 * n * 8; }
size_t slice_bytes(int n) { return (size_t)n * slice_stride(n) * 4; }

hipError_t set_smem(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

hipError_t launch_mubar(const Plan& p, float* out, int view0, int nviews, int out_view0,
                        hipStream_t s) {
  const int n = p.g.nx;
  const size_t sm = 2 * slice_bytes(n) + tab_bytes(n);
  hipError_t e = set_smem((const void*)mubar_kernel, sm);
  if (e != hipSuccess) return e;
  const int VG = kRotViewsPerGroup;
  dim3 grid(p.g.nz, (nviews + VG - 1) / VG);
  hipLaunchKernelGGL(mubar_kernel, grid, dim3(NT), sm, s, p.mu, out, n, p.g.nz, view0, nviews, VG,
                     out_view0, p.tab, p.g.dy);
  return hipGetLastError();
}

hipError_t launch_rot_fwd(const Plan& p, const float* x, const float* mb, int mb_off, float* W,
                          int view0, int nvb, hipStream_t s) {
  const int n = p.g.nx;
  const size_t sm = slice_bytes(n) + tab_bytes(n);
  hipError_t e = set_smem((const void*)rot_fwd_kernel, sm);
  if (e != hipSuccess) return e;
  const int VG = kRotViewsPerGroup;
  dim3 grid(p.g.nz, (nvb + VG - 1) / VG);
  hipLaunchKernelGGL(rot_fwd_kernel, grid, dim3(NT), sm, s, x, mb, mb_off, W, n, p.g.nz, view0,
                     nvb, VG, p.tab);
  return hipGetLastError();
}

hipError_t launch_rot_back(const Plan& p, const float* U, const float* mb, int mb_off,
                           float* partial, int view0, int nvb, bool accumulate, hipStream_t s) {
  const int n = p.g.nx;
  const size_t sm = slice_bytes(n) + tab_bytes(n);
  hipError_t e = set_smem((const void*)rot_back_kernel, sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rot_back_kernel, dim3(p.g.nz, kBackGroups), dim3(NT), sm, s, U, mb, mb_off,
                     partial, n, p.g.nz, view0, nvb, kBackGroups, accumulate ? 1 : 0, p.tab);
  return hipGetLastError();
}

hipError_t launch_back_reduce(const Plan& p, const float* partial, float* x, hipStream_t s) {
  const size_t N = (size_t)p.g.nx * p.g.ny * p.g.nz;
  hipLaunchKernelGGL(back_reduce_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                     partial, x, N, kBackGroups);
  return hipGetLastError();
}

}  // namespace spect
