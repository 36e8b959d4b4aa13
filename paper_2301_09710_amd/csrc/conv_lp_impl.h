// Kernel templates of the BF16 / FP16 / split-BF16 PSF convolution and their
// launch helpers.  Included by one translation unit per operand format
// (conv_lp_bf16.hip, conv_lp_fp16.hip, conv_lp_bf16x3.hip), each of which
// instantiates only its own kernels; the mapping is described in conv_lp.hip.
#pragma once
#include <type_traits>

#include "internal.h"

namespace spect {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class T> struct Lp;
template <> struct Lp<__bf16> {
  typedef bf16x8 vec;
  static __device__ __forceinline__ floatx4 mfma(u32x4 a, u32x4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(vec, a),
                                                  __builtin_bit_cast(vec, b), c, 0, 0, 0);
  }
};
template <> struct Lp<_Float16> {
  typedef halfx8 vec;
  static __device__ __forceinline__ floatx4 mfma(u32x4 a, u32x4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(vec, a),
                                                 __builtin_bit_cast(vec, b), c, 0, 0, 0);
  }
};

// Two values rounded to T (nearest even) packed low-first in a 32-bit word.
template <class T>
__device__ __forceinline__ unsigned pack2(float lo, float hi) {
  typedef T t2 __attribute__((ext_vector_type(2)));
  t2 v;
  v[0] = (T)lo;
  v[1] = (T)hi;
  return __builtin_bit_cast(unsigned, v);
}

// Split of an FP32 value into a leading T part and a T remainder:
// v ~ hi + lo with hi = round(v) and lo = round(v - hi) (v - hi is exact in
// FP32).  For BF16 the pair carries 16 significant bits.
template <class T>
__device__ __forceinline__ float lead(float v) { return (float)(T)v; }

template <class T, bool kLo>
__device__ __forceinline__ unsigned pack2_part(float a, float b) {
  return kLo ? pack2<T>(a - lead<T>(a), b - lead<T>(b)) : pack2<T>(a, b);
}

__device__ __forceinline__ int clampi(int q, int lo, int hi) { return q < lo ? lo : (q > hi ? hi : q); }

// PSF pair table of one plane: QP[a][q] = (Q[a][q], Q[a][q + 1]) with
//   forward  Q[a][q] = p[a][2hb + 15 - q]
//   adjoint  Q[a][q] = p[a][q - 15]
// (0 outside the PSF); row px is all zero (the chunks past the last tap).
// Staging issues the global loads of kStageIt items per thread before any
// conversion or LDS write, so that their latencies overlap.
constexpr int kStageIt = 1;

template <class T, bool kBack, bool kSplit>
__device__ __forceinline__ void stage_psf(unsigned* QP, const float* __restrict__ pj,
                                          const LpShape& s) {
  const int rows = s.px + 1, total = rows * s.QL;
  for (int base = 0; base < total; base += kStageIt * (int)blockDim.x) {
    float v[kStageIt][2];
#pragma unroll
    for (int it = 0; it < kStageIt; ++it) {
      const int e = base + threadIdx.x + it * blockDim.x;
      const int q = e / rows, a = e - q * rows;         // a fastest: PSF rows are contiguous in a
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int b = kBack ? q + h - 15 : 2 * s.hb + 15 - q - h;
        v[it][h] = (e < total && a < s.px && b >= 0 && b < s.pz) ? pj[b * s.px + a] : 0.0f;
      }
    }
#pragma unroll
    for (int it = 0; it < kStageIt; ++it) {
      const int e = base + threadIdx.x + it * blockDim.x;
      const int q = e / rows, a = e - q * rows;
      if (e < total) {
        QP[a * s.QL + q] = pack2<T>(v[it][0], v[it][1]);
        if (kSplit) QP[total + a * s.QL + q] = pack2_part<T, true>(v[it][0], v[it][1]);
      }
    }
  }
}

// The PSF table of the next plane, loaded into registers while the current
// plane is computed and written to LDS after the plane's last read of the
// table (the global-load latency hides behind the MFMAs).  Used when the
// table has at most kPsfReg items per thread.
constexpr int kPsfReg = 11;
template <class T, bool kBack, bool kSplit>
struct PsfPrefetch {
  float v[kPsfReg][2];
  __device__ __forceinline__ void load(const float* __restrict__ pj, const LpShape& s) {
    const int rows = s.px + 1, total = rows * s.QL;
#pragma unroll
    for (int it = 0; it < kPsfReg; ++it) {
      const int e = threadIdx.x + it * blockDim.x;
      const int q = e / rows, a = e - q * rows;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int b = kBack ? q + h - 15 : 2 * s.hb + 15 - q - h;
        v[it][h] = (e < total && a < s.px && b >= 0 && b < s.pz) ? pj[b * s.px + a] : 0.0f;
      }
    }
  }
  __device__ __forceinline__ void store(unsigned* QP, const LpShape& s) const {
    // indices recomputed here rather than kept live across the MFMAs from load()
    int rows = s.px + 1;
    asm volatile("" : "+s"(rows));
    const int total = rows * s.QL;
#pragma unroll
    for (int it = 0; it < kPsfReg; ++it) {
      const int e = threadIdx.x + it * blockDim.x;
      const int q = e / rows, a = e - q * rows;
      if (e < total) {
        QP[a * s.QL + q] = pack2<T>(v[it][0], v[it][1]);
        if (kSplit) QP[total + a * s.QL + q] = pack2_part<T, true>(v[it][0], v[it][1]);
      }
    }
  }
};

__device__ __forceinline__ bool psf_fits_regs(const LpShape& s) {
  return (s.px + 1) * s.QL <= kPsfReg * (int)blockDim.x;
}

// Transposed region Rt[cc][rr] (column stride RS elements) of a plane
// src[z * zstride + x]: rr <-> z = k0 - hb + rr, cc <-> x = X0 + cc with
// X0 = i0 - ha - dx aligned to 4 columns; clamped (forward, replicate
// padding) or zero outside (adjoint).  An item is 8 rows x 4 columns: eight
// 16-byte loads along x (scalar, clamped loads for the columns at the plane
// edges or when rows are not 16-byte aligned) and four 16-byte LDS writes.
template <class T, bool kClamp, bool kSplit>
__device__ __forceinline__ void stage_region(unsigned* Rt, const float* __restrict__ src,
                                             size_t zstride, const LpShape& s, int k0, int i0,
                                             bool vec_ok) {
  const int cq_n = s.RCa / 4;
  const int total = (s.RR / 8) * cq_n;
  const int X0 = i0 - s.ha - s.dx;
  u32x4* R4 = reinterpret_cast<u32x4*>(Rt);
  for (int base = 0; base < total; base += kStageIt * (int)blockDim.x) {
    float v[kStageIt][8][4];
#pragma unroll
    for (int it = 0; it < kStageIt; ++it) {
      const int e = base + threadIdx.x + it * blockDim.x;
      const int rq = e / cq_n, cq = e - rq * cq_n;
      const int x0 = X0 + 4 * cq;
      const bool inner = vec_ok && x0 >= 0 && x0 + 3 < s.nx;
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int z = k0 - s.hb + 8 * rq + h;
        const bool zin = z >= 0 && z < s.nz;
        const size_t zrow = (size_t)(kClamp ? clampi(z, 0, s.nz - 1) : z) * zstride;
        if (e < total && inner && (kClamp || zin)) {
          const float4 q = *reinterpret_cast<const float4*>(src + zrow + x0);
          v[it][h][0] = q.x; v[it][h][1] = q.y; v[it][h][2] = q.z; v[it][h][3] = q.w;
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int x = x0 + c;
            float val = 0.0f;
            if (e < total) {
              if (kClamp) val = src[zrow + clampi(x, 0, s.nx - 1)];
              else if (zin && x >= 0 && x < s.nx) val = src[zrow + x];
            }
            v[it][h][c] = val;
          }
        }
      }
    }
#pragma unroll
    for (int it = 0; it < kStageIt; ++it) {
      const int e = base + threadIdx.x + it * blockDim.x;
      const int rq = e / cq_n, cq = e - rq * cq_n;
      if (e < total) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int at = ((4 * cq + c) * s.RS) / 8 + rq;
          R4[at] = u32x4{pack2<T>(v[it][0][c], v[it][1][c]), pack2<T>(v[it][2][c], v[it][3][c]),
                         pack2<T>(v[it][4][c], v[it][5][c]), pack2<T>(v[it][6][c], v[it][7][c])};
          if (kSplit)
            R4[at + s.RCa * s.RS / 8] = u32x4{
                pack2_part<T, true>(v[it][0][c], v[it][1][c]), pack2_part<T, true>(v[it][2][c], v[it][3][c]),
                pack2_part<T, true>(v[it][4][c], v[it][5][c]), pack2_part<T, true>(v[it][6][c], v[it][7][c])};
        }
      }
    }
  }
}

// All taps of one plane, in quads: lane group g takes tap 4 tq + g (taps past
// px read the zero PSF row).  For each absolute 8-row chunk R of the region,
// the B operands of the wave's two N-blocks are read once and feed every
// M-block b whose band holds the chunk (relative chunk c = R - 2b in
// [0, C7)), with the A operand of relative chunk c kept in registers for the
// whole quad.  B of chunk R + 1 is read while the MFMAs of chunk R run.
//   acc[b][u]: M-block b (z rows k0 + 16 b ..), N-block u of this wave.
// kSplit: operands and PSF come as leading parts and remainders (tables of
// the remainders follow the leading ones in LDS) and each product takes
// three MFMAs, hi*hi + hi*lo + lo*hi.
template <class T, int C7, int WKM, bool kBack, bool kSplit>
__device__ __forceinline__ void plane_quads(floatx4 (&acc)[WKM][2], const unsigned* QP,
                                            const unsigned* Rt, const LpShape& s, int g, int m,
                                            int n, int w) {
  constexpr int kNR = 2 * (WKM - 1) + C7;             // region chunks of the tile
  constexpr int kP = kSplit ? 2 : 1;                   // parts per operand
  const u32x4* R4 = reinterpret_cast<const u32x4*>(Rt);
  const int qp_words = (s.px + 1) * s.QL, r4_words = s.RCa * s.RS / 8;
  for (int tq = 0; tq < s.ntq; ++tq) {
    const int t = 4 * tq + g;
    const bool in = t < s.px;
    const int ta = in ? t : s.px, tb = in ? t : 0;
    u32x4 A[kP][C7];
#pragma unroll
    for (int h = 0; h < kP; ++h) {
      const unsigned* q = QP + h * qp_words + ta * s.QL - m + 15;
#pragma unroll
      for (int c = 0; c < C7; ++c)
        A[h][c] = u32x4{q[8 * c], q[8 * c + 2], q[8 * c + 4], q[8 * c + 6]};
    }
    const int col = (kBack ? 32 * w + n + tb : 32 * w + n - tb + 2 * s.ha) + s.dx;
    const u32x4* b0 = R4 + (col * s.RS) / 8;             // chunk R: b0[R] (16-byte units)
    const u32x4* b1 = R4 + ((col + 16) * s.RS) / 8;
    u32x4 x0[kP], x1[kP];
#pragma unroll
    for (int h = 0; h < kP; ++h) {
      x0[h] = b0[h * r4_words];
      x1[h] = b1[h * r4_words];
    }
#pragma unroll
    for (int R = 0; R < kNR; ++R) {
      u32x4 y0[kP], y1[kP];
#pragma unroll
      for (int h = 0; h < kP; ++h) {
        y0[h] = x0[h];
        y1[h] = x1[h];
        if (R + 1 < kNR) {
          y0[h] = b0[h * r4_words + R + 1];
          y1[h] = b1[h * r4_words + R + 1];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int b = 0; b < WKM; ++b) {
        const int c = R - 2 * b;
        if (c >= 0 && c < C7) {
          if (kSplit) {
            acc[b][0] = Lp<T>::mfma(A[1][c], x0[0], acc[b][0]);
            acc[b][1] = Lp<T>::mfma(A[1][c], x1[0], acc[b][1]);
            acc[b][0] = Lp<T>::mfma(A[0][c], x0[kP - 1], acc[b][0]);
            acc[b][1] = Lp<T>::mfma(A[0][c], x1[kP - 1], acc[b][1]);
          }
          acc[b][0] = Lp<T>::mfma(A[0][c], x0[0], acc[b][0]);
          acc[b][1] = Lp<T>::mfma(A[0][c], x1[0], acc[b][1]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int h = 0; h < kP; ++h) {
        x0[h] = y0[h];
        x1[h] = y1[h];
      }
    }
  }
}

// Workgroup -> (tile, chunk, view).
__device__ __forceinline__ void decode(const LpShape& s, int& tk, int& ti, int& c, int& lb,
                                       int nchunk) {
  const int ntile = s.tiles_k * s.tiles_i;
  const int b = blockIdx.x;
  const int tile = b % ntile, rest = b / ntile;
  tk = tile / s.tiles_i;
  ti = tile - tk * s.tiles_i;
  c = rest % nchunk;
  lb = rest / nchunk;
}

__device__ __forceinline__ void plane_range(int c, int nchunk, int ny, int& j0, int& j1) {
  j0 = (int)(((long long)c * ny) / nchunk);
  j1 = (int)(((long long)(c + 1) * ny) / nchunk);
}

template <int WKM>
__device__ __forceinline__ void zero_acc(floatx4 (&acc)[WKM][2]) {
#pragma unroll
  for (int b = 0; b < WKM; ++b) acc[b][0] = acc[b][1] = floatx4{0.f, 0.f, 0.f, 0.f};
}

// acc[b][u][v] -> bin (k0 + 16 b + 4 g + v, i0 + 32 w + 16 u + n) of a plane
// whose row k starts at out + k * kstride.
template <int WKM>
__device__ __forceinline__ void store_acc(const floatx4 (&acc)[WKM][2], float* out,
                                          size_t kstride, const LpShape& s, int k0, int i0, int w,
                                          int g, int n) {
  // opaque to the optimiser, so the 64 store offsets are formed here and not
  // hoisted out of a plane loop (where they would occupy registers throughout)
  asm volatile("" : "+s"(kstride));
#pragma unroll
  for (int b = 0; b < WKM; ++b) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = k0 + 16 * b + 4 * g + v, i = i0 + 32 * w + 16 * u + n;
        if (k < s.nz && i < s.nx) out[(size_t)k * kstride + i] = acc[b][u][v];
      }
    __builtin_amdgcn_sched_barrier(0);   // one M-block's accumulators in VGPRs at a time
  }
}

// ---------------------------------------------------------------- forward
// partial[c][lb][k][i] = sum over the planes j of chunk c of (p_{j,l} * W_j)[k][i]
template <class T, int C7, int WKM, bool kSplit>
__global__ __launch_bounds__(256) void conv_fwd_lp(const float* __restrict__ W,
                                                   const float* __restrict__ psf,
                                                   float* __restrict__ partial, LpShape s,
                                                   int view0, int nvb) {
  extern __shared__ unsigned lds[];
  unsigned* Rt = lds;                                  // P x RCa * RS / 2 words
  unsigned* QP = lds + (kSplit ? 2 : 1) * s.RCa * s.RS / 2;   // P x (px + 1) * QL words
  int tk, ti, c, lb;
  decode(s, tk, ti, c, lb, s.nchunk);
  const int l = view0 + lb;
  const int k0 = tk * 16 * s.WKm, i0 = ti * 32 * s.NN;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
  int j0, j1;
  plane_range(c, s.nchunk, s.ny, j0, j1);
  const size_t zstride = (size_t)s.ny * s.nx;
  const float* Wl = W + (size_t)lb * s.nz * zstride;
  const float* psf_l = psf + (size_t)l * s.ny * s.pz * s.px;
  const size_t pstride = (size_t)s.pz * s.px;
  const bool vec_ok = (s.nx % 4) == 0 && ((uintptr_t)Wl % 16) == 0;
  const bool pref = psf_fits_regs(s);
  floatx4 acc[WKM][2];
  zero_acc(acc);
  PsfPrefetch<T, false, kSplit> nxt;
  if (pref && j0 < j1) nxt.load(psf_l + (size_t)j0 * pstride, s);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                                   // previous plane consumed
    if (pref) nxt.store(QP, s);
    else stage_psf<T, false, kSplit>(QP, psf_l + (size_t)j * pstride, s);
    stage_region<T, true, kSplit>(Rt, Wl + (size_t)j * s.nx, zstride, s, k0, i0, vec_ok);
    if (pref && j + 1 < j1) nxt.load(psf_l + (size_t)(j + 1) * pstride, s);
    __syncthreads();
    plane_quads<T, C7, WKM, false, kSplit>(acc, QP, Rt, s, g, n, n, w);
  }
  store_acc(acc, partial + ((size_t)c * nvb + lb) * s.nz * s.nx, (size_t)s.nx, s, k0, i0, w, g, n);
}

// ---------------------------------------------------------------- adjoint
// U[lb][k][j][i] = zero-padded correlation of the projection of view l with
// p_{j,l}; exact off the edge rows and columns, which the FP32 edge kernel
// rewrites afterwards.
template <class T, int C7, int WKM, bool kSplit>
__global__ __launch_bounds__(256) void conv_back_lp(const float* __restrict__ v,
                                                    const float* __restrict__ psf,
                                                    float* __restrict__ U, LpShape s, int view0,
                                                    int nvb) {
  extern __shared__ unsigned lds[];
  unsigned* Rt = lds;
  unsigned* QP = lds + (kSplit ? 2 : 1) * s.RCa * s.RS / 2;
  int tk, ti, c, lb;
  decode(s, tk, ti, c, lb, s.nchunk_back);
  const int l = view0 + lb;
  const int k0 = tk * 16 * s.WKm, i0 = ti * 32 * s.NN;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
  int j0, j1;
  plane_range(c, s.nchunk_back, s.ny, j0, j1);
  const float* vl = v + (size_t)l * s.nz * s.nx;
  const float* psf_l = psf + (size_t)l * s.ny * s.pz * s.px;
  const size_t pstride = (size_t)s.pz * s.px;
  const bool pref = psf_fits_regs(s);
  stage_region<T, false, kSplit>(Rt, vl, (size_t)s.nx, s, k0, i0,
                         (s.nx % 4) == 0 && ((uintptr_t)vl % 16) == 0);
  PsfPrefetch<T, true, kSplit> nxt;
  if (pref && j0 < j1) nxt.load(psf_l + (size_t)j0 * pstride, s);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                                   // region staged / previous plane consumed
    if (pref) nxt.store(QP, s);
    else stage_psf<T, true, kSplit>(QP, psf_l + (size_t)j * pstride, s);
    __syncthreads();
    if (pref && j + 1 < j1) nxt.load(psf_l + (size_t)(j + 1) * pstride, s);
    floatx4 acc[WKM][2];
    zero_acc(acc);
    plane_quads<T, C7, WKM, true, kSplit>(acc, QP, Rt, s, g, n, n, w);
    store_acc(acc, U + (size_t)lb * s.nz * s.ny * s.nx + (size_t)j * s.nx, (size_t)s.ny * s.nx, s,
              k0, i0, w, g, n);
  }
}

hipError_t set_lds(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Instantiations: C7 (8-row chunks of a tap band) in 2..8, WKM (16-row
// M-blocks per tile) in 1..8, T in {bf16, f16}.
#define SPECT_C7_CASES(X, W) X(2, W) X(3, W) X(4, W) X(5, W) X(6, W) X(7, W) X(8, W)
#define SPECT_LP_CASES(X) \
  SPECT_C7_CASES(X, 1) SPECT_C7_CASES(X, 2) SPECT_C7_CASES(X, 3) SPECT_C7_CASES(X, 4) \
  SPECT_C7_CASES(X, 5) SPECT_C7_CASES(X, 6) SPECT_C7_CASES(X, 7) SPECT_C7_CASES(X, 8)

template <class T, bool kSplit>
const void* fwd_fn(const LpShape& s) {
#define CASE(C, W) if (s.C7 == C && s.WKm == W) return (const void*)conv_fwd_lp<T, C, W, kSplit>;
  SPECT_LP_CASES(CASE)
#undef CASE
  return nullptr;
}

template <class T, bool kSplit>
const void* back_fn(const LpShape& s) {
#define CASE(C, W) if (s.C7 == C && s.WKm == W) return (const void*)conv_back_lp<T, C, W, kSplit>;
  SPECT_LP_CASES(CASE)
#undef CASE
  return nullptr;
}

template <class T, bool kSplit>
hipError_t launch_fwd_t(const LpShape& s, const float* W, const float* psf, float* partial,
                        int view0, int nvb, hipStream_t st) {
  const size_t sm = lp_lds_bytes(s, kSplit);
  const void* fn = fwd_fn<T, kSplit>(s);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = set_lds(fn, sm);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)(s.tiles_k * s.tiles_i * s.nchunk * nvb)), block(64 * s.NN);
  hipLaunchKernelGGL(reinterpret_cast<void (*)(const float*, const float*, float*, LpShape, int, int)>(
                         const_cast<void*>(fn)),
                     grid, block, sm, st, W, psf, partial, s, view0, nvb);
  return hipGetLastError();
}

template <class T, bool kSplit>
hipError_t launch_back_t(const LpShape& s, const float* v, const float* psf, float* U, int view0,
                         int nvb, hipStream_t st) {
  const size_t sm = lp_lds_bytes(s, kSplit);
  const void* fn = back_fn<T, kSplit>(s);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = set_lds(fn, sm);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)(s.tiles_k * s.tiles_i * s.nchunk_back * nvb)), block(64 * s.NN);
  hipLaunchKernelGGL(reinterpret_cast<void (*)(const float*, const float*, float*, LpShape, int, int)>(
                         const_cast<void*>(fn)),
                     grid, block, sm, st, v, psf, U, s, view0, nvb);
  return hipGetLastError();
}

template <class T, bool kSplit>
int lp_wgs_per_cu(const LpShape& s, bool back) {
  int nb = 0;
  const void* fn = back ? back_fn<T, kSplit>(s) : fwd_fn<T, kSplit>(s);
  const size_t sm = lp_lds_bytes(s, kSplit);
  if (!fn || set_lds(fn, sm) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64 * s.NN, sm) != hipSuccess || nb < 1)
    nb = (int)(kLdsBytes / (sm ? sm : 1));
  return nb < 1 ? 1 : nb;
}

}  // namespace
}  // namespace spect
