// PSF convolution on the matrix cores (FP32 MFMA, v_mfma_f32_16x16x4f32).
//
// The replicate-padded convolution of Sec. II-A (Alg. 1) along the z axis is
// a banded Toeplitz product, which this file maps onto 16x16x4 MFMA tiles:
//
//   rows M  = 16 output positions k (z), one M-block per wave
//   cols N  = 16 output positions i (x), two N-blocks per wave
//   K       = the 16 + pz - 1 input rows along z that the M-block touches,
//             in k-steps of 4 (KS = ceil((15 + pz) / 4) steps)
//   A[m][r] = p[a, b] with b = m - r + 2 hb (forward) / b = r - m (adjoint):
//             the Toeplitz band of PSF row a, read from a zero-padded copy
//             of that row in LDS
//   B[r][n] = the staged input plane, shifted by the PSF tap a along x
//
// and the loop over the px taps a along x, and over the depth planes j of a
// chunk (forward), accumulates in the MFMA accumulators.  The band wastes
// (16 + pz - 1) / pz of the MFMA work (1.41x for pz = 37); the roofline is
// stated against the algorithmic 2 px pz FLOP per voxel.
//
// Forward (sum over depth): each workgroup owns an output tile of
// (16 WK) x (32 WI) bins of one view and a chunk of depth planes; for every
// plane it stages the (16 WK + pz - 1) x (32 WI + px - 1) input region with
// the source indices clamped (replicate padding costs nothing in the inner
// loop) and the PSF, and adds the plane into the accumulators.  Each plane's
// MFMA sum is folded into a second accumulator set so long chains stay
// short.  Partial sums per chunk are reduced in a fixed order afterwards.
//
// Adjoint (per depth plane): the same tiles read the projection of one view,
// staged once with zero padding; replicate padding's adjoint is the fold of
// the border onto the edge rows and columns, which is handled by
//   * output rows at k = 0 / nz-1: suffix / prefix sums of the PSF row
//     along b replace the PSF row (per-lane choice of the A source);
//   * output columns at i = 0 / nx-1: prefix / suffix sums of the projection
//     along x replace the shifted projection (extra LDS columns, per-lane
//     choice of the B source).
#include "internal.h"

namespace spect {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int clampi(int q, int lo, int hi) { return q < lo ? lo : (q > hi ? hi : q); }

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// The MFMA operands of one PSF tap a: KS A values (Toeplitz band of PSF row
// a) and KS B values for each of the two N-blocks.  Loads are issued per
// k-step so that a short prefetch distance can be kept in flight: the LDS
// wait counter of gfx9 counts at most 15 outstanding LDS instructions, so
// prefetching a whole tap (about 20 of them) would force full waits.
template <int KS>
struct Ops {
  float av[KS], b0[KS], b1[KS];
  // forward: A = P[a][aoff - 4s], B = R[boff - a + 4s RSI (+16)]
  __device__ __forceinline__ void load_fwd(int s, const float* Pa, const float* Rb, int a, int PL,
                                           int RSI) {
    av[s] = Pa[a * PL - 4 * s];
    b0[s] = Rb[4 * s * RSI - a];
    b1[s] = Rb[4 * s * RSI - a + 16];
  }
  // adjoint: A = P[var][a][aoff + 4s], B = R[row + colb + a + 4s RSI]
  __device__ __forceinline__ void load_back(int s, const float* Pa, const float* B0,
                                            const float* B1, int a, int PL, int RSI) {
    av[s] = Pa[a * PL + 4 * s];
    b0[s] = B0[a + 4 * s * RSI];
    b1[s] = B1[a + 4 * s * RSI];
  }
  // even and odd k-steps feed separate accumulators: four independent MFMA
  // dependency chains per wave
  __device__ __forceinline__ void step(int s, floatx4 (&acc)[4]) const {
    acc[(s & 1) * 2 + 0] = mfma(av[s], b0[s], acc[(s & 1) * 2 + 0]);
    acc[(s & 1) * 2 + 1] = mfma(av[s], b1[s], acc[(s & 1) * 2 + 1]);
  }
};

constexpr int kPrefetch = 4;   // k-steps of operands kept in flight

// One tap `a` held in X: run its KS k-steps while loading the remaining
// steps of X and the first kPrefetch steps of the next tap into Y.
template <int KS, class LoadX, class LoadY>
__device__ __forceinline__ void tap_block(Ops<KS>& X, Ops<KS>& Y, floatx4 (&acc)[4],
                                          LoadX&& lx, LoadY&& ly) {
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int t = s + kPrefetch;
    if (t < KS) lx(X, t);
    else ly(Y, t - KS);
    X.step(s, acc);
    // keep this order: the scheduler would otherwise sink the prefetch next
    // to its use and the wait counter would stall every step
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Workgroup id -> (tile, chunk, view) so that consecutive logical ids, which
// share input planes, land on the same XCD (the hardware deals workgroups to
// the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_remap(int wg, int total) {
  const int per = total / 8, rem = total % 8, x = wg % 8, slot = wg / 8;
  // XCDs x < rem own per + 1 logical ids, the others per
  const int base = x * per + min(x, rem);
  return base + slot;
}

// Depth planes of chunk c: [c ny / nchunk, (c+1) ny / nchunk).
__device__ __forceinline__ void chunk_range(int c, int nchunk, int ny, int& j0, int& j1) {
  j0 = (int)(((long long)c * ny) / nchunk);
  j1 = (int)(((long long)(c + 1) * ny) / nchunk);
}

// Per-thread staging of one forward plane: the (RK = 4 KS) x RI input region
// (one M-block of rows, WK = 1) and the px x PL PSF rows.  Wave w stages
// region rows w, w+4, ...; lane l of a row covers columns l, l+64, l+128, so
// row offsets are wave-uniform and column offsets are per-lane constants
// that do not change from plane to plane.  The values of plane j+1 are loaded
// into registers while plane j is being computed.
constexpr int kStageCols = 3;    // 64-column sweeps per region row (RI <= 192)
constexpr int kStagePsf = 16;    // PSF elements per thread (px * PL <= 4096)

template <int KS>
struct FwdStage {
  float r[KS][kStageCols];
  float q[kStagePsf];
  __device__ __forceinline__ void load(const ConvShape& cs, const float* __restrict__ Wl,
                                       const float* __restrict__ pj, int j, int k0, int i0,
                                       size_t plane_stride, int w, int lane) {
    const float* Wj = Wl + (size_t)j * cs.nx;
#pragma unroll
    for (int r8 = 0; r8 < KS; ++r8) {
      const int rk = w + 4 * r8;                                   // < 4 KS = RK
      const float* row = Wj + (size_t)clampi(k0 - cs.hb + rk, 0, cs.nz - 1) * plane_stride;
#pragma unroll
      for (int u = 0; u < kStageCols; ++u) {
        const int ri = lane + 64 * u;
        r[r8][u] = (ri < cs.RI) ? row[clampi(i0 - cs.ha + ri, 0, cs.nx - 1)] : 0.0f;
      }
    }
#pragma unroll
    for (int t = 0; t < kStagePsf; ++t) {
      const int e = threadIdx.x + 256 * t;
      float v = 0.0f;
      if (e < cs.px * cs.PL) {
        const int a = e / cs.PL, b = e - a * cs.PL - cs.Z;
        if (b >= 0 && b < cs.pz) v = pj[b * cs.px + a];
      }
      q[t] = v;
    }
  }
  __device__ __forceinline__ void store(const ConvShape& cs, float* R, float* P, int w,
                                        int lane) const {
#pragma unroll
    for (int r8 = 0; r8 < KS; ++r8) {
      const int rk = w + 4 * r8;
#pragma unroll
      for (int u = 0; u < kStageCols; ++u) {
        const int ri = lane + 64 * u;
        if (ri < cs.RI) R[rk * cs.RSI + ri] = r[r8][u];
      }
    }
#pragma unroll
    for (int t = 0; t < kStagePsf; ++t) {
      const int e = threadIdx.x + 256 * t;
      if (e < cs.px * cs.PL) P[e] = q[t];
    }
  }
};

// ---------------------------------------------------------------- forward
template <int KS>
__global__ __launch_bounds__(256, 2) void conv_fwd_mfma(const float* __restrict__ W,
                                                        const float* __restrict__ psf,
                                                        float* __restrict__ partial, ConvShape cs,
                                                        int view0, int nvb) {
  extern __shared__ float sm[];
  float* R = sm;                               // RK x RSI: input region of one plane
  float* P = sm + cs.RK * cs.RSI;              // px x PL: zero-padded PSF rows
  const int ntile = cs.tiles_k * cs.tiles_i;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = logical % ntile, rest = logical / ntile;
  const int tk = tile / cs.tiles_i, ti = tile - tk * cs.tiles_i;
  const int c = rest % cs.nchunk, lb = rest / cs.nchunk, l = view0 + lb;
  const int k0 = tk * 16 * cs.WK, i0 = ti * 32 * cs.WI;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
  const int wk = w / cs.WI, wi = w - wk * cs.WI;
  int j0, j1;
  chunk_range(c, cs.nchunk, cs.ny, j0, j1);
  const size_t plane_stride = (size_t)cs.ny * cs.nx;
  const float* Wl = W + (size_t)lb * cs.nz * plane_stride;
  const float* psf_l = psf + (size_t)l * cs.ny * cs.pz * cs.px;
  const bool prefetch = cs.WK == 1 && cs.RI <= 64 * kStageCols && cs.px * cs.PL <= 256 * kStagePsf;

  floatx4 tot0 = {0.f, 0.f, 0.f, 0.f}, tot1 = {0.f, 0.f, 0.f, 0.f};
  const int aoff = n - g + 2 * cs.hb + cs.Z;                         // A: P[a][aoff - 4s]
  const int boff = (wk * 16 + g) * cs.RSI + wi * 32 + n + 2 * cs.ha;  // B: R[boff - a + 4s RSI]
  FwdStage<KS> st;
  if (prefetch && j0 < j1)
    st.load(cs, Wl, psf_l + (size_t)j0 * cs.pz * cs.px, j0, k0, i0, plane_stride, w, lane);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                                                 // previous plane consumed
    if (prefetch) {
      st.store(cs, R, P, w, lane);
      __syncthreads();
      if (j + 1 < j1)
        st.load(cs, Wl, psf_l + (size_t)(j + 1) * cs.pz * cs.px, j + 1, k0, i0, plane_stride, w,
                lane);
    } else {
      // general shapes: stage straight from memory
      const float* Wj = Wl + (size_t)j * cs.nx;
      int rk = threadIdx.x / cs.RI, ri = threadIdx.x - (threadIdx.x / cs.RI) * cs.RI;
      for (; rk < cs.RK;) {
        const int kk = clampi(k0 - cs.hb + rk, 0, cs.nz - 1);
        const int ii = clampi(i0 - cs.ha + ri, 0, cs.nx - 1);
        R[rk * cs.RSI + ri] = Wj[(size_t)kk * plane_stride + ii];
        ri += 256;
        while (ri >= cs.RI) { ri -= cs.RI; ++rk; }
      }
      const float* pj = psf_l + (size_t)j * cs.pz * cs.px;
      for (int e = threadIdx.x; e < cs.px * cs.PL; e += 256) {
        const int a = e / cs.PL, b = e - a * cs.PL - cs.Z;
        P[e] = (b >= 0 && b < cs.pz) ? pj[b * cs.px + a] : 0.0f;
      }
      __syncthreads();
    }
    floatx4 acc[4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f},
                      {0.f, 0.f, 0.f, 0.f}};
    // taps a along x, software-pipelined: the operands of the next k-steps are
    // read from LDS while the MFMAs of the current one run
    Ops<KS> A, B;
    const float* Pa = P + aoff;
    const float* Rb = R + boff;
#pragma unroll
    for (int s = 0; s < kPrefetch; ++s) A.load_fwd(s, Pa, Rb, 0, cs.PL, cs.RSI);
    for (int a = 0; a < cs.px; a += 2) {
      const int a1 = min(a + 1, cs.px - 1), a2 = min(a + 2, cs.px - 1);
      tap_block<KS>(A, B, acc,
                    [&](Ops<KS>& o, int t) { o.load_fwd(t, Pa, Rb, a, cs.PL, cs.RSI); },
                    [&](Ops<KS>& o, int t) { o.load_fwd(t, Pa, Rb, a1, cs.PL, cs.RSI); });
      if (a + 1 < cs.px)
        tap_block<KS>(B, A, acc,
                      [&](Ops<KS>& o, int t) { o.load_fwd(t, Pa, Rb, a1, cs.PL, cs.RSI); },
                      [&](Ops<KS>& o, int t) { o.load_fwd(t, Pa, Rb, a2, cs.PL, cs.RSI); });
    }
    tot0 += acc[0] + acc[2];
    tot1 += acc[1] + acc[3];
  }
  // D[4g + v][n]: output k = k0 + 16 wk + 4g + v, i = i0 + 32 wi + 16 nb + n
  float* out = partial + ((size_t)c * nvb + lb) * cs.nz * cs.nx;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int k = k0 + wk * 16 + 4 * g + v;
    const int i = i0 + wi * 32 + n;
    if (k < cs.nz) {
      if (i < cs.nx) out[(size_t)k * cs.nx + i] = tot0[v];
      if (i + 16 < cs.nx) out[(size_t)k * cs.nx + i + 16] = tot1[v];
    }
  }
}

// Per-thread staging of one adjoint plane's PSF rows: P[0] the rows
// themselves (offset 15: index b + 15), on z-edge tiles also P[1] the suffix
// sums (b' >= b) and P[2] the prefix sums (b' <= b) along b; nz = 1 uses the
// full row sum for both.
struct BackPsf {
  float v0[kStagePsf], v1[kStagePsf], v2[kStagePsf];
  __device__ __forceinline__ void load_range(const ConvShape& cs, const float* __restrict__ psf,
                                             const float* __restrict__ psf_cum, int l, int j,
                                             bool kedge, int base) {
    const size_t off = ((size_t)l * cs.ny + j) * cs.pz * cs.px;
    const float* pj = psf + off;
    const float* suf = psf_cum + off;
    const float* pre = suf + (size_t)cs.nview_ny_pz_px;
#pragma unroll
    for (int t = 0; t < kStagePsf; ++t) {
      const int e = base + threadIdx.x + 256 * t;
      float x0 = 0.0f, x1 = 0.0f, x2 = 0.0f;
      if (e < cs.px * cs.PL) {
        const int a = e / cs.PL, b = e - a * cs.PL - 15;
        if (b >= 0 && b < cs.pz) x0 = pj[b * cs.px + a];
        if (kedge) {
          const float tot = suf[a];
          if (cs.nz == 1) { x1 = tot; x2 = tot; }
          else {
            x1 = (b < 0) ? tot : (b < cs.pz ? suf[b * cs.px + a] : 0.0f);
            x2 = (b < 0) ? 0.0f : pre[min(b, cs.pz - 1) * cs.px + a];
          }
        }
      }
      v0[t] = x0; v1[t] = x1; v2[t] = x2;
    }
  }
  __device__ __forceinline__ void store_range(const ConvShape& cs, float* P, bool kedge,
                                              int base) const {
    const int m = cs.px * cs.PL;
#pragma unroll
    for (int t = 0; t < kStagePsf; ++t) {
      const int e = base + threadIdx.x + 256 * t;
      if (e < m) {
        P[e] = v0[t];
        if (kedge) { P[m + e] = v1[t]; P[2 * m + e] = v2[t]; }
      }
    }
  }
  __device__ __forceinline__ void load(const ConvShape& cs, const float* psf, const float* psf_cum,
                                       int l, int j, bool kedge) {
    load_range(cs, psf, psf_cum, l, j, kedge, 0);
  }
  __device__ __forceinline__ void store(const ConvShape& cs, float* P, bool kedge) const {
    store_range(cs, P, kedge, 0);
  }
};

// ---------------------------------------------------------------- adjoint
template <int KS>
__global__ __launch_bounds__(256, 2) void conv_back_mfma(const float* __restrict__ v,
                                                         const float* __restrict__ psf,
                                                         const float* __restrict__ psf_cum,
                                                         float* __restrict__ U, ConvShape cs,
                                                         int view0, int nvb) {
  extern __shared__ float sm[];
  float* R = sm;                               // RK x RSI: projection region + edge columns
  float* P = sm + cs.RK * cs.RSI;              // 3 x px x PL: PSF rows, suffix sums, prefix sums
  const int ntile = cs.tiles_k * cs.tiles_i;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = logical % ntile, rest = logical / ntile;
  const int tk = tile / cs.tiles_i, ti = tile - tk * cs.tiles_i;
  const int c = rest % cs.nchunk, lb = rest / cs.nchunk, l = view0 + lb;
  const int k0 = tk * 16 * cs.WK, i0 = ti * 32 * cs.WI;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
  const int wk = w / cs.WI, wi = w - wk * cs.WI;
  int j0, j1;
  chunk_range(c, cs.nchunk, cs.ny, j0, j1);
  const float* vl = v + (size_t)l * cs.nz * cs.nx;
  const int ELO = cs.RI, EHI = cs.RI + cs.px;  // edge column blocks
  const bool kedge = (k0 == 0) || (k0 + 16 * cs.WK >= cs.nz);

  // Stage the projection region once: row rk <-> input k = k0 - hb + rk (zero outside),
  // col ri <-> input i = i0 - ha + ri (zero outside); col ELO + a holds the sum of
  // v[k][i] over i <= a - ha, col EHI + a the sum over i >= nx-1 + a - ha (nx = 1: all i).
  for (int e = threadIdx.x; e < cs.RK * cs.RI; e += 256) {
    const int rk = e / cs.RI, ri = e - rk * cs.RI;
    const int kk = k0 - cs.hb + rk, ii = i0 - cs.ha + ri;
    R[rk * cs.RSI + ri] =
        (kk >= 0 && kk < cs.nz && ii >= 0 && ii < cs.nx) ? vl[(size_t)kk * cs.nx + ii] : 0.0f;
  }
  for (int e = threadIdx.x; e < cs.RK * 2; e += 256) {
    const int rk = e >> 1, hi = e & 1;
    const int kk = k0 - cs.hb + rk;
    float* dst = R + rk * cs.RSI + (hi ? EHI : ELO);
    if (kk < 0 || kk >= cs.nz) {
      for (int a = 0; a < cs.px; ++a) dst[a] = 0.0f;
      continue;
    }
    const float* row = vl + (size_t)kk * cs.nx;
    if (!hi) {
      float run = 0.0f;
      int upto = -1;                                   // sum of row[0..upto]
      for (int a = 0; a < cs.px; ++a) {
        const int t = (cs.nx == 1) ? 0 : min(a - cs.ha, cs.nx - 1);
        while (upto < t) run += row[++upto];
        dst[a] = (t < 0) ? 0.0f : run;
      }
    } else {
      for (int a = 0; a < cs.px; ++a) {
        const int t = (cs.nx == 1) ? 0 : max(cs.nx - 1 + a - cs.ha, 0);
        float run = 0.0f;
        for (int i = t; i < cs.nx; ++i) run += row[i];
        dst[a] = run;
      }
    }
  }

  // per-lane sources
  const int kout = k0 + wk * 16 + n;                               // this lane's A row (output k)
  int var = 0;
  if (cs.nz == 1 || kout == 0) var = 1;
  else if (kout == cs.nz - 1) var = 2;
  const int aoff = var * cs.px * cs.PL + g - n + 15;               // A: P[var][a][aoff + 4s]
  int colb[2];
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int iout = i0 + wi * 32 + nb * 16 + n;                   // this lane's B column
    if (cs.nx == 1 || iout == 0) colb[nb] = ELO;
    else if (iout == cs.nx - 1) colb[nb] = EHI;
    else colb[nb] = wi * 32 + nb * 16 + n;                         // + a: input i = iout + a - ha
  }
  const int rowb = (wk * 16 + g) * cs.RSI;

  // PSF rows of the next plane are prefetched into registers during the
  // current plane (with their suffix / prefix sums on z-edge tiles)
  const bool prefetch = cs.px * cs.PL <= 256 * kStagePsf;
  BackPsf pf;
  if (prefetch && j0 < j1) pf.load(cs, psf, psf_cum, l, j0, kedge);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                                               // region staged / plane consumed
    if (prefetch) {
      pf.store(cs, P, kedge);
    } else {
      BackPsf one;
      for (int base = 0; base < cs.px * cs.PL; base += 256 * kStagePsf) {
        one.load_range(cs, psf, psf_cum, l, j, kedge, base);
        one.store_range(cs, P, kedge, base);
      }
    }
    __syncthreads();
    if (prefetch && j + 1 < j1) pf.load(cs, psf, psf_cum, l, j + 1, kedge);
    floatx4 acc[4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f},
                      {0.f, 0.f, 0.f, 0.f}};
    const float* B0 = R + rowb + colb[0];
    const float* B1 = R + rowb + colb[1];
    Ops<KS> A, B;
    const float* Pa = P + aoff;
#pragma unroll
    for (int s = 0; s < kPrefetch; ++s) A.load_back(s, Pa, B0, B1, 0, cs.PL, cs.RSI);
    for (int a = 0; a < cs.px; a += 2) {
      const int a1 = min(a + 1, cs.px - 1), a2 = min(a + 2, cs.px - 1);
      tap_block<KS>(A, B, acc,
                    [&](Ops<KS>& o, int t) { o.load_back(t, Pa, B0, B1, a, cs.PL, cs.RSI); },
                    [&](Ops<KS>& o, int t) { o.load_back(t, Pa, B0, B1, a1, cs.PL, cs.RSI); });
      if (a + 1 < cs.px)
        tap_block<KS>(B, A, acc,
                      [&](Ops<KS>& o, int t) { o.load_back(t, Pa, B0, B1, a1, cs.PL, cs.RSI); },
                      [&](Ops<KS>& o, int t) { o.load_back(t, Pa, B0, B1, a2, cs.PL, cs.RSI); });
    }
    float* out = U + (size_t)lb * cs.nz * cs.ny * cs.nx + (size_t)j * cs.nx;
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const int k = k0 + wk * 16 + 4 * g + vv;
      const int i = i0 + wi * 32 + n;
      if (k < cs.nz) {
        float* row = out + (size_t)k * cs.ny * cs.nx;
        if (i < cs.nx) row[i] = acc[0][vv] + acc[2][vv];
        if (i + 16 < cs.nx) row[i + 16] = acc[1][vv] + acc[3][vv];
      }
    }
  }
}

template <int KS>
hipError_t launch_fwd_ks(const ConvShape& cs, const float* W, const float* psf, float* partial,
                         int view0, int nvb, hipStream_t s) {
  const size_t sm = conv_mfma_lds_bytes(cs, false);
  hipError_t e = hipFuncSetAttribute((const void*)conv_fwd_mfma<KS>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  dim3 grid(cs.tiles_k * cs.tiles_i * cs.nchunk * nvb);
  hipLaunchKernelGGL(conv_fwd_mfma<KS>, grid, dim3(256), sm, s, W, psf, partial, cs, view0, nvb);
  return hipGetLastError();
}

template <int KS>
hipError_t launch_back_ks(const ConvShape& cs, const float* v, const float* psf,
                          const float* psf_cum, float* U, int view0, int nvb, hipStream_t s) {
  const size_t sm = conv_mfma_lds_bytes(cs, true);
  hipError_t e = hipFuncSetAttribute((const void*)conv_back_mfma<KS>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  dim3 grid(cs.tiles_k * cs.tiles_i * cs.nchunk * nvb);
  hipLaunchKernelGGL(conv_back_mfma<KS>, grid, dim3(256), sm, s, v, psf, psf_cum, U, cs, view0,
                     nvb);
  return hipGetLastError();
}

// grid (ceil(px/64), ny, nview): suffix and prefix sums of every PSF row along b.
__global__ void psf_cum_kernel(const float* __restrict__ psf, float* __restrict__ out, int ny,
                               int pz, int px, long long total) {
  const int a = blockIdx.x * 64 + threadIdx.x;
  if (a >= px) return;
  const size_t base = ((size_t)blockIdx.z * ny + blockIdx.y) * pz * px + a;
  float run = 0.0f;
  for (int b = pz - 1; b >= 0; --b) {
    run += psf[base + (size_t)b * px];
    out[base + (size_t)b * px] = run;
  }
  run = 0.0f;
  for (int b = 0; b < pz; ++b) {
    run += psf[base + (size_t)b * px];
    out[total + base + (size_t)b * px] = run;
  }
}

}  // namespace

hipError_t launch_psf_cum(const Plan& p, float* out, hipStream_t s) {
  const spect_geom& g = p.g;
  dim3 grid((g.px + 63) / 64, g.ny, g.nview);
  hipLaunchKernelGGL(psf_cum_kernel, grid, dim3(64), 0, s, p.psf, out, g.ny, g.pz, g.px,
                     (long long)g.nview * g.ny * g.pz * g.px);
  return hipGetLastError();
}

// Row stride of a staged region: >= cols, and = 16 or 48 (mod 64) so that the
// four 16-lane row groups of a B read fall in distinct LDS banks.
static int region_stride(int cols) {
  int s = cols;
  while ((s % 64) != 16 && (s % 64) != 48) ++s;
  return s;
}

size_t conv_mfma_lds_bytes(const ConvShape& cs, bool back) {
  return back ? (size_t)(cs.RK * cs.RSI_back + 3 * cs.px * cs.PL) * sizeof(float)
              : (size_t)(cs.RK * cs.RSI + cs.px * cs.PL) * sizeof(float);
}

bool conv_mfma_supported(const spect_geom& g) {
  const int ks = (15 + g.pz + 3) / 4;
  if (ks < 4 || ks > kMaxMfmaKSteps) return false;
  ConvShape cs = make_conv_shape(g, kFwdJChunk, kBackJChunk);
  return conv_mfma_lds_bytes(cs, false) <= kLdsBytes && conv_mfma_lds_bytes(cs, true) <= kLdsBytes;
}

ConvShape make_conv_shape(const spect_geom& g, int jc_fwd, int jc_back) {
  ConvShape cs;
  cs.nx = g.nx; cs.ny = g.ny; cs.nz = g.nz; cs.px = g.px; cs.pz = g.pz;
  cs.ha = (g.px - 1) / 2; cs.hb = (g.pz - 1) / 2;
  cs.KS = (15 + g.pz + 3) / 4;
  cs.WI = g.nx > 64 ? 4 : (g.nx > 32 ? 2 : 1);
  cs.WK = 4 / cs.WI;
  cs.tiles_k = (g.nz + 16 * cs.WK - 1) / (16 * cs.WK);
  cs.tiles_i = (g.nx + 32 * cs.WI - 1) / (32 * cs.WI);
  cs.RK = 16 * (cs.WK - 1) + 4 * cs.KS;        // rows read by the last k-step of the last wave
  cs.RI = 32 * cs.WI + g.px - 1;
  cs.RSI = region_stride(cs.RI);
  cs.RSI_back = region_stride(cs.RI + 2 * g.px);
  cs.PL = 4 * cs.KS + 15;
  cs.Z = 4 * cs.KS - 1 - 2 * cs.hb;
  cs.jc = jc_fwd;
  cs.nchunk = (g.ny + jc_fwd - 1) / jc_fwd;
  cs.jc_back = jc_back;
  cs.nchunk_back = (g.ny + jc_back - 1) / jc_back;
  cs.nview_ny_pz_px = (long long)g.nview * g.ny * g.pz * g.px;
  return cs;
}

// Workgroups of one launch resident per CU (HIP occupancy query).
template <int KS>
int wgs_per_cu_ks(const ConvShape& cs, bool back) {
  int nb = 0;
  const size_t sm = conv_mfma_lds_bytes(cs, back);
  hipError_t e = back ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, (const void*)conv_back_mfma<KS>, 256, sm)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                            &nb, (const void*)conv_fwd_mfma<KS>, 256, sm);
  if (e != hipSuccess || nb < 1) nb = (int)(kLdsBytes / (sm ? sm : 1));
  return nb < 1 ? 1 : nb;
}

// Depth chunks per (tile, view): minimise rounds * planes-per-workgroup, the
// length of the schedule when the resident slots are refilled in waves.
static int pick_chunks(int ny, long long tiles_views, long long slots) {
  int best = 1;
  long long best_cost = -1;
  for (int n = 1; n <= kMaxChunks && n <= ny; ++n) {
    const long long wgs = tiles_views * n;
    const long long rounds = (wgs + slots - 1) / slots;
    const long long cost = rounds * ((ny + n - 1) / n);
    if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = n; }
  }
  return best;
}

#define SPECT_KS_CASES(X) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20)

hipError_t launch_conv_fwd_mfma(const Plan& p, const float* W, float* partial, int view0, int nvb,
                                hipStream_t s) {
  const ConvShape& cs = p.conv;
  switch (cs.KS) {
#define CASE(K) case K: return launch_fwd_ks<K>(cs, W, p.psf, partial, view0, nvb, s);
    SPECT_KS_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_conv_back_mfma(const Plan& p, const float* v, float* U, int view0, int nvb,
                                 hipStream_t s) {
  ConvShape cs = p.conv;
  cs.RSI = cs.RSI_back;
  cs.jc = cs.jc_back;
  cs.nchunk = cs.nchunk_back;
  switch (cs.KS) {
#define CASE(K) case K: return launch_back_ks<K>(cs, v, p.psf, p.psf_cum, U, view0, nvb, s);
    SPECT_KS_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spect

namespace spect {
void tune_conv_chunks(ConvShape& cs, int views) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    return;
  int fw = 1, bw = 1;
  switch (cs.KS) {
#define CASE(K) case K: fw = wgs_per_cu_ks<K>(cs, false); bw = wgs_per_cu_ks<K>(cs, true); break;
    SPECT_KS_CASES(CASE)
#undef CASE
    default: return;
  }
  const long long tv = (long long)cs.tiles_k * cs.tiles_i * views;
  cs.nchunk = pick_chunks(cs.ny, tv, (long long)cus * fw);
  cs.nchunk_back = pick_chunks(cs.ny, tv, (long long)cus * bw);
  cs.jc = (cs.ny + cs.nchunk - 1) / cs.nchunk;
  cs.jc_back = (cs.ny + cs.nchunk_back - 1) / cs.nchunk_back;
}
}  // namespace spect
