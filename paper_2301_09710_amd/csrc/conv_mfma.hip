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
// staged once with zero padding, and compute the zero-padded correlation,
// which is the exact adjoint at every bin off the edge rows (k = 0, nz-1)
// and columns (i = 0, nx-1).  Replicate padding's adjoint folds the border
// onto those edges; conv_back_edges recomputes the edge bins exactly as a
// small dense MFMA product over cumulative sums of the projection (planes as
// rows), so the main kernel stays uniform across lanes.
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
  // adjoint: A = P[a][aoff + 4s], B = R[boff + a + 4s RSI (+16)]
  __device__ __forceinline__ void load_back(int s, const float* Pa, const float* Rb, int a, int PL,
                                            int RSI) {
    av[s] = Pa[a * PL + 4 * s];
    b0[s] = Rb[4 * s * RSI + a];
    b1[s] = Rb[4 * s * RSI + a + 16];
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

// Per-thread staging of one adjoint plane's PSF rows: P[a][b + 15].
struct BackPsf {
  float v0[kStagePsf];
  __device__ __forceinline__ void load_range(const ConvShape& cs, const float* __restrict__ psf,
                                             int l, int j, int base) {
    const float* pj = psf + ((size_t)l * cs.ny + j) * cs.pz * cs.px;
#pragma unroll
    for (int t = 0; t < kStagePsf; ++t) {
      const int e = base + threadIdx.x + 256 * t;
      float x0 = 0.0f;
      if (e < cs.px * cs.PL) {
        const int a = e / cs.PL, b = e - a * cs.PL - 15;
        if (b >= 0 && b < cs.pz) x0 = pj[b * cs.px + a];
      }
      v0[t] = x0;
    }
  }
  __device__ __forceinline__ void store_range(const ConvShape& cs, float* P, int base) const {
#pragma unroll
    for (int t = 0; t < kStagePsf; ++t) {
      const int e = base + threadIdx.x + 256 * t;
      if (e < cs.px * cs.PL) P[e] = v0[t];
    }
  }
};

// ---------------------------------------------------------------- adjoint
// Interior formula for every output bin of a tile:
//   u[k][i] = sum_{a,b} p[a,b] v[k + b - hb][i + a - ha]   (v zero outside)
// which is the exact adjoint everywhere except on the edge rows k = 0, nz-1
// and edge columns i = 0, nx-1, where replicate padding folds the border;
// conv_back_edges overwrites those afterwards.
template <int KS>
__global__ __launch_bounds__(256, 2) void conv_back_mfma(const float* __restrict__ v,
                                                         const float* __restrict__ psf,
                                                         float* __restrict__ U, ConvShape cs,
                                                         int view0, int nvb) {
  extern __shared__ float sm[];
  float* R = sm;                               // RK x RSI: zero-padded projection region
  float* P = sm + cs.RK * cs.RSI;              // px x PL: PSF rows
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

  // region row rk <-> input k = k0 - hb + rk, column ri <-> input i = i0 - ha + ri
  for (int e = threadIdx.x; e < cs.RK * cs.RI; e += 256) {
    const int rk = e / cs.RI, ri = e - rk * cs.RI;
    const int kk = k0 - cs.hb + rk, ii = i0 - cs.ha + ri;
    R[rk * cs.RSI + ri] =
        (kk >= 0 && kk < cs.nz && ii >= 0 && ii < cs.nx) ? vl[(size_t)kk * cs.nx + ii] : 0.0f;
  }
  // A[m][r] = p[a][b = r - m] (row offset 15), B = R[(16 wk + g + 4s) RSI + 32 wi + n + a (+16)]
  const int aoff = g - n + 15;
  const int boff = (wk * 16 + g) * cs.RSI + wi * 32 + n;
  // PSF rows of the next plane are prefetched into registers during the current one
  const bool prefetch = cs.px * cs.PL <= 256 * kStagePsf;
  BackPsf pf;
  if (prefetch && j0 < j1) pf.load_range(cs, psf, l, j0, 0);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                                               // region staged / plane consumed
    if (prefetch) {
      pf.store_range(cs, P, 0);
    } else {
      BackPsf one;
      for (int base = 0; base < cs.px * cs.PL; base += 256 * kStagePsf) {
        one.load_range(cs, psf, l, j, base);
        one.store_range(cs, P, base);
      }
    }
    __syncthreads();
    if (prefetch && j + 1 < j1) pf.load_range(cs, psf, l, j + 1, 0);
    floatx4 acc[4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f},
                      {0.f, 0.f, 0.f, 0.f}};
    Ops<KS> A, B;
    const float* Pa = P + aoff;
    const float* Rb = R + boff;
#pragma unroll
    for (int s = 0; s < kPrefetch; ++s) A.load_back(s, Pa, Rb, 0, cs.PL, cs.RSI);
    for (int a = 0; a < cs.px; a += 2) {
      const int a1 = min(a + 1, cs.px - 1), a2 = min(a + 2, cs.px - 1);
      tap_block<KS>(A, B, acc,
                    [&](Ops<KS>& o, int t) { o.load_back(t, Pa, Rb, a, cs.PL, cs.RSI); },
                    [&](Ops<KS>& o, int t) { o.load_back(t, Pa, Rb, a1, cs.PL, cs.RSI); });
      if (a + 1 < cs.px)
        tap_block<KS>(B, A, acc,
                      [&](Ops<KS>& o, int t) { o.load_back(t, Pa, Rb, a1, cs.PL, cs.RSI); },
                      [&](Ops<KS>& o, int t) { o.load_back(t, Pa, Rb, a2, cs.PL, cs.RSI); });
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

// ---------------------------------------------------------------- adjoint, edges
// Exact adjoint on the edge rows and columns of every depth plane of a view,
// overwriting what conv_back_mfma wrote there.  For an output bin (k', i')
//   u = sum_{a,b} p[a,b] * sum { v[k][i] : clamp(k - b + hb) = k',
//                                          clamp(i - a + ha) = i' }.
// On an edge row k' (0 or nz-1) the k-sum depends only on (b, i), so with
// Tk[b][i] = sum_{k in K(b)} v[k][i] the plane's row is
//   u[k'][i'] = sum_a sum_b p[a,b,j] Tk[b][i' + a - ha]   (Tk zero outside),
// a dense product over b with the depth planes j as rows (M), the bins i' as
// columns (N), looped over a: no band waste.  Corner bins (i' = 0, nx-1)
// also fold along i: their B value is sum_{i in I(a)} Tk[b][i].  Edge columns
// are the same with the roles of (a, i) and (b, k) swapped, rows excluded.
// Tk[b] vanishes unless the fold set K(b) is nonempty: b >= hb on the edge
// k' = 0 and b <= hb on k' = nz-1 (every b when nz = 1), so K runs over that
// window only, about half of the taps.
// grid: (nvb, 2 edges of one kind, ceil(ny / 64)); each wave owns 16 planes.
// Rows and columns are two launches, each with its own NB (N-blocks per pass).
constexpr int kEdgeMaxNB = 9;

// Sizes of the edge problem: q = taps contracted in K (along the folded
// axis), t = taps looped outside, o = output bins along the edge line.
struct EdgeDims {
  int nq, hq, nt, ht, nout, nfold, ksteps, nqs, TWp;
};
__host__ __device__ inline EdgeDims edge_dims(const ConvShape& cs, bool krow) {
  EdgeDims d;
  d.nq = krow ? cs.pz : cs.px;
  d.hq = krow ? cs.hb : cs.ha;
  d.nt = krow ? cs.px : cs.pz;
  d.ht = krow ? cs.ha : cs.hb;
  d.nout = krow ? cs.nx : cs.nz;
  d.nfold = krow ? cs.nz : cs.nx;
  // K window: the taps with a possibly nonempty fold set, the same length on both edges
  const int nwin = d.nfold > 1 ? (d.nq - d.hq > d.hq + 1 ? d.nq - d.hq : d.hq + 1) : d.nq;
  d.ksteps = (nwin + 3) / 4;
  d.nqs = 4 * d.ksteps;                                         // padded with zero rows
  d.TWp = 16 * ((d.nout + 15) / 16) + 2 * d.ht;                 // columns read by the N-blocks
  return d;
}

template <int NB>
__global__ __launch_bounds__(256) void conv_back_edges(const float* __restrict__ v,
                                                       const float* __restrict__ psf,
                                                       float* __restrict__ U, ConvShape cs,
                                                       int view0, int kind0) {
  extern __shared__ float sm[];
  const int lb = blockIdx.x, kind = kind0 + blockIdx.y, l = view0 + lb;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4;
  const int jblk = blockIdx.z * 64 + w * 16;                     // this wave's 16 planes
  const bool krow = kind < 2;                                    // edge row (k) or column (i)
  // skip duplicates of a size-1 axis (both edges are the same line)
  if ((kind == 1 && cs.nz == 1) || (kind == 3 && cs.nx == 1)) return;
  if (!krow && cs.nz <= 2) return;                               // no interior rows to fix
  const float* vl = v + (size_t)l * cs.nz * cs.nx;
  EdgeDims d = edge_dims(cs, krow);
  const int eout = (kind & 1) ? d.nfold - 1 : 0;  // the edge position on the folded axis
  const int qlo = (eout == 0 && d.nfold > 1) ? d.hq : 0;         // first tap of the K window
  float* T = sm;                                  // nqs x TWp: folded sums, zero-padded
  float* Cx = T + d.nqs * d.TWp;                  // nqs x nt x 2: corner sums, then one zero
  float* As = Cx + (krow ? d.nqs * d.nt * 2 + 1 : 1);  // 256 x nt: per-lane A scratch
  // The fold sets of an edge lie within hq + 1 lines of it: stage that band of the
  // projection (lines along the folded axis, bins along the edge) in the A scratch.
  const int bw = min(d.hq + 1, d.nfold);
  const int fbase = (eout == 0) ? 0 : d.nfold - bw;              // first folded line staged
  float* Vb = As;                                                // bw x nout
  for (int e = threadIdx.x; e < bw * d.nout; e += 256) {
    const int f = e / d.nout, o = e - f * d.nout;
    Vb[e] = krow ? vl[(size_t)(fbase + f) * cs.nx + o] : vl[(size_t)o * cs.nx + fbase + f];
  }
  if (threadIdx.x == 0) Cx[krow ? d.nqs * d.nt * 2 : 0] = 0.0f;   // zero slot of empty N-blocks
  __syncthreads();

  // T[q - qlo][c] = sum over f in F(q) of v at (fold f, other c - ht), with
  // F(q) = {f : clamp(f - q + hq) = eout}.  The sets grow monotonically in q
  // (ascending for eout = 0, descending for eout = nfold-1), so one running
  // sum per column fills every q with additions only; rows outside the taps
  // (q >= nq) are zero.
  const bool up = (eout == 0);
  const int qend = max(d.nq, qlo + d.nqs);
  for (int cc = threadIdx.x; cc < d.TWp; cc += 256) {
    const int o = cc - d.ht;
    const bool live = o >= 0 && o < d.nout;
    float sum = 0.0f;
    int clo = 0, chi = -1;                                        // current set [clo, chi]
    for (int step = 0; step < qend; ++step) {
      const int q = up ? step : qend - 1 - step;
      int flo = (eout == 0) ? 0 : eout + q - d.hq;
      int fhi = (eout == d.nfold - 1) ? d.nfold - 1 : eout + q - d.hq;
      flo = max(flo, 0);
      fhi = min(fhi, d.nfold - 1);
      const bool ok = live && q < d.nq && flo <= fhi;
      if (ok) {
        if (chi < clo) { clo = fhi + 1; chi = fhi; }            // start empty at the fixed end
        for (int f = clo - 1; f >= flo; --f) sum += Vb[(f - fbase) * d.nout + o];
        for (int f = chi + 1; f <= fhi; ++f) sum += Vb[(f - fbase) * d.nout + o];
        clo = min(clo, flo);
        chi = max(chi, fhi);
      }
      if (q >= qlo && q < qlo + d.nqs) T[(q - qlo) * d.TWp + cc] = ok ? sum : 0.0f;
    }
  }
  __syncthreads();
  // corners (edge rows only): Cx[q - qlo][t][side] = sum over o in O_side(t) of
  // T[q - qlo][o + ht]; Cx[nqs nt 2] is a zero read by the other lanes of the corner N-block
  if (krow) {
    for (int e = threadIdx.x; e < d.nqs * d.nt * 2 + 1; e += 256) Cx[e] = 0.0f;
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * d.nqs; e += 256) {
      const int side = e / d.nqs, qq = e - side * d.nqs;         // qq = q - qlo
      if (qlo + qq >= d.nq) continue;
      const int oe = side ? d.nout - 1 : 0;
      const bool oup = (oe == 0);
      float sum = 0.0f;
      int clo = 0, chi = -1;
      for (int step = 0; step < d.nt; ++step) {
        const int t = oup ? step : d.nt - 1 - step;
        int olo = (oe == 0) ? 0 : oe + t - d.ht;
        int ohi = (oe == d.nout - 1) ? d.nout - 1 : oe + t - d.ht;
        olo = max(olo, 0);
        ohi = min(ohi, d.nout - 1);
        if (olo <= ohi) {
          if (chi < clo) { clo = ohi + 1; chi = ohi; }
          for (int o = clo - 1; o >= olo; --o) sum += T[qq * d.TWp + o + d.ht];
          for (int o = chi + 1; o <= ohi; ++o) sum += T[qq * d.TWp + o + d.ht];
          clo = min(clo, olo);
          chi = max(chi, ohi);
        }
        if (!(side == 1 && d.nout == 1)) Cx[(qq * d.nt + t) * 2 + side] = (olo <= ohi) ? sum : 0.0f;
      }
    }
    __syncthreads();
  }
  if (jblk >= cs.ny) return;
  const int jm = min(jblk + n, cs.ny - 1);                       // A row (plane); clamped rows unused
  const float* pj = psf + ((size_t)l * cs.ny + jm) * cs.pz * cs.px;
  float* Al = As + ((size_t)w * 64 + lane) * d.nt;
  // N-blocks: the bins 0 .. nout-1 (edge bins of rows excluded: corners), then for rows one
  // block whose lanes 0 and 1 are the two corners
  const int nblocks = (d.nout + 15) / 16;
  const int nall = nblocks + (krow ? 1 : 0);
  for (int nb0 = 0; nb0 < nall; nb0 += NB) {
    floatx4 acc[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) acc[u] = {0.f, 0.f, 0.f, 0.f};
    for (int s = 0; s < d.ksteps; ++s) {
      const int qq = 4 * s + g, q = qlo + qq;                    // K index of this lane
      // A[m = plane][K = q] = p[a][b]: krow -> (a = t, b = q), else (a = q, b = t)
      for (int t0 = 0; t0 < d.nt; t0 += 16) {                   // 16 independent loads at a time
        float r16[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int t = t0 + u;
          r16[u] = (q < d.nq && t < d.nt) ? (krow ? pj[q * cs.px + t] : pj[t * cs.px + q]) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (t0 + u < d.nt) Al[t0 + u] = r16[u];
      }
      // B source of each N-block for this lane: a pointer advanced by `step` per tap t
      const float* zero = Cx + (krow ? d.nqs * d.nt * 2 : 0);   // a zero slot
      const float* bp[NB];
      int bst[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int blk = nb0 + u;
        if (blk < nblocks) { bp[u] = T + qq * d.TWp + 16 * blk + n; bst[u] = 1; }
        else if (blk == nblocks && krow && n < 2) { bp[u] = Cx + qq * d.nt * 2 + n; bst[u] = 2; }
        else { bp[u] = zero; bst[u] = 0; }
      }
      // pipelined over taps: the operands of t+1 are read while t's MFMAs run
      float avA, avB, bvA[NB], bvB[NB];
      auto load = [&](float& av, float (&bv)[NB], int t) {
        av = Al[t];
#pragma unroll
        for (int u = 0; u < NB; ++u) bv[u] = bp[u][t * bst[u]];
      };
      auto run = [&](float av, const float (&bv)[NB]) {
#pragma unroll
        for (int u = 0; u < NB; ++u) acc[u] = mfma(av, bv[u], acc[u]);
      };
      load(avA, bvA, 0);
      for (int t = 0; t < d.nt; t += 2) {
        load(avB, bvB, min(t + 1, d.nt - 1));
        __builtin_amdgcn_sched_barrier(0);
        run(avA, bvA);
        __builtin_amdgcn_sched_barrier(0);
        load(avA, bvA, min(t + 2, d.nt - 1));
        __builtin_amdgcn_sched_barrier(0);
        if (t + 1 < d.nt) run(avB, bvB);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // D[4g + r][n]: plane jblk + 4g + r, output position of (block, lane)
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int blk = nb0 + u;
      int o;
      if (blk < nblocks) {
        o = 16 * blk + n;
        if (o >= d.nout || o == 0 || o == d.nout - 1) continue;  // edge bins: corner block / rows
      } else if (blk == nblocks && krow && n < 2 && !(n == 1 && d.nout == 1)) {
        o = n ? d.nout - 1 : 0;
      } else {
        continue;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jblk + 4 * g + r;
        if (j >= cs.ny) continue;
        const int k = krow ? eout : o, i = krow ? o : eout;
        U[(((size_t)lb * cs.nz + k) * cs.ny + j) * cs.nx + i] = acc[u][r];
      }
    }
  }
}

// N-blocks per pass for nall blocks: issued blocks plus the fixed cost of a
// pass (its PSF loads and K loop, about three blocks' worth), then fewer passes.
int edge_pick_nb(int nall) {
  int best = kEdgeMaxNB, cost = -1;
  for (int nb = kEdgeMaxNB; nb >= 1; --nb) {
    const int passes = (nall + nb - 1) / nb;
    const int c = passes * nb + 3 * passes;
    if (cost < 0 || c < cost) { cost = c; best = nb; }
  }
  return best;
}

size_t edge_lds_floats(const ConvShape& cs, bool krow) {
  const EdgeDims e = edge_dims(cs, krow);
  const size_t band = (size_t)(e.hq + 1 < e.nfold ? e.hq + 1 : e.nfold) * e.nout;
  const size_t lanes = 256 * (size_t)e.nt;
  const size_t scratch = band > lanes ? band : lanes;
  return (size_t)e.nqs * e.TWp + (krow ? (size_t)e.nqs * e.nt * 2 + 1 : 1) + scratch;
}

template <int NB>
hipError_t launch_edges_nb(const ConvShape& cs, const float* v, const float* psf, float* U,
                           int view0, int nvb, bool krow, hipStream_t s) {
  const size_t sm = edge_lds_floats(cs, krow) * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)conv_back_edges<NB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  dim3 grid(nvb, 2, (cs.ny + 63) / 64);
  hipLaunchKernelGGL(conv_back_edges<NB>, grid, dim3(256), sm, s, v, psf, U, cs, view0,
                     krow ? 0 : 2);
  return hipGetLastError();
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
hipError_t launch_back_ks(const ConvShape& cs, const float* v, const float* psf, float* U,
                          int view0, int nvb, hipStream_t s) {
  const size_t sm = conv_mfma_lds_bytes(cs, true);
  hipError_t e = hipFuncSetAttribute((const void*)conv_back_mfma<KS>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  dim3 grid(cs.tiles_k * cs.tiles_i * cs.nchunk * nvb);
  hipLaunchKernelGGL(conv_back_mfma<KS>, grid, dim3(256), sm, s, v, psf, U, cs, view0, nvb);
  return hipGetLastError();
}

}  // namespace

// Row stride of a staged region: >= cols, and = 16 or 48 (mod 64) so that the
// four 16-lane row groups of a B read fall in distinct LDS banks.
static int region_stride(int cols) {
  int s = cols;
  while ((s % 64) != 16 && (s % 64) != 48) ++s;
  return s;
}

size_t conv_mfma_lds_bytes(const ConvShape& cs, bool back) {
  return back ? (size_t)(cs.RK * cs.RSI_back + cs.px * cs.PL) * sizeof(float)
              : (size_t)(cs.RK * cs.RSI + cs.px * cs.PL) * sizeof(float);
}

bool conv_mfma_supported(const spect_geom& g) {
  const int ks = (15 + g.pz + 3) / 4;
  if (ks < 4 || ks > kMaxMfmaKSteps) return false;
  ConvShape cs = make_conv_shape(g, kFwdJChunk, kBackJChunk);
  return conv_mfma_lds_bytes(cs, false) <= kLdsBytes && conv_mfma_lds_bytes(cs, true) <= kLdsBytes &&
         conv_edges_lds_bytes(cs) <= kLdsBytes;
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
  cs.RSI_back = region_stride(cs.RI);
  cs.PL = 4 * cs.KS + 15;
  cs.Z = 4 * cs.KS - 1 - 2 * cs.hb;
  cs.jc = jc_fwd;
  cs.nchunk = (g.ny + jc_fwd - 1) / jc_fwd;
  cs.jc_back = jc_back;
  cs.nchunk_back = (g.ny + jc_back - 1) / jc_back;
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
  if (p.use_m4) return launch_conv_m4(p, false, W, partial, view0, nvb, s);
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
  if (p.use_m4) return launch_conv_m4(p, true, v, U, view0, nvb, s);
  ConvShape cs = p.conv;
  cs.RSI = cs.RSI_back;
  cs.jc = cs.jc_back;
  cs.nchunk = cs.nchunk_back;
  switch (cs.KS) {
#define CASE(K) case K: return launch_back_ks<K>(cs, v, p.psf, U, view0, nvb, s);
    SPECT_KS_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spect

namespace spect {
size_t conv_edges_lds_bytes(const ConvShape& cs) {
  const size_t r = edge_lds_floats(cs, true), c = edge_lds_floats(cs, false);
  return (r > c ? r : c) * sizeof(float);
}

hipError_t launch_conv_back_edges(const Plan& p, const float* v, float* U, int view0, int nvb,
                                  hipStream_t s) {
  const ConvShape& cs = p.conv;
  for (int pass = 0; pass < 2; ++pass) {
    const bool krow = pass == 0;
    if (!krow && cs.nz <= 2) break;                       // no interior rows: no column edges
    const int nall = (krow ? cs.nx : cs.nz) / 16 + ((krow ? cs.nx : cs.nz) % 16 != 0) + krow;
    hipError_t e;
    switch (edge_pick_nb(nall)) {
      case 1: e = launch_edges_nb<1>(cs, v, p.psf, U, view0, nvb, krow, s); break;
      case 2: e = launch_edges_nb<2>(cs, v, p.psf, U, view0, nvb, krow, s); break;
      case 3: e = launch_edges_nb<3>(cs, v, p.psf, U, view0, nvb, krow, s); break;
      case 4: e = launch_edges_nb<4>(cs, v, p.psf, U, view0, nvb, krow, s); break;
      case 5: e = launch_edges_nb<5>(cs, v, p.psf, U, view0, nvb, krow, s); break;
      case 6: e = launch_edges_nb<6>(cs, v, p.psf, U, view0, nvb, krow, s); break;
      case 7: e = launch_edges_nb<7>(cs, v, p.psf, U, view0, nvb, krow, s); break;
      case 8: e = launch_edges_nb<8>(cs, v, p.psf, U, view0, nvb, krow, s); break;
      default: e = launch_edges_nb<9>(cs, v, p.psf, U, view0, nvb, krow, s); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

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
