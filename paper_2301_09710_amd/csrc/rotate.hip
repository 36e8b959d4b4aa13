// Rotation kernels (Sec. II-A): rotate activity and attenuation slices by
// theta_l with an exact quarter turn and three 1-D linear-interpolation
// shears, form the attenuation factor of Eq. (1), weight; and the exact
// transpose of those steps accumulated over views (Alg. 2).
//
// One workgroup owns one z-slice (n x n, n = nx = ny) and loops over several
// views.  Each pass is a two-tap gather along rows or columns with per-line
// offset and weights from the host tables:
//   forward   out[q] = w.x in[q + o] + w.y in[q + o + 1]
//   transpose out[q] = w.x in[q - o] + w.y in[q - o - 1]
// with every sample outside [0, n) equal to zero.  The quarter turn P_m is
// an affine remapping of cell addresses; the transpose applies P_m^T last,
// on the way into the accumulators.
//
// Slices that fit LDS (3-pass): rot_fwd_lines_kernel stages P_m x per view
// into a zero-guarded buffer and runs the three passes in place, each wave
// owning whole lines, with the attenuation weight fused into the last pass;
// rot_back_lines_kernel (n <= 128) runs the transposed passes the same way,
// the last one (S1^T) inside the gather into its accumulators.
// The attenuation kernel runs the passes in sequence on slices of odd row
// stride n + 1 (row passes, column passes and quarter-turned reads are then
// free of bank conflicts).
//
// With SPECT_ROT_BILINEAR the three passes are replaced by one 2-D bilinear
// gather per pixel after the same quarter turn (forward and attenuation), and
// the transpose gathers, for each pixel, the output pixels whose samples used
// it (see bil_adj_px).  rot_fwd_kernel (one gather per output pixel from a
// single staged slice, the three passes fused or the bilinear sample) and
// rot_back_kernel (the passes in sequence) serve the bilinear rotation and
// slices above the LDS limit, whose working slices then live in global
// scratch and whose column passes run through LDS in bands of columns.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace spect {
namespace {

constexpr int NT = kRotThreads;
constexpr int NW = NT / 64;                                   // waves per workgroup

__host__ __device__ __forceinline__ int slice_stride(int n) { return n + 1; }

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

// One line's two-tap interpolation: weights (w.x, w.y) and offset o, packed
// so that a lookup is a single 16-byte LDS read.
struct __align__(16) TabEntry {
  float2 w;
  int o, pad;
};

struct ViewTab {          // per-view tables in LDS
  TabEntry* e13;          // passes 1 and 3, indexed by row j
  TabEntry* e2;           // pass 2, indexed by column i
};

__device__ __forceinline__ bool inside(int q, int n) { return (unsigned)q < (unsigned)n; }

// Tables (2n entries) at `after`, which callers keep 16-byte aligned.
__device__ __forceinline__ ViewTab carve_tab(float* after, int n) {
  ViewTab t;
  t.e13 = reinterpret_cast<TabEntry*>(after);
  t.e2 = t.e13 + n;
  return t;
}

// Floats of an LDS slice rounded up to 16 bytes.
__host__ __device__ __forceinline__ int round4(int floats) { return (floats + 3) & ~3; }

__device__ __forceinline__ void load_tab(const Tables& tab, int l, int n, const ViewTab& t) {
  const int2* off = reinterpret_cast<const int2*>(tab.off) + (size_t)l * 2 * n;
  const float2* w = tab.w + (size_t)l * 2 * n;
  for (int e = threadIdx.x; e < 2 * n; e += NT) {
    TabEntry te;                       // e13 and e2 are contiguous: [0, n) rows, [n, 2n) columns
    const int2 o = off[e];
    te.w = w[e];
    te.o = o.x;
    te.pad = o.y;
    t.e13[e] = te;
  }
}

__device__ __forceinline__ void stage_slice(float* X, const float* __restrict__ src, int n, int S) {
  for (int p = threadIdx.x; p < n * n; p += NT) {
    const int j = p / n, i = p - j * n;
    X[j * S + i] = src[p];
  }
}

// Line ownership: wave w owns lines w, w + NW, ...; lane l covers positions
// l, l + 64, ... (EPL = elements per lane) of a line.
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// pass 1 (forward) read from the unrotated slice X through the quarter turn
__device__ __forceinline__ float pass1_px(const float* X, int n, const QAddr& qa,
                                          const ViewTab& t, int i, int j) {
  const TabEntry te = t.e13[j];
  const int o = te.o;
  const float2 w = te.w;
  const int ia = i + o, ib = ia + 1;
  const float a = inside(ia, n) ? X[qa.base + qa.ci * ia + qa.cj * j] : 0.0f;
  const float b = inside(ib, n) ? X[qa.base + qa.ci * ib + qa.cj * j] : 0.0f;
  return w.x * a + w.y * b;
}

// row pass (along i) on Y: forward (kSgn = +1) or transpose (kSgn = -1)
template <int kSgn>
__device__ __forceinline__ float row_px(const float* Y, int n, int S, const ViewTab& t, int i,
                                        int j) {
  const TabEntry te = t.e13[j];
  const int o = te.o;
  const float2 w = te.w;
  const int ia = i + kSgn * o, ib = ia + kSgn;
  // unsigned offsets (nonnegative where read): a uniform base plus a 32-bit
  // offset when Y is in global memory
  const float a = inside(ia, n) ? Y[(unsigned)(j * S + ia)] : 0.0f;
  const float b = inside(ib, n) ? Y[(unsigned)(j * S + ib)] : 0.0f;
  return w.x * a + w.y * b;
}

// column pass (along j) on Y: forward or transpose
template <int kSgn>
__device__ __forceinline__ float col_px(const float* Y, int n, int S, const ViewTab& t, int i,
                                        int j) {
  const TabEntry te = t.e2[i];
  const int o = te.o;
  const float2 w = te.w;
  const int ja = j + kSgn * o, jb = ja + kSgn;
  const float a = inside(ja, n) ? Y[ja * S + i] : 0.0f;
  const float b = inside(jb, n) ? Y[jb * S + i] : 0.0f;
  return w.x * a + w.y * b;
}

// ---------------------------------------------------------------- bilinear
// 2-D bilinear rotation, the alternative to the 3-pass shears: output pixel
// p = (i, j) samples the quarter-turned slice at s(p) = R(phi)^-1 (p - c) + c
// with zero padding.  The tables hold the terms of s as integer part plus
// fraction, a column term in i (t.e2) and a row term in j (t.e13), so a
// sample position costs two integer and two float additions.
struct BilPos { int qi, qj; float fi, fj; };
__device__ __forceinline__ BilPos bil_pos(const ViewTab& t, int i, int j) {
  const TabEntry a = t.e2[i], b = t.e13[j];
  BilPos p;
  p.qi = a.o + b.o;
  p.qj = a.pad + b.pad;
  p.fi = a.w.x + b.w.x;
  p.fj = a.w.y + b.w.y;
  if (p.fi >= 1.0f) { p.fi -= 1.0f; ++p.qi; }
  if (p.fj >= 1.0f) { p.fj -= 1.0f; ++p.qj; }
  return p;
}

// (B P_m x)(i, j) from the unrotated slice X, read through the quarter turn.
__device__ __forceinline__ float bil_px(const float* X, int n, const QAddr& qa, const ViewTab& t,
                                        int i, int j) {
  const BilPos p = bil_pos(t, i, j);
  float v = 0.0f;
#pragma unroll
  for (int dj = 0; dj < 2; ++dj) {
    const int jj = p.qj + dj;
    if (!inside(jj, n)) continue;
    const int row = qa.base + __mul24(qa.cj, jj);
    const int ia = p.qi, ib = ia + 1;
    const float a = inside(ia, n) ? X[row + __mul24(qa.ci, ia)] : 0.0f;
    const float b = inside(ib, n) ? X[row + __mul24(qa.ci, ib)] : 0.0f;
    v += (dj ? p.fj : 1.0f - p.fj) * ((1.0f - p.fi) * a + p.fi * b);
  }
  return v;
}

// (B^T Y)(qi, qj): the sum over the output pixels p whose sample uses
// (qi, qj), i.e. |s(p) - q| < 1 on both axes.  Those p lie within sqrt(2) of
// R(phi)(q - c) + c for |phi| <= pi/4, so the 3 x 3 pixels around its
// rounding cover them; each weight is recomputed from the tables exactly as
// the forward computes it.  cs = (cos phi, sin phi), c = (n - 1) / 2.
__device__ __forceinline__ float bil_adj_px(const float* Y, int n, int S, const ViewTab& t,
                                            float2 cs, float c, int qi, int qj) {
  const float u = (float)qi - c, v = (float)qj - c;
  const int pi0 = __float2int_rn(c + cs.x * u - cs.y * v) - 1;
  const int pj0 = __float2int_rn(c + cs.y * u + cs.x * v) - 1;
  // the three column and three row terms of the candidates, loaded once;
  // outside the grid a candidate gets an entry that can never hit q
  TabEntry ca[3], rb[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int pi = pi0 + d, pj = pj0 + d;
    ca[d] = inside(pi, n) ? t.e2[pi] : TabEntry{make_float2(0.0f, 0.0f), -4 * n, 0};
    rb[d] = inside(pj, n) ? t.e13[pj] : TabEntry{make_float2(0.0f, 0.0f), 0, -4 * n};
  }
  float acc = 0.0f;
#pragma unroll
  for (int dj = 0; dj < 3; ++dj) {
    const int pj = min(max(pj0 + dj, 0), n - 1);          // address only; weight 0 outside
#pragma unroll
    for (int di = 0; di < 3; ++di) {
      const int pi = min(max(pi0 + di, 0), n - 1);
      int ri = ca[di].o + rb[dj].o, rj = ca[di].pad + rb[dj].pad;
      float fi = ca[di].w.x + rb[dj].w.x, fj = ca[di].w.y + rb[dj].w.y;
      if (fi >= 1.0f) { fi -= 1.0f; ++ri; }
      if (fj >= 1.0f) { fj -= 1.0f; ++rj; }
      const float wi = qi == ri ? 1.0f - fi : (qi == ri + 1 ? fi : 0.0f);
      const float wj = qj == rj ? 1.0f - fj : (qj == rj + 1 ? fj : 0.0f);
      acc += wj * (wi * Y[pj * S + pi]);
    }
  }
  return acc;
}

// In-place pass over the lines a wave owns: each line is read completely
// (every lane's taps) before any lane writes it, so no workgroup barrier is
// needed inside the pass; EPL values per lane are held in registers.
template <int kSgn, bool kRows, int EPL>
__device__ __forceinline__ void line_pass(float* Y, int n, int S, const ViewTab& t) {
  const int lane = lane_id();
  for (int line = wave_id(); line < n; line += NW) {
    float v[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int q = lane + 64 * e;
      v[e] = (q < n) ? (kRows ? row_px<kSgn>(Y, n, S, t, q, line) : col_px<kSgn>(Y, n, S, t, line, q))
                     : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int q = lane + 64 * e;
      if (q < n) Y[kRows ? line * S + q : q * S + line] = v[e];
    }
  }
}

// ---------------------------------------------------------------- banded column pass
// Column shear of a working slice Y in global memory (row stride S), for
// slices too large for LDS.  Lanes along a column would touch one cache line
// each, so the pass runs through LDS in bands of kBand columns: `stage`
// fills a band B (rows -1 .. n, stride kBand + 1; rows -1 and n zero, set
// once by the caller) with coalesced row accesses, each wave shears its
// columns in place (lanes along the rows, one table read per column, sample
// positions clamped into the zero rows), and the band goes to Y with
// coalesced row writes.  stage(Bd, c0) writes rows 0 .. n-1 of columns
// c0 .. c0 + kBand - 1 at Bd[r * kBandStride + c], zero beyond column n - 1.
// Starts and ends with a workgroup barrier.
constexpr int kBand = 64;
constexpr int kBandStride = kBand + 1;
__host__ __device__ __forceinline__ size_t band_floats(int n) { return (size_t)(n + 2) * kBandStride; }

template <int kSgn, int EPL, class F>
__device__ __forceinline__ void banded_passes(float* Y, int n, int S, const ViewTab& t, float* B,
                                              F&& stage) {
  static_assert(kBand == 64, "one lane per band column");
  float* Bd = B + kBandStride;                     // row r of the band at Bd[r * kBandStride]
  const int lane = lane_id(), w = wave_id();
  for (int c0 = 0; c0 < n; c0 += kBand) {
    __syncthreads();                               // inputs ready / previous band written back
    stage(Bd, c0);
    __syncthreads();
#pragma unroll 1
    for (int c = w; c < kBand && c0 + c < n; c += NW) {
      const TabEntry te = t.e2[c0 + c];
      float v[EPL];
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int q = lane + 64 * e;
        const int qa = min(max(q + kSgn * te.o, -1), n);
        const int qb = min(max(q + kSgn * (te.o + 1), -1), n);
        v[e] = te.w.x * Bd[qa * kBandStride + c] + te.w.y * Bd[qb * kBandStride + c];
      }
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int q = lane + 64 * e;
        if (q < n) Bd[q * kBandStride + c] = v[e];
      }
    }
    __syncthreads();
    const int q = c0 + lane;
#pragma unroll 4
    for (int r = w; r < n; r += NW)
      if (q < n) Y[r * S + q] = Bd[r * kBandStride + lane];
  }
  __syncthreads();
}

// Column pass over a working slice already in Y.
template <int kSgn, int EPL>
__device__ void banded_col_pass(float* Y, int n, int S, const ViewTab& t, float* B) {
  banded_passes<kSgn, EPL>(Y, n, S, t, B, [&](float* Bd, int c0) {
    for (int p = threadIdx.x; p < n * kBand; p += NT) {
      const int r = p / kBand, c = p - r * kBand;
      Bd[r * kBandStride + c] = c0 + c < n ? Y[r * S + c0 + c] : 0.0f;
    }
  });
}

// Transposed passes 3 and 2 of one view for slices too large for LDS:
// pass 3 transposed, a two-tap gather along each row, is evaluated as each
// band is staged, straight from U and the attenuation factors (wave w takes
// rows w, w + NW, ..., lane L column c0 + L, with the loads of kStageRows
// rows issued before any is used); pass 2 transposed runs in the band; the
// band goes to Y.
constexpr int kStageRows = 4;
template <int EPL>
__device__ void banded_adj_passes(float* Y, const float* __restrict__ u,
                                  const float* __restrict__ a, int n, int S, const ViewTab& t,
                                  float* B) {
  banded_passes<-1, EPL>(Y, n, S, t, B, [&](float* Bd, int c0) {
    const int lane = lane_id(), w = wave_id(), q = c0 + lane;
#pragma unroll 1
    for (int r0 = w; r0 < n; r0 += NW * kStageRows) {
      float ua[kStageRows], ma[kStageRows], ub[kStageRows], mb[kStageRows];
#pragma unroll
      for (int c = 0; c < kStageRows; ++c) {
        const int r = r0 + c * NW;
        const int ia = q - t.e13[r < n ? r : 0].o, ib = ia - 1;
        const bool ok = r < n && q < n;
        const int at = r * n + ia;                 // < n * n: 32-bit offsets
        ua[c] = ok && inside(ia, n) ? u[at] : 0.0f;
        ma[c] = ok && inside(ia, n) ? a[at] : 0.0f;
        ub[c] = ok && inside(ib, n) ? u[at - 1] : 0.0f;
        mb[c] = ok && inside(ib, n) ? a[at - 1] : 0.0f;
      }
#pragma unroll
      for (int c = 0; c < kStageRows; ++c) {
        const int r = r0 + c * NW;
        if (r < n) {
          const float2 wt = t.e13[r].w;
          Bd[r * kBandStride + lane] = wt.x * (ua[c] * ma[c]) + wt.y * (ub[c] * mb[c]);
        }
      }
    }
  });
}

// Passes 1 and 2 of R_l X into Y (and pass 3 when kAllThree; otherwise the
// caller fuses pass 3 with its output).  Ends with Y complete (barrier).
template <bool kAllThree, int EPL>
__device__ __forceinline__ void rotate_into(float* Y, const float* X, int n, int S, int SX, int m,
                                            const ViewTab& t, float* band = nullptr) {
  const QAddr qa = quarter_addr(m, n, SX);
  const int lane = lane_id();
  for (int j = wave_id(); j < n; j += NW)
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int i = lane + 64 * e;
      if (i < n) Y[j * S + i] = pass1_px(X, n, qa, t, i, j);
    }
  if (band) {                                          // Y in global memory
    banded_col_pass<1, EPL>(Y, n, S, t, band);
  } else {
    __syncthreads();
    line_pass<1, false, EPL>(Y, n, S, t);
    __syncthreads();
  }
  if (kAllThree) {
    line_pass<1, true, EPL>(Y, n, S, t);
    __syncthreads();
  }
}

// Bilinear R_l X into Y.  Ends with Y complete (barrier).
template <int EPL>
__device__ __forceinline__ void bil_into(float* Y, const float* X, int n, int S, int SX, int m,
                                         const ViewTab& t) {
  const QAddr qa = quarter_addr(m, n, SX);
  const int lane = lane_id();
  for (int j = wave_id(); j < n; j += NW)
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int i = lane + 64 * e;
      if (i < n) Y[j * S + i] = bil_px(X, n, qa, t, i, j);
    }
  __syncthreads();
}

// ---------------------------------------------------------------- Eq. (1)
// Column suffix scan of a rotated attenuation slice in Y (detector beyond
// j = n-1): kScanSeg threads per column each own a run of rows; run sums in
// FP64 are combined through LDS, then every thread writes its run.
constexpr int kScanSeg = 8;

__device__ void mubar_scan(float* Y, double* seg, int n, int S, double dy) {
  const int per = (n + kScanSeg - 1) / kScanSeg;
  const int sgi = threadIdx.x % kScanSeg;
  const int j0 = sgi * per, j1 = min(n, j0 + per);
  for (int col = threadIdx.x / kScanSeg; col < n; col += NT / kScanSeg) {
    double own = 0.0;
    for (int j = j0; j < j1; ++j) own += (double)Y[j * S + col];
    seg[col * kScanSeg + sgi] = own;
  }
  __syncthreads();
  for (int col = threadIdx.x / kScanSeg; col < n; col += NT / kScanSeg) {
    double run = 0.0;                                   // everything beyond this run
    for (int s2 = sgi + 1; s2 < kScanSeg; ++s2) run += seg[col * kScanSeg + s2];
    for (int j = j1 - 1; j >= j0; --j) {
      const float mu = Y[j * S + col];
      Y[j * S + col] = (float)exp(-dy * (0.5 * (double)mu + run));
      run += (double)mu;
    }
  }
  __syncthreads();
}

// grid (nz, ceil(nviews / VG)): out[(l - out_view0)][k] = mubar of view l.
// kGlobal (slices larger than LDS allows): the source slice is read in place
// from mu and the working slice Y is the workgroup's own slice of `scratch`
// (L2-resident); the scan segments and tables stay in LDS.
template <int EPL, bool kGlobal, bool kBil, int kN>
__global__ __launch_bounds__(NT) void mubar_kernel(const float* __restrict__ mu,
                                                   float* __restrict__ out, int n_arg, int nz,
                                                   int view0, int nviews, int VG, int out_view0,
                                                   Tables tab, double dy, float* scratch) {
  const int n = kN ? kN : n_arg;                   // kN: the slice size fixed at compile time
  extern __shared__ float smem[];
  const int S = slice_stride(n);
  const int k = blockIdx.x;
  const size_t nn = (size_t)n * n;
  const float* X;
  float* Y;
  double* seg;
  int SX;
  if (kGlobal) {
    X = mu + (size_t)k * nn;
    SX = n;
    Y = scratch + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * n * S;
    seg = reinterpret_cast<double*>(smem);
  } else {
    float* Xs = smem;
    Y = Xs + n * S;
    seg = reinterpret_cast<double*>(Y + n * S);         // offset 2 n (n+1) floats: 8-byte aligned
    stage_slice(Xs, mu + (size_t)k * nn, n, S);
    X = Xs;
    SX = S;
  }
  ViewTab t = carve_tab(reinterpret_cast<float*>(seg + kScanSeg * n), n);
  // global working slice: the column pass goes through LDS bands after the tables
  float* band = kGlobal ? reinterpret_cast<float*>(seg + kScanSeg * n) + 8 * n : nullptr;
  if (kGlobal && !kBil)
    for (int p = threadIdx.x; p < band_floats(n); p += NT) band[p] = 0.0f;   // guard rows stay zero
  const int lb0 = blockIdx.y * VG, lb1 = min(nviews, lb0 + VG);
  for (int lb = lb0; lb < lb1; ++lb) {
    const int l = view0 + lb;
    __syncthreads();                                   // X staged / previous view written out
    load_tab(tab, l, n, t);
    __syncthreads();
    if (kBil) bil_into<EPL>(Y, X, n, S, SX, tab.quarter[l], t);
    else rotate_into<true, EPL>(Y, X, n, S, SX, tab.quarter[l], t, band);
    mubar_scan(Y, seg, n, S, dy);
    float* dst = out + ((size_t)(l - out_view0) * nz + k) * nn;
    for (int p = threadIdx.x; p < n * n; p += NT) {
      const int j = p / n, i = p - j * n;
      dst[p] = Y[j * S + i];
    }
  }
}

// ---------------------------------------------------------------- forward
// The forward kernel keeps a single staged slice and evaluates the three
// passes as one fused gather per output pixel: pass 3 needs two pass-2
// values, each needing two pass-1 values, each needing two quarter-turned
// pixels (at most 8 LDS reads and 14 two-tap blends), with every intermediate
// sample outside [0, n) equal to zero exactly as in a pass over the whole
// slice.  One slice in LDS lets two workgroups share a CU.  A wave owns 8 x 8
// pixel tiles and the slice row stride is 8 (mod 16) floats, so the gathers of
// a rotated tile spread over the LDS banks for every angle.
__host__ __device__ __forceinline__ int gather_stride(int n) { return n + ((8 - n % 16) + 16) % 16; }

// Pixel of this lane in iteration r: 8x8 tile (w + NW r) of the slice, with
// tpr = ceil(n / 8) tiles per row and rtpr = 1 / tpr (tile < 2^12 and tpr <= 32,
// so the float quotient rounds to the exact integer division).
__device__ __forceinline__ bool tile_pixel(int n, int tpr, float rtpr, int r, int& i, int& j) {
  const int tile = wave_id() + NW * r;
  const int tj = (int)(((float)tile + 0.5f) * rtpr), ti = tile - tj * tpr;
  i = 8 * ti + (lane_id() & 7);
  j = 8 * tj + (lane_id() >> 3);
  return tj < tpr && i < n && j < n;
}

// (S3 S2 S1 P_m x)(i, j) from the unrotated slice X.
__device__ __forceinline__ float rotated_pixel(const float* X, int n, const QAddr& qa,
                                               const ViewTab& t, int i, int j) {
  float f3 = 0.0f;
  const TabEntry e3 = t.e13[j];
  const int o3 = e3.o;
  const float2 w3 = e3.w;
#pragma unroll
  for (int t3 = 0; t3 < 2; ++t3) {
    const int i2 = i + o3 + t3;
    if (!inside(i2, n)) continue;
    const TabEntry e2 = t.e2[i2];
    const int o2 = e2.o;
    const float2 w2 = e2.w;
    float f2 = 0.0f;
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2) {
      const int j1 = j + o2 + t2;
      if (!inside(j1, n)) continue;
      const TabEntry e1 = t.e13[j1];
      const int o1 = e1.o;
      const float2 w1 = e1.w;
      const int ia = i2 + o1, ib = ia + 1;
      // |ci|, |cj| <= S and indices < n: 24-bit multiplies are exact (full rate)
      const int row = qa.base + __mul24(qa.cj, j1);
      const float a = inside(ia, n) ? X[row + __mul24(qa.ci, ia)] : 0.0f;
      const float b = inside(ib, n) ? X[row + __mul24(qa.ci, ib)] : 0.0f;
      f2 += (t2 == 0 ? w2.x : w2.y) * (w1.x * a + w1.y * b);
    }
    f3 += (t3 == 0 ? w3.x : w3.y) * f2;
  }
  return f3;
}

// grid (nz, ceil(nvb / VG)): W[lb][k] = (R_l x)[k] * mubar_l[k] for the views
// lb of this group; mubar of view lb is at mb + (lb + mb_off) * N.  RM = 8x8
// tiles per wave, visited kCh at a time.
constexpr int kCh = 4;
// kGlobal: the slice is gathered in place from x (L2-resident), no staging.
template <int RM, bool kGlobal, bool kBil>
__global__ __launch_bounds__(NT) void rot_fwd_kernel(const float* __restrict__ x,
                                                     const float* __restrict__ mb, int mb_off,
                                                     float* __restrict__ W, int n, int nz,
                                                     int view0, int nvb, int VG, Tables tab) {
  extern __shared__ float smem[];
  const int k = blockIdx.x;
  const size_t nn = (size_t)n * n, N = nn * nz;
  const int S = kGlobal ? n : gather_stride(n);
  const float* X;
  ViewTab t;
  if (kGlobal) {
    X = x + (size_t)k * nn;
    t = carve_tab(smem, n);
  } else {
    stage_slice(smem, x + (size_t)k * nn, n, S);
    X = smem;
    t = carve_tab(smem + n * S, n);
  }
  const int tpr = (n + 7) >> 3;
  const float rtpr = 1.0f / (float)tpr;
  const int lb0 = blockIdx.y * VG, lb1 = min(nvb, lb0 + VG);
  for (int lb = lb0; lb < lb1; ++lb) {
    const int l = view0 + lb;
    const float* mbs = mb + (size_t)(lb + mb_off) * N + (size_t)k * nn;
    float* dst = W + (size_t)lb * N + (size_t)k * nn;
    // attenuation factors of the next kCh tiles are loaded while the current
    // ones are gathered
    float att[kCh];
#pragma unroll
    for (int c = 0; c < kCh; ++c) {
      int i, j;
      att[c] = tile_pixel(n, tpr, rtpr, c, i, j) ? mbs[j * n + i] : 0.0f;
    }
    __syncthreads();                       // X staged / previous view's readers done
    load_tab(tab, l, n, t);
    __syncthreads();
    const QAddr qa = quarter_addr(tab.quarter[l], n, S);
#pragma unroll 1
    for (int r0 = 0; r0 < RM; r0 += kCh) {
      float nxt[kCh];
#pragma unroll
      for (int c = 0; c < kCh; ++c) {
        int i, j;
        nxt[c] = (r0 + kCh + c < RM && tile_pixel(n, tpr, rtpr, r0 + kCh + c, i, j)) ? mbs[j * n + i] : 0.0f;
      }
#pragma unroll
      for (int c = 0; c < kCh; ++c) {
        int i, j;
        if (r0 + c < RM && tile_pixel(n, tpr, rtpr, r0 + c, i, j))
          dst[j * n + i] =
              (kBil ? bil_px(X, n, qa, t, i, j) : rotated_pixel(X, n, qa, t, i, j)) * att[c];
      }
#pragma unroll
      for (int c = 0; c < kCh; ++c) att[c] = nxt[c];
    }
  }
}

// ---------------------------------------------------------------- forward, line passes
// The 3-pass forward on slices that fit LDS: per view the slice is staged
// quarter-turned (P_m x) into one working buffer and the three shears run as
// in-place line passes, the last one fused with the attenuation weight and
// the store.  Each line's table entry is one broadcast read, and samples
// outside [0, n) fall on zero guard cells (clamped positions) instead of
// branches.  The source slice stays in registers across the workgroup's views;
// a view's attenuation factors are requested before its staging and first two
// passes, which cover their latency.
//
// Guarded buffer: cell (i, j), -2 <= i, j <= n + 1, at Yd[j S + i] with
// Yd = Y + 2 S + 2 and S = guarded_stride(n) (odd, >= n + 4): rows and
// columns -2, -1, n and n + 1 are zero.  A two-tap sample at positions p and
// p + 1 reads cells (c, c + 1) with c = clamp(p, -2, n): both taps are exact
// (zero outside [0, n)) for every p, so one clamp serves both taps and the
// two reads are adjacent.
__host__ __device__ __forceinline__ int guarded_stride(int n) { return (n + 4) | 1; }
__host__ __device__ __forceinline__ int guarded_floats(int n) { return (n + 4) * guarded_stride(n); }
__host__ __device__ __forceinline__ int guarded_origin(int n) { return 2 * guarded_stride(n) + 2; }

__device__ __forceinline__ int clamp_guard(int q, int n) { return min(max(q, -2), n); }

// Cell of pixel (i, j) under P_m (the position quarter_dst gives) in a
// buffer of row stride S: qb + qi i + qj j.
__device__ __forceinline__ void quarter_cell(int m, int n, int S, int& qb, int& qi, int& qj) {
  if (m == 0) { qb = 0; qi = 1; qj = S; }
  else if (m == 1) { qb = n - 1; qi = S; qj = -1; }
  else if (m == 2) { qb = (n - 1) * S + n - 1; qi = -1; qj = -S; }
  else { qb = (n - 1) * S; qi = -S; qj = 1; }
}

// In-place shear of the lines a wave owns (rows: along i with the per-row
// entries, kRows = false: along j with the per-column entries), forward
// (kSgn = +1: out[q] = w.x in[q + o] + w.y in[q + o + 1]) or transposed
// (kSgn = -1: out[q] = w.x in[q - o] + w.y in[q - o - 1]); the lower tap of
// the pair sits at c = clamp(q + o) or clamp(q - o - 1).
template <int kSgn, bool kRows, int EPL, int LPW>
__device__ __forceinline__ void guarded_pass(float* Yd, int n, int S, const TabEntry* lines) {
  const int lane = lane_id(), w = wave_id();
#pragma unroll 2
  for (int r = 0; r < LPW; ++r) {
    const int L = w + NW * r;
    if (L >= n) break;                             // uniform per wave
    const TabEntry te = lines[L];
    float v[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int q = lane + 64 * e;
      const int c = clamp_guard(kSgn > 0 ? q + te.o : q - te.o - 1, n);
      const float lo = kRows ? Yd[L * S + c] : Yd[c * S + L];
      const float hi = kRows ? Yd[L * S + c + 1] : Yd[(c + 1) * S + L];
      v[e] = kSgn > 0 ? te.w.x * lo + te.w.y * hi : te.w.x * hi + te.w.y * lo;
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int q = lane + 64 * e;
      if (q < n) (kRows ? Yd[L * S + q] : Yd[q * S + L]) = v[e];
    }
  }
}

// grid (nz, ceil(nvb / VG)): W[lb][k] = (R_l x)[k] * mubar_l[k] for the views
// of this group.  Thread (wave w, lane) owns pixels i = lane + 64 e,
// j = w + NW r for staging, the last pass and the store.  The tables of all
// the group's views are read into LDS once, at the start: a per-view table
// read would wait for every memory operation in flight (the counter is in
// order), i.e. for the previous view's stores and this view's attenuation
// factors, which instead land while the view's first passes run.  kN != 0
// fixes the slice size at compile time (see with_fixed_n).
template <int EPL, int LPW, int kN>
__global__ __launch_bounds__(NT) void rot_fwd_lines_kernel(const float* __restrict__ x,
                                                           const float* __restrict__ mb, int mb_off,
                                                           float* __restrict__ W, int n_arg, int nz,
                                                           int view0, int nvb, int VG, Tables tab) {
  const int n = kN ? kN : n_arg;                   // kN: the slice size fixed at compile time
  extern __shared__ float smem[];
  const int S = guarded_stride(n);
  float* Yd = smem + guarded_origin(n);
  float* tabs = smem + round4(guarded_floats(n));    // VG views' tables, 8 n floats each
  const int k = blockIdx.x, lane = lane_id(), w = wave_id();
  const size_t nn = (size_t)n * n, N = nn * nz;
  for (int p = threadIdx.x; p < guarded_floats(n); p += NT) smem[p] = 0.0f;
  const int lb0 = blockIdx.y * VG, lb1 = min(nvb, lb0 + VG);
  for (int lb = lb0; lb < lb1; ++lb) load_tab(tab, view0 + lb, n, carve_tab(tabs + (lb - lb0) * 8 * n, n));
  // rows j = w + NW r with j < n (uniform per wave); columns i = lane + 64 e
  float xv[LPW][EPL], mbv[LPW][EPL];
  const int pix = w * n + lane;                   // offset of this thread's (r, e) = (0, 0) pixel
  const float* xs = x + (size_t)k * nn;
#pragma unroll
  for (int r = 0; r < LPW; ++r) {
    if (w + NW * r >= n) break;
#pragma unroll
    for (int e = 0; e < EPL; ++e)
      xv[r][e] = lane + 64 * e < n ? xs[pix + NW * n * r + 64 * e] : 0.0f;
  }
  for (int lb = lb0; lb < lb1; ++lb) {
    const int l = view0 + lb;
    const int m = tab.quarter[l];
    const float* mbs = mb + (size_t)(lb + mb_off) * N + (size_t)k * nn;
#pragma unroll
    for (int r = 0; r < LPW; ++r) {
      if (w + NW * r >= n) break;
#pragma unroll
      for (int e = 0; e < EPL; ++e)
        mbv[r][e] = lane + 64 * e < n ? mbs[pix + NW * n * r + 64 * e] : 0.0f;
    }
    int qb, qi, qj;
    quarter_cell(m, n, S, qb, qi, qj);
    const int sb = qb + qi * lane + qj * w;
    const ViewTab t = carve_tab(tabs + (lb - lb0) * 8 * n, n);
    __syncthreads();                               // guards zeroed / previous view's readers done
#pragma unroll
    for (int r = 0; r < LPW; ++r) {
      if (w + NW * r >= n) break;
#pragma unroll
      for (int e = 0; e < EPL; ++e)
        if (lane + 64 * e < n) Yd[sb + qi * 64 * e + qj * NW * r] = xv[r][e];
    }
    __syncthreads();
    guarded_pass<1, true, EPL, LPW>(Yd, n, S, t.e13);   // pass 1 (along i)
    __syncthreads();
    guarded_pass<1, false, EPL, LPW>(Yd, n, S, t.e2);   // pass 2 (along j)
    __syncthreads();
    float* dst = W + (size_t)lb * N + (size_t)k * nn;
#pragma unroll
    for (int r = 0; r < LPW; ++r) {                 // pass 3 (along i), weight, store
      const int j = w + NW * r;
      if (j >= n) break;
      const TabEntry te = t.e13[j];
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int i = lane + 64 * e;
        const int c = clamp_guard(i + te.o, n);
        const float v = te.w.x * Yd[j * S + c] + te.w.y * Yd[j * S + c + 1];
        if (i < n) dst[pix + NW * n * r + 64 * e] = v * mbv[r][e];
      }
    }
  }
}

// ---------------------------------------------------------------- back, line passes
// grid (nz, G) on slices that fit LDS: partial[g][k] (+)= sum over views
// lb = g, g+G, ... of P_m^T S1^T S2^T S3^T (U[lb][k] * mubar_l[k]).  Per view
// the weighted slice is staged into the zero-guarded buffer, S3^T and S2^T
// run as in-place line passes, and the accumulators (thread (w, lane) owns
// pixels i = lane + 64 e, j = w + NW r) gather S1^T at the quarter-turned
// positions, so that P_m^T S1^T costs no pass of its own.  The next view's U
// and mubar are loaded during the passes.  kN != 0 fixes the slice size at
// compile time (see with_fixed_n).
template <int EPL, int LPW, int kN>
__global__ __launch_bounds__(NT) void rot_back_lines_kernel(const float* __restrict__ U,
                                                            const float* __restrict__ mb, int mb_off,
                                                            float* __restrict__ partial, int n_arg,
                                                            int nz, int view0, int nvb, int G,
                                                            int accumulate, Tables tab) {
  const int n = kN ? kN : n_arg;                   // kN: the slice size fixed at compile time
  extern __shared__ float smem[];
  const int S = guarded_stride(n);
  float* Yd = smem + guarded_origin(n);
  ViewTab t = carve_tab(smem + round4(guarded_floats(n)), n);
  const int k = blockIdx.x, g = blockIdx.y, lane = lane_id(), w = wave_id();
  const size_t nn = (size_t)n * n, N = nn * nz;
  for (int p = threadIdx.x; p < guarded_floats(n); p += NT) smem[p] = 0.0f;
  const int pix = w * n + lane;
  float acc[LPW][EPL], uv[LPW][EPL], mv[LPW][EPL];
#pragma unroll
  for (int r = 0; r < LPW; ++r)
#pragma unroll
    for (int e = 0; e < EPL; ++e) acc[r][e] = 0.0f;
  auto load_view = [&](int lb) {
    const float* src = U + (size_t)lb * N + (size_t)k * nn;
    const float* mbs = mb + (size_t)(lb + mb_off) * N + (size_t)k * nn;
#pragma unroll
    for (int r = 0; r < LPW; ++r) {
      if (w + NW * r >= n) break;
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const bool in = lane + 64 * e < n;
        uv[r][e] = in ? src[pix + NW * n * r + 64 * e] : 0.0f;
        mv[r][e] = in ? mbs[pix + NW * n * r + 64 * e] : 0.0f;
      }
    }
  };
  if (g < nvb) load_view(g);
  for (int lb = g; lb < nvb; lb += G) {
    const int l = view0 + lb;
    const int m = tab.quarter[l];
    __syncthreads();                               // guards zeroed / previous view's readers done
    load_tab(tab, l, n, t);
#pragma unroll
    for (int r = 0; r < LPW; ++r) {                 // Y = U * mubar
      if (w + NW * r >= n) break;
#pragma unroll
      for (int e = 0; e < EPL; ++e)
        if (lane + 64 * e < n) Yd[(w + NW * r) * S + lane + 64 * e] = uv[r][e] * mv[r][e];
    }
    if (lb + G < nvb) load_view(lb + G);
    __syncthreads();
    guarded_pass<-1, true, EPL, LPW>(Yd, n, S, t.e13);    // S3^T (along i)
    __syncthreads();
    guarded_pass<-1, false, EPL, LPW>(Yd, n, S, t.e2);    // S2^T (along j)
    __syncthreads();
    // S1^T (along i) evaluated where the accumulators gather it:
    // x(i, j) += w.x Y[dj][di - o] + w.y Y[dj][di - o - 1] with (di, dj) the
    // position of (i, j) under P_m, an affine map (a0 + ai i + aj j,
    // b0 + bi i + bj j) whose indices are formed per view (hoisted out of the
    // view loop, those of every pixel a lane owns would spill)
    int ln = lane, wv = w;
    asm volatile("" : "+v"(ln), "+v"(wv));
    const int a0 = (m == 1 || m == 2) ? n - 1 : 0, b0 = (m >= 2) ? n - 1 : 0;
    const int ai = m == 0 ? 1 : (m == 2 ? -1 : 0), aj = m == 1 ? -1 : (m == 3 ? 1 : 0);
    const int bi = m == 1 ? 1 : (m == 3 ? -1 : 0), bj = m == 0 ? 1 : (m == 2 ? -1 : 0);
    const int di0 = a0 + ai * ln + aj * wv, dj0 = b0 + bi * ln + bj * wv;
#pragma unroll
    for (int r = 0; r < LPW; ++r) {
      if (w + NW * r >= n) break;
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        if (lane + 64 * e < n) {
          const int di = di0 + ai * 64 * e + aj * NW * r, dj = dj0 + bi * 64 * e + bj * NW * r;
          const TabEntry te = t.e13[dj];
          const int c = clamp_guard(di - te.o - 1, n);
          const float v = te.w.x * Yd[dj * S + c + 1] + te.w.y * Yd[dj * S + c];
          acc[r][e] += v;
        }
      }
    }
  }
  float* dst = partial + (size_t)g * N + (size_t)k * nn;
#pragma unroll
  for (int r = 0; r < LPW; ++r) {
    if (w + NW * r >= n) break;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int p = pix + NW * n * r + 64 * e;
      if (lane + 64 * e < n) dst[p] = accumulate ? dst[p] + acc[r][e] : acc[r][e];
    }
  }
}

// ---------------------------------------------------------------- back
// grid (nz, G): partial[g][k] (+)= sum over views lb = g, g+G, ... of
//   P_m^T S1^T S2^T S3^T (U[lb][k] * mubar_l[k]).
// Output pixel (i, j) accumulates in wave j mod NW, lane i mod 64.
// kGlobal: the working slice Y is the workgroup's own slice of `scratch`;
// with the 3-pass rotation, passes 3 and 2 transposed run band by band
// (banded_adj_passes) and pass 1 transposed gathers from Y.
template <int EPL, int LPW, bool kGlobal, bool kBil>
__global__ __launch_bounds__(NT) void rot_back_kernel(const float* __restrict__ U,
                                                      const float* __restrict__ mb, int mb_off,
                                                      float* __restrict__ partial, int n, int nz,
                                                      int view0, int nvb, int G, int accumulate,
                                                      Tables tab, float* scratch) {
  extern __shared__ float smem[];
  const int S = slice_stride(n);
  const int k = blockIdx.x, g = blockIdx.y, lane = lane_id(), w = wave_id();
  float* Y = kGlobal ? scratch + ((size_t)g * nz + k) * n * S : smem;
  ViewTab t = carve_tab(kGlobal ? smem : Y + round4(n * S), n);
  float* band = kGlobal ? smem + 8 * n : nullptr;   // after the tables (2n entries of 4 floats)
  if (kGlobal)
    for (int p = threadIdx.x; p < band_floats(n); p += NT) band[p] = 0.0f;   // guard rows stay zero
  const size_t nn = (size_t)n * n, N = nn * nz;
  float acc[LPW][EPL];
#pragma unroll
  for (int r = 0; r < LPW; ++r)
#pragma unroll
    for (int e = 0; e < EPL; ++e) acc[r][e] = 0.0f;
  for (int lb = g; lb < nvb; lb += G) {
    const int l = view0 + lb;
    const int m = tab.quarter[l];
    __syncthreads();                                   // previous view's readers done
    load_tab(tab, l, n, t);
    const float* src = U + (size_t)lb * N + (size_t)k * nn;
    const float* mbs = mb + (size_t)(lb + mb_off) * N + (size_t)k * nn;
    if (kGlobal && !kBil) {
      banded_adj_passes<EPL>(Y, src, mbs, n, S, t, band);   // passes 3 and 2 transposed
    } else {
      // stage U * mubar: a thread keeps column i = tid mod n and visits rows
      // j = tid / n + lpi r, with the loads of kStageRows rows issued first
      const int lpi = NT / n, i = threadIdx.x % n, v0 = threadIdx.x / n;
      if (v0 < lpi) {
#pragma unroll 1
        for (int jb = v0; jb < n; jb += kStageRows * lpi) {
          float u[kStageRows], a[kStageRows];
#pragma unroll
          for (int c = 0; c < kStageRows; ++c) {
            const int j = jb + c * lpi;
            u[c] = j < n ? src[j * n + i] : 0.0f;
            a[c] = j < n ? mbs[j * n + i] : 0.0f;
          }
#pragma unroll
          for (int c = 0; c < kStageRows; ++c) {
            const int j = jb + c * lpi;
            if (j < n) Y[j * S + i] = u[c] * a[c];
          }
        }
      }
      __syncthreads();
      if (!kBil) {
        line_pass<-1, true, EPL>(Y, n, S, t);          // pass 3 transpose
        __syncthreads();
        line_pass<-1, false, EPL>(Y, n, S, t);         // pass 2 transpose
        __syncthreads();
      }
    }
    const float2 cs = tab.rot[l];
    const float cc = 0.5f * (float)(n - 1);
    if (kGlobal && kBil) {
      // bilinear, large slices: accumulate in this workgroup's own slice of
      // `partial` (each pixel has one owner lane, so the order of additions
      // is fixed); the 9-candidate gather is too long to unroll over the 64
      // pixels a lane owns
      float* dst = partial + (size_t)g * N + (size_t)k * nn;
      const bool first = lb == g;
#pragma unroll 1
      for (int r = 0; r < LPW; ++r) {
        const int j = w + NW * r;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const int i = lane + 64 * e;
          if (j < n && i < n) {
            int di, dj;
            quarter_dst(m, n, i, j, di, dj);
            const float val = bil_adj_px(Y, n, S, t, cs, cc, di, dj);
            const float prev = (first && !accumulate) ? 0.0f : dst[j * n + i];
            dst[j * n + i] = prev + val;
          }
        }
      }
      continue;
    }
    // pixel indices formed per view: hoisted out of the view loop, those of
    // the 64 pixels a lane owns in large slices would spill the accumulators
    int ln = lane, wv = w;
    if (kGlobal) asm volatile("" : "+v"(ln), "+v"(wv));
#pragma unroll
    for (int r = 0; r < LPW; ++r) {                    // pass 1 transpose, then P_m^T
      const int j = wv + NW * r;
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int i = ln + 64 * e;
        if (j < n && i < n) {
          int di, dj;
          quarter_dst(m, n, i, j, di, dj);             // x(i, j) = h(P_m position)
          acc[r][e] += kBil ? bil_adj_px(Y, n, S, t, cs, cc, di, dj)
                            : row_px<-1>(Y, n, S, t, di, dj);
        }
      }
      // Y in global memory: one line's loads in flight at a time, not all
      // (their addresses and results would spill the accumulators)
      if (kGlobal) __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (kGlobal && kBil) {
    // a workgroup with no view in this batch still owns its slice
    if (g >= nvb && !accumulate) {
      float* dst = partial + (size_t)g * N + (size_t)k * nn;
      for (int p = threadIdx.x; p < n * n; p += NT) dst[p] = 0.0f;
    }
    return;
  }
  float* dst = partial + (size_t)g * N + (size_t)k * nn;
#pragma unroll
  for (int r = 0; r < LPW; ++r) {
    const int j = w + NW * r;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int i = lane + 64 * e;
      if (j < n && i < n) dst[j * n + i] = accumulate ? dst[j * n + i] + acc[r][e] : acc[r][e];
    }
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

// The same sums, four consecutive voxels per thread (N a multiple of 4, x
// 16-byte aligned); each voxel adds its groups in the same order.
__global__ void back_reduce4_kernel(const float4* __restrict__ partial, float4* __restrict__ x,
                                    size_t N4, int G) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N4) return;
  float4 s = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  for (int g = 0; g < G; ++g) {
    const float4 v = partial[(size_t)g * N4 + p];
    s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
  }
  x[p] = s;
}

size_t tab_bytes(int n) { return (size_t)2 * n * sizeof(TabEntry); }
constexpr int kMaxFwdViews = 16;   // views per workgroup of the forward line-pass kernel, at most
// the forward line-pass kernel: the guarded slice and the tables of its VG views
size_t fwd_lines_lds(int n, int VG) { return (size_t)round4(guarded_floats(n)) * 4 + VG * tab_bytes(n); }
size_t slice_bytes(int n) { return (size_t)n * slice_stride(n) * 4; }

hipError_t set_smem(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

size_t rotation_lds_bytes(int n) {
  // mubar kernel with slices in LDS: two slices, the FP64 scan segments, tables
  return 2 * slice_bytes(n) + (size_t)kScanSeg * n * 8 + tab_bytes(n);
}

size_t rotation_scratch_bytes(int n, int nz, int nview) {
  if (n <= kMaxLdsN) return 0;
  const int VG = kRotViewsPerGroup;
  const int groups = std::max((nview + VG - 1) / VG, kBackGroups);
  return (size_t)groups * nz * n * slice_stride(n) * sizeof(float);
}

// Instantiation by slice size: EPL = elements of a line per lane, LPW =
// lines per wave, and whether the working slices live in LDS or in global
// scratch (n > kMaxLdsN).
template <class F>
hipError_t with_shape(int n, F&& f) {
  using std::integral_constant;
  if (n <= 64) return f(integral_constant<int, 1>(), integral_constant<int, 4>(), std::false_type());
  if (n <= 128) return f(integral_constant<int, 2>(), integral_constant<int, 8>(), std::false_type());
  if (n <= kMaxLdsN)
    return f(integral_constant<int, 3>(), integral_constant<int, (kMaxLdsN + NW - 1) / NW>(),
             std::false_type());
  return f(integral_constant<int, (kMaxN + 63) / 64>(), integral_constant<int, (kMaxN + NW - 1) / NW>(),
           std::true_type());
}

// The line-pass kernels with the slice size fixed at compile time for the
// common sizes (every index and offset then folds into constants and
// immediates: about 15% faster at 128), else read at run time (kN = 0).
template <class EC, class F>
hipError_t with_fixed_n(int n, EC, F&& f) {
  using std::integral_constant;
  if constexpr (EC::value == 1) {
    if (n == 64) return f(integral_constant<int, 64>());
  } else if constexpr (EC::value == 2) {
    if (n == 128) return f(integral_constant<int, 128>());
    if (n == 96) return f(integral_constant<int, 96>());
  }
  return f(integral_constant<int, 0>());
}

hipError_t launch_mubar(const Plan& p, float* out, int view0, int nviews, int out_view0,
                        hipStream_t s) {
  const int n = p.g.nx;
  const bool glob = n > kMaxLdsN;
  const size_t sm = glob ? (size_t)kScanSeg * n * 8 + tab_bytes(n) + band_floats(n) * 4
                         : rotation_lds_bytes(n);
  const int VG = kRotViewsPerGroup;
  dim3 grid(p.g.nz, (nviews + VG - 1) / VG);
  return with_shape(n, [&](auto E, auto, auto G) {
    auto go = [&](auto B, auto N) {
      hipError_t e = set_smem((const void*)mubar_kernel<E.value, G.value, B.value, N.value>, sm);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((mubar_kernel<E.value, G.value, B.value, N.value>), grid, dim3(NT), sm, s,
                         p.mu, out, n, p.g.nz, view0, nviews, VG, out_view0, p.tab, p.g.dy,
                         p.rot_scratch);
      return hipGetLastError();
    };
    if (p.bilinear) return go(std::true_type(), std::integral_constant<int, 0>());
    if constexpr (!G.value)
      return with_fixed_n(n, E, [&](auto N) { return go(std::false_type(), N); });
    return go(std::false_type(), std::integral_constant<int, 0>());
  });
}

hipError_t launch_rot_fwd(const Plan& p, const float* x, const float* mb, int mb_off, float* W,
                          int view0, int nvb, hipStream_t s) {
  const int n = p.g.nx;
  const bool glob = n > kMaxLdsN;
  if (!glob && !p.bilinear) {
    const int VG = p.rot_fwd_vg > 0 ? p.rot_fwd_vg : kRotViewsPerGroup;
    const size_t sm = fwd_lines_lds(n, VG);
    dim3 grid(p.g.nz, (nvb + VG - 1) / VG);
    return with_shape(n, [&](auto E, auto L, auto G) {
      if constexpr (G.value) {
        return hipErrorInvalidValue;               // not reached: n <= kMaxLdsN here
      } else {
        auto go = [&](auto N) {
          hipError_t e = set_smem((const void*)rot_fwd_lines_kernel<E.value, L.value, N.value>, sm);
          if (e != hipSuccess) return e;
          hipLaunchKernelGGL((rot_fwd_lines_kernel<E.value, L.value, N.value>), grid, dim3(NT), sm, s,
                             x, mb, mb_off, W, n, p.g.nz, view0, nvb, VG, p.tab);
          return hipGetLastError();
        };
        return with_fixed_n(n, E, go);
      }
    });
  }
  const size_t sm = glob ? tab_bytes(n) : (size_t)n * gather_stride(n) * 4 + tab_bytes(n);
  const int VG = kRotViewsPerGroup;
  dim3 grid(p.g.nz, (nvb + VG - 1) / VG);
  auto go = [&](auto RM, auto G) {
    auto run = [&](auto B) {
      hipError_t e = set_smem((const void*)rot_fwd_kernel<RM.value, G.value, B.value>, sm);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((rot_fwd_kernel<RM.value, G.value, B.value>), grid, dim3(NT), sm, s, x,
                         mb, mb_off, W, n, p.g.nz, view0, nvb, VG, p.tab);
      return hipGetLastError();
    };
    return p.bilinear ? run(std::true_type()) : run(std::false_type());
  };
  // 8x8 tiles per wave: ceil(ceil(n/8)^2 / NW)
  using std::integral_constant;
  if (n <= 64) return go(integral_constant<int, 4>(), std::false_type());
  if (n <= 128) return go(integral_constant<int, 16>(), std::false_type());
  constexpr int tl = (kMaxLdsN + 7) / 8, tg = (kMaxN + 7) / 8;
  if (n <= kMaxLdsN) return go(integral_constant<int, (tl * tl + NW - 1) / NW>(), std::false_type());
  return go(integral_constant<int, (tg * tg + NW - 1) / NW>(), std::true_type());
}

int tune_rot_fwd_views(const spect_geom& g, int nvb) {
  const int n = g.nx;
  if (n > kMaxLdsN || (g.flags & SPECT_ROT_BILINEAR)) return kRotViewsPerGroup;
  int dev = 0, cus = 0, per_cu = 0;
  const size_t sm = fwd_lines_lds(n, kMaxFwdViews);
  hipError_t e = with_shape(n, [&](auto E, auto L, auto G) {
    if constexpr (G.value) {
      return hipErrorInvalidValue;
    } else {
      return with_fixed_n(n, E, [&](auto N) {
        const void* fn = (const void*)rot_fwd_lines_kernel<E.value, L.value, N.value>;
        hipError_t r = set_smem(fn, sm);
        if (r != hipSuccess) return r;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, sm);
      });
    }
  });
  if (e != hipSuccess || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1 || per_cu < 1)
    return kRotViewsPerGroup;
  // time ~ rounds x (views per workgroup + the per-workgroup set-up, about
  // half a view: guard zeroing and the source slice)
  const long long slots = (long long)cus * per_cu;
  int best = kRotViewsPerGroup;
  double best_cost = -1.0;
  for (int vg = 1; vg <= kMaxFwdViews; ++vg) {
    const long long wgs = (long long)g.nz * ((nvb + vg - 1) / vg);
    const double cost = (double)((wgs + slots - 1) / slots) * (vg + 0.5);
    if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = vg; }
  }
  return best;
}

hipError_t launch_rot_back(const Plan& p, const float* U, const float* mb, int mb_off,
                           float* partial, int view0, int nvb, bool accumulate, hipStream_t s) {
  const int n = p.g.nx;
  const bool glob = n > kMaxLdsN;
  // line passes up to 128 (two values per lane; wider lines would spill)
  if (n <= 128 && !p.bilinear) {
    const size_t sm = (size_t)round4(guarded_floats(n)) * 4 + tab_bytes(n);
    return with_shape(n, [&](auto E, auto L, auto G) {
      if constexpr (G.value || E.value > 2) {
        return hipErrorInvalidValue;               // not reached: n <= 128 here
      } else {
        auto go = [&](auto N) {
          hipError_t e = set_smem((const void*)rot_back_lines_kernel<E.value, L.value, N.value>, sm);
          if (e != hipSuccess) return e;
          hipLaunchKernelGGL((rot_back_lines_kernel<E.value, L.value, N.value>),
                             dim3(p.g.nz, kBackGroups), dim3(NT), sm, s, U, mb, mb_off, partial, n,
                             p.g.nz, view0, nvb, kBackGroups, accumulate ? 1 : 0, p.tab);
          return hipGetLastError();
        };
        return with_fixed_n(n, E, go);
      }
    });
  }
  const size_t sm = glob ? tab_bytes(n) + band_floats(n) * 4
                         : (size_t)round4(n * slice_stride(n)) * 4 + tab_bytes(n);
  return with_shape(n, [&](auto E, auto L, auto G) {
    auto go = [&](auto B) {
      hipError_t e = set_smem((const void*)rot_back_kernel<E.value, L.value, G.value, B.value>, sm);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((rot_back_kernel<E.value, L.value, G.value, B.value>),
                         dim3(p.g.nz, kBackGroups), dim3(NT), sm, s, U, mb, mb_off, partial, n,
                         p.g.nz, view0, nvb, kBackGroups, accumulate ? 1 : 0, p.tab, p.rot_scratch);
      return hipGetLastError();
    };
    return p.bilinear ? go(std::true_type()) : go(std::false_type());
  });
}

hipError_t launch_back_reduce(const Plan& p, const float* partial, float* x, hipStream_t s) {
  const size_t N = (size_t)p.g.nx * p.g.ny * p.g.nz;
  if (N % 4 == 0 && (uintptr_t)x % 16 == 0 && (uintptr_t)partial % 16 == 0) {
    const size_t N4 = N / 4;
    hipLaunchKernelGGL(back_reduce4_kernel, dim3((unsigned)((N4 + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(partial), reinterpret_cast<float4*>(x), N4,
                       kBackGroups);
  } else {
    hipLaunchKernelGGL(back_reduce_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s,
                       partial, x, N, kBackGroups);
  }
  return hipGetLastError();
}

}  // namespace spect
