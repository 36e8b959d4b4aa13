// PSF convolution on FP32 matrix cores with 4x4 blocks (v_mfma_f32_4x4x1f32:
// sixteen independent 4x4 rank-1 updates per instruction), the replicate-
// padded convolution of Sec. II-A (Alg. 1) and its zero-padded correlation
// (Alg. 2, interior of the adjoint).
//
// The 16x16x4 Toeplitz form (conv_mfma.hip) executes (16 + pz - 1) / pz of
// the algorithmic work because an M-block is 16 output rows tall and the band
// of a PSF row spans 16 + pz - 1 input rows.  With 4-row blocks the band
// costs (pz + 3) / pz instead (1.08x for pz = 37), at the same FP32 matrix
// rate per instruction cycle.
//
// Mapping.  Lane 4b + q of a wave belongs to block b (of 16) and holds row q
// of the block's A column, column q of its B row, and column q of its 4x4
// result (result row = accumulator register).  Each block owns kZt x kXt
// output tiles of 4 x 4 bins (z x x); for one PSF column a (x tap) and one
// input row, a tile's update is
//   C[m][n] += p[b(m, row)][a] * in[row][x_n -/+ a]
// with b(m, row) the z tap that links output row m to the input row.  For a
// tile whose first output row lies delta rows before the input row, the A
// column depends on delta only, so the steps of one tap run over delta: one
// A value serves every tile of the step, and each input row is read from LDS
// once per tap and kept in registers while the tiles that need it pass (rows
// delta, delta + 4, ..., delta + 4 (kZt - 1)).
//
// A wave's 16 blocks form BZ x BX (z x x) and the workgroup's waves WZ x WX,
// so a workgroup tile is TH = 4 kZt BZ WZ by TW = 4 kXt BX WX bins.  With
// BX >= 8 each half wave holds one row of blocks, 32 distinct columns at one
// z offset, whose B reads fall in 32 distinct banks for any odd RRS.
//
// Operands come from LDS:
//   - the input region is stored transposed (z contiguous, odd column stride
//     RRS chosen on the host against bank conflicts of a half wave), so
//     every row offset is an instruction immediate;
//   - the PSF is stored as one zero-padded column per x tap, laid out so that
//     step delta of lane q reads a fixed immediate offset from a per-tap base.
//
// Forward: a workgroup owns a TH x TW output tile of one view and a chunk of
// depth planes, stages each plane's region (replicate padding by
// clamped source indices) and PSF, and adds the plane into the accumulators;
// each plane's sum is folded into a second set, so FP32 chains stay one plane
// long.  The next plane's region and PSF are loaded into registers while the
// current plane is being computed.  Partial sums per chunk are reduced in a
// fixed order afterwards.  Adjoint: the projection region is staged once with
// zero padding and every depth plane of the chunk is computed from it with its
// own PSF; the edge rows and columns are rewritten by conv_back_edges.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "internal.h"

namespace spect {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kZt = 5;       // z tiles (4 rows each) per block
constexpr int kLook = 2;     // steps of input rows loaded ahead of their MFMAs
constexpr int kMaxRR = 128;  // region rows
constexpr int kPfCols = 3;   // 64-column sweeps of a region row (RC <= 192)
constexpr int kMaxPsf = 4096;  // PSF table elements (px * PL4)

// Waves per workgroup: with 8, every SIMD runs two of them, so one wave's LDS
// waits and barriers overlap the other's MFMAs (the kernels are built with
// 8; with 4, each block would hold 2 x tiles).
constexpr int kM4Waves = 8;
template <int NW>
struct Waves {
  static constexpr int kXt = 8 / NW;             // x tiles (4 columns each) per block
  static constexpr int kThreads = 64 * NW;
  static constexpr int kPfRows = kMaxRR / NW;    // region rows per wave held for the next plane
  static constexpr int kPfPsf = kMaxPsf / kThreads;  // PSF table elements per thread
};

__device__ __forceinline__ int clampi(int q, int lo, int hi) { return q < lo ? lo : (q > hi ? hi : q); }

// Workgroup id -> logical id, so that consecutive logical ids (which share
// input planes) land on the same XCD; workgroups are dealt to the 8 XCDs
// round-robin.
__device__ __forceinline__ int xcd_remap(int wg, int total) {
  const int per = total / 8, rem = total % 8, x = wg % 8, slot = wg / 8;
  return x * per + min(x, rem) + slot;
}

// Depth planes of chunk c: [c ny / nchunk, (c+1) ny / nchunk).
__device__ __forceinline__ void chunk_range(int c, int nchunk, int ny, int& j0, int& j1) {
  j0 = (int)(((long long)c * ny) / nchunk);
  j1 = (int)(((long long)(c + 1) * ny) / nchunk);
}

// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1 (compile-time
// step indices, so that each step's broadcast block is an immediate).
template <class F, int... I>
__device__ __forceinline__ void unroll_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>()), ...);
}
template <int N, class F>
__device__ __forceinline__ void unroll(F&& f) {
  unroll_seq(f, std::make_integer_sequence<int, N>());
}

// All taps of one plane into acc.
//   A: every block uses the same PSF column, so lane 4b + q holds the A row q
//   of step 16 g + b (group g) and each MFMA broadcasts the A operand of the
//   block that holds its step (cbsz = 4, abid = step mod 16): one LDS read
//   per 16 steps.  Step t of tap a reads P[a PL4 + q + ND - 1 - t] forward,
//   P[a PL4 + 3 - q + t] adjoint.
//   B: pb = RT + pb_lane (tap 0, x tile 0), moved by -RRS (forward) or +RRS
//   (adjoint) per tap, x tile j at +4 j RRS, input row r at +r.
// kMirror (PSF rows symmetric in x): tap a also stands for tap px - 1 - a,
// whose input column pb2 = RT + pb2_lane moves the opposite way; the two
// columns are added before the product, and ntap = ha + 1 (the centre tap's
// PSF column is stored halved and meets its own column twice).
template <int ND4, int kXt, bool kBack, bool kMirror>
__device__ __forceinline__ void m4_plane(const float* __restrict__ P, const float* __restrict__ RT,
                                         int pb_lane, int pb2_lane, int PL4, int RRS, int ntap,
                                         floatx4 (&acc)[kZt][kXt]) {
  constexpr int ND = 4 * ND4;                 // steps per tap
  constexpr int NR = 4 * (kZt - 1) + ND;      // input rows per tap
  constexpr int NF = 4 * kZt;                 // rows 0 .. NF-1: first used in steps 0..3
  constexpr int NG = (ND + 15) / 16;          // A groups per tap
  constexpr int NSP = ND >= 16 ? ND - 8 : ND; // steps that carry the next tap's first rows
  const int lane = threadIdx.x & 63, q = lane & 3, blk = lane >> 2;
  int aoff[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int t = min(16 * g + blk, ND - 1);  // slots past the last step repeat it (unused)
    aoff[g] = kBack ? 3 - q + t : q + ND - 1 - t;
  }
  // Rows as loaded (X: the tap's column, Y: the mirror tap's column).  The
  // first rows of consecutive taps alternate between the sets F0 and F1 (the
  // tap loop is unrolled by two, so no copies are needed); rows NF .. NR-1
  // are loaded during their own tap into R.  B, the MFMA operand, is formed at
  // the row's first step, so no load is waited for in the step that issues it.
  float Ag[2][NG];
  float F0x[NF][kXt], F0y[NF][kXt], F1x[NF][kXt], F1y[NF][kXt];
  float Rx[NR][kXt], Ry[NR][kXt], B[NR][kXt];
  const int tstep = kBack ? RRS : -RRS;
  const int xstep = 4 * RRS;
  auto ld = [&](float (&d1)[kXt], float (&d2)[kXt], const float* pb, const float* pb2, int off) {
#pragma unroll
    for (int j = 0; j < kXt; ++j) {
      d1[j] = pb[j * xstep + off];
      if (kMirror) d2[j] = pb2[j * xstep + off];
    }
  };
  auto form = [&](const float (&x)[kXt], const float (&y)[kXt], int r) {
#pragma unroll
    for (int j = 0; j < kXt; ++j) B[r][j] = kMirror ? x[j] + y[j] : x[j];
  };
  // k-th first row in order of first use: row 4 i + u (tile i, step u) for
  // k = u kZt + i; its index is first_k(r) for r < NF
  auto first_row = [](int k) { return 4 * (k % kZt) + k / kZt; };
  auto first_k = [](int r) { return (r % 4) * kZt + r / 4; };
  // one tap: a = the tap, kOdd selects which first-row and A sets are current
  auto tap = [&](auto Odd, int a) {
    constexpr bool kOdd = decltype(Odd)::value;
    auto& Fx = kOdd ? F1x : F0x;
    auto& Fy = kOdd ? F1y : F0y;
    auto& Nx = kOdd ? F0x : F1x;
    auto& Ny = kOdd ? F0y : F1y;
    const float* pb = RT + pb_lane + a * tstep;
    const float* pb2 = RT + pb2_lane - a * tstep;
    const int an = a + 1 < ntap ? a + 1 : a;  // the last tap reloads itself (values unused)
    const float* pan = P + an * PL4;
    const float* pbn = RT + pb_lane + an * tstep;
    const float* pb2n = RT + pb2_lane - an * tstep;
    unroll<ND>([&](auto S) {
      constexpr int s = decltype(S)::value;
      // the row first used kLook steps ahead (rows of later steps are needed
      // by the last tile only)
      constexpr int t = s + kLook;
      if constexpr (t >= 4 && t < ND) ld(Rx[t + 4 * (kZt - 1)], Ry[t + 4 * (kZt - 1)], pb, pb2,
                                         t + 4 * (kZt - 1));
      // the next tap's first rows, spread over the first NSP steps
      if constexpr (s < NSP) {
#pragma unroll
        for (int k = s * NF / NSP; k < (s + 1) * NF / NSP; ++k) ld(Nx[k], Ny[k], pbn, pb2n, first_row(k));
      }
      if constexpr (s == ND / 2) {
#pragma unroll
        for (int g = 0; g < NG; ++g) Ag[kOdd ? 0 : 1][g] = pan[aoff[g]];
      }
      // operands of the rows first used at this step
      if constexpr (s < 4) {
#pragma unroll
        for (int i = 0; i < kZt; ++i) form(Fx[first_k(s + 4 * i)], Fy[first_k(s + 4 * i)], s + 4 * i);
      } else {
        form(Rx[s + 4 * (kZt - 1)], Ry[s + 4 * (kZt - 1)], s + 4 * (kZt - 1));
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < kZt; ++i)
#pragma unroll
        for (int j = 0; j < kXt; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_4x4x1f32(Ag[kOdd ? 1 : 0][s / 16], B[s + 4 * i][j],
                                                         acc[i][j], 4, s % 16, 0);
      __builtin_amdgcn_sched_barrier(0);
    });
  };
#pragma unroll
  for (int g = 0; g < NG; ++g) Ag[0][g] = P[aoff[g]];
#pragma unroll
  for (int k = 0; k < NF; ++k) ld(F0x[k], F0y[k], RT + pb_lane, RT + pb2_lane, first_row(k));
  int a = 0;
  for (; a + 1 < ntap; a += 2) {
    tap(std::false_type(), a);
    tap(std::true_type(), a + 1);
  }
  if (a < ntap) tap(std::false_type(), a);
}

// PSF table of one plane: P[a PL4 + t] = p[t - Z][a] (zero outside the taps),
// Z = ND - pz forward (column reversed by the read order), 3 adjoint.
// kMirror: columns a = 0 .. ha only, the centre column halved (exact).
template <int NW, bool kMirror>
struct PsfTable {
  static constexpr int kPfPsf = Waves<NW>::kPfPsf;
  float v[kPfPsf];
  __device__ __forceinline__ void load(const M4Shape& s, const float* __restrict__ pj, int Z) {
    const int ncol = kMirror ? s.ha + 1 : s.px;
#pragma unroll
    for (int u = 0; u < kPfPsf; ++u) {
      const int e = threadIdx.x + Waves<NW>::kThreads * u;
      float x = 0.0f;
      if (e < ncol * s.PL4) {
        const int a = e / s.PL4, b = e - a * s.PL4 - Z;
        if (b >= 0 && b < s.pz) x = pj[b * s.px + a];
        if (kMirror && a == s.ha) x *= 0.5f;
      }
      v[u] = x;
    }
  }
  __device__ __forceinline__ void store(const M4Shape& s, float* P) const {
    const int ncol = kMirror ? s.ha + 1 : s.px;
#pragma unroll
    for (int u = 0; u < kPfPsf; ++u) {
      const int e = threadIdx.x + Waves<NW>::kThreads * u;
      if (e < ncol * s.PL4) P[e] = v[u];
    }
  }
};

// Forward input region of one plane, rows w + NW r (input k = k0 - hb + row,
// clamped) and columns lane + 64 u (input i = i0 - ha + column, clamped).
template <int NW>
struct FwdRegion {
  static constexpr int kPfRows = Waves<NW>::kPfRows;
  float r[kPfRows][kPfCols];
  __device__ __forceinline__ void load(const M4Shape& s, const float* __restrict__ Wj, int k0,
                                       int i0, size_t row_stride, int w, int lane) {
#pragma unroll
    for (int rr = 0; rr < kPfRows; ++rr) {
      const int row = w + NW * rr;
      const float* src = Wj + (size_t)clampi(k0 - s.hb + row, 0, s.nz - 1) * row_stride;
#pragma unroll
      for (int u = 0; u < kPfCols; ++u) {
        const int col = lane + 64 * u;
        r[rr][u] = (row < s.RR && col < s.RC) ? src[clampi(i0 - s.ha + col, 0, s.nx - 1)] : 0.0f;
      }
    }
  }
  __device__ __forceinline__ void store(const M4Shape& s, float* RT, int w, int lane) const {
#pragma unroll
    for (int rr = 0; rr < kPfRows; ++rr) {
      const int row = w + NW * rr;
#pragma unroll
      for (int u = 0; u < kPfCols; ++u) {
        const int col = lane + 64 * u;
        if (row < s.RR && col < s.RC) RT[col * s.RRS + row] = r[rr][u];
      }
    }
  }
};

// ---------------------------------------------------------------- forward
template <int ND4, int NW, bool kMirror>
__global__ __launch_bounds__(64 * NW, 1) void conv_fwd_m4(const float* __restrict__ W,
                                                      const float* __restrict__ psf,
                                                      float* __restrict__ partial, M4Shape s,
                                                      int view0, int nvb) {
  extern __shared__ float sm[];
  float* RT = sm;                                  // RC x RRS: input region, z contiguous
  float* P = sm + s.RC * s.RRS;                    // px x PL4: PSF columns
  const int ntile = s.tiles_k * s.tiles_i;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = logical % ntile, rest = logical / ntile;
  const int tk = tile / s.tiles_i, ti = tile - tk * s.tiles_i;
  const int c = rest % s.nchunk, lb = rest / s.nchunk, l = view0 + lb;
  const int k0 = tk * s.TH, i0 = ti * s.TW;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane & 3, blk = lane >> 2;
  const int bz = blk / s.BX, bx = blk - bz * s.BX, wz = w / s.WX, wx = w - wz * s.WX;
  constexpr int kXt = Waves<NW>::kXt;
  // block origin in the tile
  const int zb = 4 * kZt * (s.BZ * wz + bz), xo = 4 * kXt * (s.BX * wx + bx);
  int j0, j1;
  chunk_range(c, s.nchunk, s.ny, j0, j1);
  const size_t row_stride = (size_t)s.ny * s.nx;
  const float* Wl = W + (size_t)lb * s.nz * row_stride;
  const float* psf_l = psf + (size_t)l * s.ny * s.pz * s.px;
  constexpr int ND = 4 * ND4;
  const int Z = ND - s.pz;
  // step t of tap a: A = P[a PL4 + q + ND - 1 - t] = p[2 hb - t + q][a];
  // B (x tile j, row r) = RT[(xo + 4 j + q + 2 ha - a) RRS + zb + r]
  const int pb_lane = (xo + q + 2 * s.ha) * s.RRS + zb;
  const int pb2_lane = (xo + q) * s.RRS + zb;            // mirror tap px - 1 - a
  const int ntap = kMirror ? s.ha + 1 : s.px;

  floatx4 tot[kZt][kXt];
#pragma unroll
  for (int i = 0; i < kZt; ++i)
#pragma unroll
    for (int j = 0; j < kXt; ++j) tot[i][j] = {0.f, 0.f, 0.f, 0.f};
  FwdRegion<NW> reg;
  PsfTable<NW, kMirror> tab;
  if (j0 < j1) {
    reg.load(s, Wl + (size_t)j0 * s.nx, k0, i0, row_stride, w, lane);
    tab.load(s, psf_l + (size_t)j0 * s.pz * s.px, Z);
  }
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                               // previous plane consumed
    reg.store(s, RT, w, lane);
    tab.store(s, P);
    __syncthreads();
    if (j + 1 < j1) {
      reg.load(s, Wl + (size_t)(j + 1) * s.nx, k0, i0, row_stride, w, lane);
      tab.load(s, psf_l + (size_t)(j + 1) * s.pz * s.px, Z);
    }
    floatx4 acc[kZt][kXt];
#pragma unroll
    for (int i = 0; i < kZt; ++i)
#pragma unroll
      for (int jj = 0; jj < kXt; ++jj) acc[i][jj] = {0.f, 0.f, 0.f, 0.f};
    m4_plane<ND4, kXt, false, kMirror>(P, RT, pb_lane, pb2_lane, s.PL4, s.RRS, ntap, acc);
#pragma unroll
    for (int i = 0; i < kZt; ++i)
#pragma unroll
      for (int jj = 0; jj < kXt; ++jj) tot[i][jj] += acc[i][jj];
  }
  // result row v of tile (i, jj): k = k0 + zb + 4 i + v, x = i0 + xo + 4 jj + q
  float* out = partial + ((size_t)c * nvb + lb) * s.nz * s.nx;
#pragma unroll
  for (int i = 0; i < kZt; ++i)
#pragma unroll
    for (int jj = 0; jj < kXt; ++jj) {
      const int x = i0 + xo + 4 * jj + q;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = k0 + zb + 4 * i + v;
        if (k < s.nz && x < s.nx) out[(size_t)k * s.nx + x] = tot[i][jj][v];
      }
    }
}

// ---------------------------------------------------------------- adjoint
// u[k][i] = sum_{a,b} p[b][a] v[k + b - hb][i + a - ha] (v zero outside) for
// every bin of the tile and every plane of the chunk.
template <int ND4, int NW, bool kMirror>
__global__ __launch_bounds__(64 * NW, 1) void conv_back_m4(const float* __restrict__ v,
                                                       const float* __restrict__ psf,
                                                       float* __restrict__ U, M4Shape s,
                                                       int view0, int nvb) {
  extern __shared__ float sm[];
  float* RT = sm;                                  // RC x RRS: projection region, z contiguous
  float* P = sm + s.RC * s.RRS;                    // px x PL4: PSF columns
  const int ntile = s.tiles_k * s.tiles_i;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = logical % ntile, rest = logical / ntile;
  const int tk = tile / s.tiles_i, ti = tile - tk * s.tiles_i;
  const int c = rest % s.nchunk_back, lb = rest / s.nchunk_back, l = view0 + lb;
  const int k0 = tk * s.TH, i0 = ti * s.TW;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane & 3, blk = lane >> 2;
  const int bz = blk / s.BX, bx = blk - bz * s.BX, wz = w / s.WX, wx = w - wz * s.WX;
  constexpr int kXt = Waves<NW>::kXt;
  const int zb = 4 * kZt * (s.BZ * wz + bz), xo = 4 * kXt * (s.BX * wx + bx);
  int j0, j1;
  chunk_range(c, s.nchunk_back, s.ny, j0, j1);
  const float* vl = v + (size_t)l * s.nz * s.nx;
  const float* psf_l = psf + (size_t)l * s.ny * s.pz * s.px;

  // region row r <-> input k = k0 - hb + r, column cc <-> input i = i0 - ha + cc
  for (int e = threadIdx.x; e < s.RR * s.RC; e += Waves<NW>::kThreads) {
    const int r = e / s.RC, cc = e - r * s.RC;
    const int kk = k0 - s.hb + r, ii = i0 - s.ha + cc;
    RT[cc * s.RRS + r] =
        (kk >= 0 && kk < s.nz && ii >= 0 && ii < s.nx) ? vl[(size_t)kk * s.nx + ii] : 0.0f;
  }
  // step t of tap a: A = P[a PL4 + 3 - q + t] = p[t - q][a];
  // B (x tile j, row r) = RT[(xo + 4 j + q + a) RRS + zb + r]
  const int pb_lane = (xo + q) * s.RRS + zb;
  const int pb2_lane = (xo + q + 2 * s.ha) * s.RRS + zb;  // mirror tap px - 1 - a
  const int ntap = kMirror ? s.ha + 1 : s.px;
  PsfTable<NW, kMirror> tab;
  if (j0 < j1) tab.load(s, psf_l + (size_t)j0 * s.pz * s.px, 3);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                               // region staged / previous plane consumed
    tab.store(s, P);
    __syncthreads();
    if (j + 1 < j1) tab.load(s, psf_l + (size_t)(j + 1) * s.pz * s.px, 3);
    floatx4 acc[kZt][kXt];
#pragma unroll
    for (int i = 0; i < kZt; ++i)
#pragma unroll
      for (int jj = 0; jj < kXt; ++jj) acc[i][jj] = {0.f, 0.f, 0.f, 0.f};
    m4_plane<ND4, kXt, true, kMirror>(P, RT, pb_lane, pb2_lane, s.PL4, s.RRS, ntap, acc);
    float* out = U + (size_t)lb * s.nz * s.ny * s.nx + (size_t)j * s.nx;
#pragma unroll
    for (int i = 0; i < kZt; ++i)
#pragma unroll
      for (int jj = 0; jj < kXt; ++jj) {
        const int x = i0 + xo + 4 * jj + q;
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
          const int k = k0 + zb + 4 * i + vv;
          if (k < s.nz && x < s.nx) out[(size_t)k * s.ny * s.nx + x] = acc[i][jj][vv];
        }
      }
  }
}

// ---------------------------------------------------------------- PSF symmetry
// flag = 1, then 0 if any PSF row differs from its mirror image in x
// (exact comparison; a NaN counts as a difference).
__global__ void psf_mirror_flag_init(int* flag) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 1;
}

__global__ void psf_mirror_check(const float* __restrict__ psf, long long pairs, int px, int ha,
                                 int* flag) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < pairs; e += stride) {
    const long long r = e / ha;
    const int a = (int)(e - r * ha);
    const float* row = psf + r * px;
    if (!(row[a] == row[px - 1 - a])) *flag = 0;
  }
}

#define SPECT_M4_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

size_t m4_lds_bytes(const M4Shape& s) {
  return ((size_t)s.RC * s.RRS + (size_t)s.px * s.PL4) * sizeof(float);
}

template <int ND4, int NW, bool kMirror>
hipError_t launch_m4_nw(const M4Shape& s, bool back, const float* in, const float* psf, float* out,
                        int view0, int nvb, hipStream_t st) {
  const size_t sm = m4_lds_bytes(s);
  const void* fn = back ? (const void*)conv_back_m4<ND4, NW, kMirror>
                        : (const void*)conv_fwd_m4<ND4, NW, kMirror>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  dim3 grid(s.tiles_k * s.tiles_i * (back ? s.nchunk_back : s.nchunk) * nvb);
  dim3 block(Waves<NW>::kThreads);
  if (back)
    hipLaunchKernelGGL((conv_back_m4<ND4, NW, kMirror>), grid, block, sm, st, in, psf, out, s, view0,
                       nvb);
  else
    hipLaunchKernelGGL((conv_fwd_m4<ND4, NW, kMirror>), grid, block, sm, st, in, psf, out, s, view0,
                       nvb);
  return hipGetLastError();
}

template <int ND4>
hipError_t launch_m4(const M4Shape& s, bool back, const float* in, const float* psf, float* out,
                     int view0, int nvb, hipStream_t st) {
  return s.mirror ? launch_m4_nw<ND4, kM4Waves, true>(s, back, in, psf, out, view0, nvb, st)
                  : launch_m4_nw<ND4, kM4Waves, false>(s, back, in, psf, out, view0, nvb, st);
}

// Workgroups per CU (the same for the paired-tap form: same LDS, fewer registers).
template <int ND4>
int m4_wgs_per_cu(const M4Shape& s, bool back) {
  int nb = 0;
  const void* fn = back ? (const void*)conv_back_m4<ND4, kM4Waves, false>
                        : (const void*)conv_fwd_m4<ND4, kM4Waves, false>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, Waves<kM4Waves>::kThreads,
                                                   m4_lds_bytes(s)) != hipSuccess)
    nb = 0;
  return nb < 1 ? 1 : nb;
}

// Largest number of lanes of one half wave (32 lanes) that share an LDS bank
// for the B reads of a column stride rrs (32 banks of 4 bytes).
int m4_bank_conflicts(int rrs, int BX, int xt) {
  int worst = 0;
  for (int h = 0; h < 2; ++h) {
    int count[32] = {0};
    for (int lane = 32 * h; lane < 32 * h + 32; ++lane) {
      const int blk = lane >> 2, q = lane & 3, bz = blk / BX, bx = blk % BX;
      const long long addr = (long long)(4 * xt * bx + q) * rrs + 4 * kZt * bz;
      const int bank = (int)(addr % 32);
      if (++count[bank] > worst) worst = count[bank];
    }
  }
  return worst;
}

// Depth chunks per (tile, view): minimise rounds * planes per workgroup.
int m4_pick_chunks(int ny, long long tiles_views, long long slots) {
  int best = 1;
  long long best_cost = -1;
  for (int n = 1; n <= kMaxChunks && n <= ny; ++n) {
    const long long rounds = (tiles_views * n + slots - 1) / slots;
    const long long cost = rounds * ((ny + n - 1) / n);
    if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = n; }
  }
  return best;
}

}  // namespace

M4Shape make_m4_shape(const spect_geom& g) {
  M4Shape best{};
  best.ok = false;
  double best_cost = 0.0;
  const int ND4 = (g.pz + 3 + 3) / 4;
  constexpr int kXt = Waves<kM4Waves>::kXt;
  for (int BX = 1; BX <= 16; BX *= 2)
    for (int WX = 1; WX <= kM4Waves; WX *= 2) {
      M4Shape s{};
      s.nx = g.nx; s.ny = g.ny; s.nz = g.nz; s.px = g.px; s.pz = g.pz;
      s.ha = (g.px - 1) / 2; s.hb = (g.pz - 1) / 2;
      s.ND4 = ND4;
      s.mirror = false;
      s.BX = BX;
      s.BZ = 16 / BX;
      s.WX = WX;
      s.WZ = kM4Waves / WX;
      s.TH = 4 * kZt * s.BZ * s.WZ;
      s.TW = 4 * kXt * BX * WX;
      s.tiles_k = (g.nz + s.TH - 1) / s.TH;
      s.tiles_i = (g.nx + s.TW - 1) / s.TW;
      s.RR = s.TH - 4 + 4 * ND4;
      s.RC = s.TW + g.px - 1;
      s.PL4 = 4 * ND4 + 3;
      int rrs = s.RR | 1, best_rrs = rrs, best_conf = 1 << 30;
      for (; rrs < s.RR + 64; rrs += 2) {
        const int cf = m4_bank_conflicts(rrs, BX, kXt);
        if (cf < best_conf) { best_conf = cf; best_rrs = rrs; }
        if (cf <= 1) break;
      }
      s.RRS = best_rrs;
      s.nchunk = 1;
      s.nchunk_back = 1;
      s.ok = ND4 >= 1 && ND4 <= 16 && s.RR <= kMaxRR && s.RC <= 64 * kPfCols &&
             g.px * s.PL4 <= kMaxPsf && m4_lds_bytes(s) <= kLdsBytes;
      if (!s.ok) continue;
      // padded output area; an n-way conflict on the B reads costs about
      // (n - 1) / 8 more (they are half the LDS reads, LDS about half busy)
      const double cost = (double)s.tiles_k * s.TH * s.tiles_i * s.TW * (1.0 + 0.125 * (best_conf - 1));
      if (!best.ok || cost < best_cost) { best = s; best_cost = cost; }
    }
  return best;
}

// Relative issue cost of the two FP32 tilings for a plane and a tap: padded
// output area times the products issued per output bin (the K rows of a
// 16-row band, or the steps of a 4-row one), the 4x4 blocks at the 0.92
// relative instruction rate measured for them against 16x16x4.
bool m4_preferred(const M4Shape& s, const ConvShape& cs) {
  if (!s.ok) return false;
  const double old_cost = (double)cs.tiles_k * 16 * cs.WK * cs.tiles_i * 32 * cs.WI * 4 * cs.KS;
  const double new_cost = (double)s.tiles_k * s.TH * s.tiles_i * s.TW * 4 * s.ND4 / 0.92;
  return new_cost < old_cost;
}

void tune_m4_chunks(M4Shape& s, int views) {
  int dev = 0, cus = 0;
  if (!s.ok || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    return;
  int fw = 1, bw = 1;
  switch (s.ND4) {
#define CASE(K) case K: fw = m4_wgs_per_cu<K>(s, false); bw = m4_wgs_per_cu<K>(s, true); break;
    SPECT_M4_CASES(CASE)
#undef CASE
    default: return;
  }
  const long long tv = (long long)s.tiles_k * s.tiles_i * views;
  s.nchunk = m4_pick_chunks(s.ny, tv, (long long)cus * fw);
  s.nchunk_back = m4_pick_chunks(s.ny, tv, (long long)cus * bw);
}

hipError_t detect_m4_mirror(Plan& p, int* d_flag, hipStream_t st) {
  p.m4.mirror = false;
  const long long pairs = (long long)p.g.nview * p.g.ny * p.g.pz * p.m4.ha;
  hipLaunchKernelGGL(psf_mirror_flag_init, dim3(1), dim3(64), 0, st, d_flag);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && pairs > 0) {
    const long long blocks = std::min<long long>((pairs + 255) / 256, 4096);
    hipLaunchKernelGGL(psf_mirror_check, dim3((unsigned)blocks), dim3(256), 0, st, p.psf, pairs,
                       p.g.px, p.m4.ha, d_flag);
    e = hipGetLastError();
  }
  int h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d_flag, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) p.m4.mirror = h == 1;
  return e;
}

hipError_t launch_conv_m4(const Plan& p, bool back, const float* in, float* out, int view0,
                          int nvb, hipStream_t st) {
  switch (p.m4.ND4) {
#define CASE(K) case K: return launch_m4<K>(p.m4, back, in, p.psf, out, view0, nvb, st);
    SPECT_M4_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spect
