// PSF convolution with separable (rank-1) PSFs, p[b][a] = fz[b] fx[a]: the
// replicate-padded convolution of Sec. II-A (Alg. 1) and its exact adjoint
// (Alg. 2) as two 1-D passes per depth plane, 2 (px + pz) FLOP per voxel
// instead of 2 px pz.  The paper's PSFs are fits of 2-D Gaussians per
// distance; an axis-aligned Gaussian is exactly separable.
//
// Clamping acts on each axis on its own, so with c = conv_x(conv_z(w))
//   conv_z: t[k][x] = sum_b fz[b] w[clamp(k + hb - b)][x]
//   conv_x: c[k][i] = sum_a fx[a] t[k][clamp(i + ha - a)]
// is the 2-D convolution of the outer-product PSF.  The adjoint is
// conv_z^T conv_x^T, each the zero-padded correlation plus the fold of
// replicate padding onto the edge: for n > 1
//   g[0]     = sum_i y[i] Fsuf(h + i),      Fsuf(m) = sum_{a >= m} f[a]
//   g[n - 1] = sum_i y[i] Fpre(i + h - n + 1), Fpre(m) = sum_{a <= m} f[a]
// (only the h + 1 samples nearest the edge contribute) and g[0] = y[0] sum f
// for n = 1.
//
// Both passes use one register-blocked 1-D kernel: a thread computes eight
// consecutive outputs out[d] = sum_b g[b] src(r0 + d - b) with the taps in
// groups of four, reading one new source sample per tap (the eight-sample
// window slides down the source), so every LDS read feeds eight FMAs.  Taps
// are zero-padded to a multiple of four; the adjoint uses the reversed taps.
//
// Work split: a workgroup (512 threads) owns a strip of ZS output rows (z) of
// one view and a chunk of depth planes.  Forward: per plane, stage the input
// rows the strip needs (clamped; the next plane's rows are loaded into
// registers meanwhile), run the z pass on the real columns and copy the edge
// columns into the halo, then the x pass, accumulating the depth sum in
// registers; partial sums per chunk are reduced in a fixed order afterwards.
// Adjoint: the projection rows the strip needs are staged once (zero
// outside); per plane the x pass (and its edge fold) fills an intermediate
// strip on the rows inside the volume (the others stay zero), and the z pass
// (and its edge fold) writes the plane's output rows.
#include "internal.h"

namespace spect {
namespace {

constexpr int kSepThreads = 512;
constexpr int kSepOcts = 4;         // output octets per thread held across planes (forward)

__device__ __forceinline__ int clampi(int q, int lo, int hi) { return q < lo ? lo : (q > hi ? hi : q); }

// out[d] += sum_{b < nb4} g[b] * src[(r0 + d - b) * st], d = 0..D-1; g is in
// LDS, 16-byte aligned, zero from the real tap count up to nb4 (a multiple of
// 4).  The window of D source samples slides down by four per tap group, so
// each group reads four new samples for 4 D FMAs.  Reads rows r0 - nb4 ..
// r0 + D - 1 of src.
template <int D>
__device__ __forceinline__ void convD(const float* __restrict__ src, int st, int r0,
                                      const float* __restrict__ g, int nb4, float (&out)[D]) {
  const float* s = src + r0 * st;
  float w[D];
#pragma unroll
  for (int d = 0; d < D; ++d) w[d] = s[d * st];
  // the next group's samples and taps are read while this group's FMAs run
  float nn[4];
  float4 tn = *reinterpret_cast<const float4*>(g);
#pragma unroll
  for (int m = 0; m < 4; ++m) nn[m] = s[-(m + 1) * st];
  for (int b = 0; b < nb4; b += 4) {
    const float4 t = tn;
    float n[4];                                   // rows r0 - b - 1 .. r0 - b - 4
#pragma unroll
    for (int m = 0; m < 4; ++m) n[m] = nn[m];
    if (b + 4 < nb4) {                            // uniform: the last group loads nothing
      const float* sb = s - (b + 4) * st;
      tn = *reinterpret_cast<const float4*>(g + b + 4);
#pragma unroll
      for (int m = 0; m < 4; ++m) nn[m] = sb[-(m + 1) * st];
    }
    const float tv[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)                // tap b + tt reads row r0 - b - tt + d
#pragma unroll
      for (int d = 0; d < D; ++d) out[d] = fmaf(tv[tt], d >= tt ? w[d - tt] : n[tt - d - 1], out[d]);
#pragma unroll
    for (int d = D - 1; d >= 4; --d) w[d] = w[d - 4];
#pragma unroll
    for (int m = 0; m < 4; ++m) w[m] = n[3 - m];
  }
}

constexpr int kOct = 8;             // outputs per thread per pass

__device__ __forceinline__ void strip_range(const SepShape& s, int strip, int& k0, int& k1) {
  k0 = strip * s.ZS;
  k1 = min(k0 + s.ZS, s.nz);
}

// Per-plane taps in LDS: forward fz, fx (zero-padded); adjoint reversed
// fz, fx and the prefix / suffix sums of fz and fx for the edge folds.
struct SepTaps {
  float* gz;   // NBz
  float* gx;   // NBx
  float* szf;  // pz + 1: suffix sums of fz (szf[m] = sum_{b >= m} fz[b], szf[pz] = 0)
  float* szp;  // pz: prefix sums of fz
  float* sxf;  // px + 1
  float* sxp;  // px
};

__device__ __forceinline__ SepTaps carve_taps(float* at, const SepShape& s) {
  SepTaps t;
  t.gz = at;
  t.gx = t.gz + s.NBz;
  t.szf = t.gx + s.NBx;
  t.szp = t.szf + s.pz + 1;
  t.sxf = t.szp + s.pz;
  t.sxp = t.sxf + s.px + 1;
  return t;
}

__host__ __device__ inline int sep_taps_floats(const SepShape& s) {
  return s.NBz + s.NBx + 2 * (s.pz + 1) + 2 * (s.px + 1);
}

// pj: fz[0..pz) then fx[0..px) of one plane.
__device__ __forceinline__ void load_taps(const SepShape& s, const float* __restrict__ pj,
                                          const SepTaps& t, bool back) {
  for (int e = threadIdx.x; e < s.NBz; e += kSepThreads)
    t.gz[e] = e < s.pz ? pj[back ? s.pz - 1 - e : e] : 0.0f;
  for (int e = threadIdx.x; e < s.NBx; e += kSepThreads)
    t.gx[e] = e < s.px ? pj[s.pz + (back ? s.px - 1 - e : e)] : 0.0f;
  if (back) {
    // four threads run the four sequential sums (px, pz <= a few dozen)
    if (threadIdx.x == 0) {
      float a = 0.0f;
      t.szf[s.pz] = 0.0f;
      for (int b = s.pz - 1; b >= 0; --b) { a += pj[b]; t.szf[b] = a; }
    } else if (threadIdx.x == 64) {
      float a = 0.0f;
      for (int b = 0; b < s.pz; ++b) { a += pj[b]; t.szp[b] = a; }
    } else if (threadIdx.x == 128) {
      float a = 0.0f;
      t.sxf[s.px] = 0.0f;
      for (int b = s.px - 1; b >= 0; --b) { a += pj[s.pz + b]; t.sxf[b] = a; }
    } else if (threadIdx.x == 192) {
      float a = 0.0f;
      for (int b = 0; b < s.px; ++b) { a += pj[s.pz + b]; t.sxp[b] = a; }
    }
  }
}

// ---------------------------------------------------------------- forward
// Input rows of one plane for the z pass, prefetched into registers while
// the previous plane is computed: rows w + 8 r (w = wave of the workgroup)
// and columns lane + 64 u.
constexpr int kPfRows = 16;   // staged rows per wave (WR <= 8 * 16)
constexpr int kPfCols = 4;    // 64-column sweeps (nx <= 256)
struct SepRows {
  float v[kPfRows][kPfCols];
  __device__ __forceinline__ void load(const SepShape& s, const float* __restrict__ Wj,
                                       int rbase, int WR, size_t row_stride) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int rr = 0; rr < kPfRows; ++rr) {
      const int r = w + (kSepThreads / 64) * rr;
      const float* src = Wj + (size_t)clampi(rbase + r, 0, s.nz - 1) * row_stride;
#pragma unroll
      for (int u = 0; u < kPfCols; ++u) {
        const int x = lane + 64 * u;
        v[rr][u] = (r < WR && x < s.nx) ? src[x] : 0.0f;
      }
    }
  }
  __device__ __forceinline__ void store(const SepShape& s, float* Ws, int WR) const {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int rr = 0; rr < kPfRows; ++rr) {
      const int r = w + (kSepThreads / 64) * rr;
#pragma unroll
      for (int u = 0; u < kPfCols; ++u) {
        const int x = lane + 64 * u;
        if (r < WR && x < s.nx) Ws[r * s.nx + x] = v[rr][u];
      }
    }
  }
};

// grid: nstrip * nchunk * nvb workgroups of 512 threads.
// LDS: Ws (ZS + NBz) x nx input rows (clamped), T ZS x TS z-pass output on
// the padded column range (halo columns copied from the edge columns), taps.
__global__ __launch_bounds__(kSepThreads) void conv_fwd_sep(const float* __restrict__ W,
                                                            const float* __restrict__ psf,
                                                            float* __restrict__ partial,
                                                            SepShape s, int view0, int nvb) {
  extern __shared__ float sm[];
  const int strip = blockIdx.x % s.nstrip, rest = blockIdx.x / s.nstrip;
  const int c = rest % s.nchunk, lb = rest / s.nchunk, l = view0 + lb;
  int k0, k1;
  strip_range(s, strip, k0, k1);
  const int j0 = (int)(((long long)c * s.ny) / s.nchunk), j1 = (int)(((long long)(c + 1) * s.ny) / s.nchunk);
  const int WR = s.ZS + s.NBz;                     // staged input rows
  const int TW = s.nx8 + s.NBx;                    // z-pass columns
  const int TS = TW | 1;                           // odd row stride: rows of a wave hit distinct banks
  float* Ws = sm;                                  // WR x nx
  float* T = Ws + WR * s.nx;                       // ZS x TS
  SepTaps tp = carve_taps(T + s.ZS * TS, s);
  // staged row r <-> input row clamp(k0 + hb - NBz + r); T column tc <-> x = clamp(tc - xo)
  const int rbase = k0 + s.hb - s.NBz, xo = s.NBx - s.ha;
  const size_t row_stride = (size_t)s.ny * s.nx;
  const float* Wl = W + (size_t)lb * s.nz * row_stride;
  const int zo = s.ZS / kOct, xoct = s.nx8 / kOct;
  float acc[kSepOcts][kOct];
#pragma unroll
  for (int u = 0; u < kSepOcts; ++u)
#pragma unroll
    for (int d = 0; d < kOct; ++d) acc[u][d] = 0.0f;
  SepRows pf;
  if (j0 < j1) pf.load(s, Wl + (size_t)j0 * s.nx, rbase, WR, row_stride);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                               // previous plane consumed
    pf.store(s, Ws, WR);
    load_taps(s, psf + ((size_t)l * s.ny + j) * (s.pz + s.px), tp, false);
    __syncthreads();
    if (j + 1 < j1) pf.load(s, Wl + (size_t)(j + 1) * s.nx, rbase, WR, row_stride);
    // z pass on the real columns: T[kk][x + xo] = sum_b fz[b] w[clamp(k + hb - b)][x],
    // output kk = 8 q + d reads staged row kk + NBz - b; the edge columns also
    // fill the halo columns (clamped x)
    for (int e = threadIdx.x; e < zo * s.nx; e += kSepThreads) {
      const int q = e / s.nx, x = e - q * s.nx;
      float o[kOct];
#pragma unroll
      for (int d = 0; d < kOct; ++d) o[d] = 0.0f;
      convD<kOct>(Ws + x, s.nx, kOct * q + s.NBz, tp.gz, s.NBz, o);
#pragma unroll
      for (int d = 0; d < kOct; ++d) T[(kOct * q + d) * TS + x + xo] = o[d];
    }
    __syncthreads();
    // halo columns: copies of the edge columns (x clamped)
    const int nh = TW - s.nx;
    for (int e = threadIdx.x; e < s.ZS * nh; e += kSepThreads) {
      const int kk = e / nh, h = e - kk * nh;
      float* row = T + kk * TS;
      const int tc = h < xo ? h : s.nx + h;       // h >= xo: right halo column nx + h
      row[tc] = row[h < xo ? xo : xo + s.nx - 1];
    }
    __syncthreads();
    // x pass: out[kk][i] += sum_a fx[a] T[kk][i + NBx - a] (lanes along kk)
#pragma unroll
    for (int u = 0; u < kSepOcts; ++u) {
      const int e = threadIdx.x + kSepThreads * u;
      if (e < s.ZS * xoct) {
        const int io = e / s.ZS, kk = e - io * s.ZS;
        convD<kOct>(T + kk * TS, 1, kOct * io + s.NBx, tp.gx, s.NBx, acc[u]);
      }
    }
  }
  float* out = partial + ((size_t)c * nvb + lb) * s.nz * s.nx;
#pragma unroll
  for (int u = 0; u < kSepOcts; ++u) {
    const int e = threadIdx.x + kSepThreads * u;
    if (e < s.ZS * xoct) {
      const int io = e / s.ZS, kk = e - io * s.ZS;
      const int k = k0 + kk;
#pragma unroll
      for (int d = 0; d < kOct; ++d) {
        const int i = kOct * io + d;
        if (k < k1 && i < s.nx) out[(size_t)k * s.nx + i] = acc[u][d];
      }
    }
  }
}

// ---------------------------------------------------------------- adjoint
// grid: nstrip * nchunk_back * nvb workgroups.
// LDS: Vs GR x VS projection rows (zero outside), G GR x GS x-pass output,
// taps.  Staged / intermediate row r <-> z = k0 + hb - NBz + r.
__global__ __launch_bounds__(kSepThreads) void conv_back_sep(const float* __restrict__ v,
                                                             const float* __restrict__ psf,
                                                             float* __restrict__ U, SepShape s,
                                                             int view0, int nvb) {
  extern __shared__ float sm[];
  const int strip = blockIdx.x % s.nstrip, rest = blockIdx.x / s.nstrip;
  const int c = rest % s.nchunk_back, lb = rest / s.nchunk_back, l = view0 + lb;
  int k0, k1;
  strip_range(s, strip, k0, k1);
  const int j0 = (int)(((long long)c * s.ny) / s.nchunk_back);
  const int j1 = (int)(((long long)(c + 1) * s.ny) / s.nchunk_back);
  const int GR = s.ZS + s.NBz;
  const int VW = s.nx8 + s.NBx;                    // column vc <-> x = vc + ha - NBx
  const int VS = VW | 1, GS = s.nx8 | 1;           // odd row strides (rows of a wave: distinct banks)
  float* Vs = sm;                                  // GR x VS
  float* G = Vs + GR * VS;                         // GR x GS
  SepTaps tp = carve_taps(G + GR * GS, s);
  const int rbase = k0 + s.hb - s.NBz, xbase = s.ha - s.NBx;
  const int r_lo = max(0, -rbase), r_hi = min(GR, s.nz - rbase);   // rows inside the volume
  const float* vl = v + (size_t)l * s.nz * s.nx;
  for (int e = threadIdx.x; e < GR * VW; e += kSepThreads) {
    const int r = e / VW, vc = e - r * VW;
    const int z = rbase + r, x = xbase + vc;
    Vs[r * VS + vc] = (z >= 0 && z < s.nz && x >= 0 && x < s.nx) ? vl[(size_t)z * s.nx + x] : 0.0f;
  }
  // rows outside the volume are the zero padding of the z pass, for every plane
  for (int e = threadIdx.x; e < GR * GS; e += kSepThreads) {
    const int r = e / GS;
    if (r < r_lo || r >= r_hi) G[e] = 0.0f;
  }
  const int nr = r_hi - r_lo, xoct = s.nx8 / kOct, zo = s.ZS / kOct;
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                               // projection staged / previous plane consumed
    load_taps(s, psf + ((size_t)l * s.ny + j) * (s.pz + s.px), tp, true);
    __syncthreads();
    // x pass (zero-padded correlation): G[r][i] = sum_a fx[a] v[z][i - ha + a]
    //   = sum_b gx[b] Vs[r][i + NBx - b], gx reversed (lanes along r)
    for (int e = threadIdx.x; e < nr * xoct; e += kSepThreads) {
      const int io = e / nr, r = r_lo + (e - io * nr);
      float o[kOct];
#pragma unroll
      for (int d = 0; d < kOct; ++d) o[d] = 0.0f;
      convD<kOct>(Vs + r * VS, 1, kOct * io + s.NBx, tp.gx, s.NBx, o);
#pragma unroll
      for (int d = 0; d < kOct; ++d) G[r * GS + kOct * io + d] = o[d];
    }
    __syncthreads();
    // x edges: the fold of replicate padding onto x = 0 and x = nx - 1
    for (int e = threadIdx.x; e < 2 * nr; e += kSepThreads) {
      const int r = r_lo + (e >> 1), side = e & 1;
      const float* row = Vs + r * VS - xbase;      // row[x] = v[z][x]
      float a = 0.0f;
      if (s.nx == 1) {
        a = row[0] * tp.sxf[0];
      } else if (side == 0) {
        for (int i = 0; i <= s.ha && i < s.nx; ++i) a = fmaf(row[i], tp.sxf[s.ha + i], a);
      } else {
        for (int i = max(0, s.nx - 1 - s.ha); i < s.nx; ++i) a = fmaf(row[i], tp.sxp[i + s.ha - s.nx + 1], a);
      }
      if (side == 0 || s.nx > 1) G[r * GS + (side ? s.nx - 1 : 0)] = a;
    }
    __syncthreads();
    // z pass (zero-padded correlation): u[k][i] = sum_b fz[b] G(k - hb + b)[i]
    //   = sum_b gz[b] G[kk + NBz - b][i], kk = k - k0; edge rows come next
    float* Uj = U + (size_t)lb * s.nz * s.ny * s.nx + (size_t)j * s.nx;
    const size_t kst = (size_t)s.ny * s.nx;
    for (int e = threadIdx.x; e < zo * s.nx; e += kSepThreads) {
      const int q = e / s.nx, i = e - q * s.nx;
      float o[kOct];
#pragma unroll
      for (int d = 0; d < kOct; ++d) o[d] = 0.0f;
      convD<kOct>(G + i, GS, kOct * q + s.NBz, tp.gz, s.NBz, o);
#pragma unroll
      for (int d = 0; d < kOct; ++d) {
        const int k = k0 + kOct * q + d;
        const bool edge = (k == 0 || k == s.nz - 1);
        if (k < k1 && !edge) Uj[(size_t)k * kst + i] = o[d];
      }
    }
    // z edges of this strip: k = 0 and k = nz - 1 (G row of z is z - rbase)
    for (int e = threadIdx.x; e < 2 * s.nx; e += kSepThreads) {
      const int side = e / s.nx, i = e - side * s.nx;
      const int k = side ? s.nz - 1 : 0;
      if (k < k0 || k >= k1 || (side == 1 && s.nz == 1)) continue;
      float a = 0.0f;
      if (s.nz == 1) {
        a = G[(0 - rbase) * GS + i] * tp.szf[0];
      } else if (side == 0) {
        for (int z = 0; z <= s.hb && z < s.nz; ++z)
          a = fmaf(G[(z - rbase) * GS + i], tp.szf[s.hb + z], a);
      } else {
        for (int z = max(0, s.nz - 1 - s.hb); z < s.nz; ++z)
          a = fmaf(G[(z - rbase) * GS + i], tp.szp[z + s.hb - s.nz + 1], a);
      }
      Uj[(size_t)k * kst + i] = a;
    }
  }
}

int sep_wgs_per_cu(const void* fn, size_t sm) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kSepThreads, sm) != hipSuccess) nb = 0;
  return nb < 1 ? 1 : nb;
}

int sep_pick_chunks(int ny, long long units, long long slots) {
  int best = 1;
  long long best_cost = -1;
  for (int n = 1; n <= kMaxChunks && n <= ny; ++n) {
    const long long rounds = (units * n + slots - 1) / slots;
    const long long cost = rounds * ((ny + n - 1) / n);
    if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = n; }
  }
  return best;
}

}  // namespace

size_t sep_lds_bytes(const SepShape& s, bool back) {
  const size_t taps = (size_t)sep_taps_floats(s);
  const size_t rows = (size_t)s.ZS + s.NBz;
  if (back) return (rows * ((s.nx8 + s.NBx) | 1) + rows * (s.nx8 | 1) + taps) * sizeof(float);
  return (rows * s.nx + (size_t)s.ZS * ((s.nx8 + s.NBx) | 1) + taps) * sizeof(float);
}

SepShape make_sep_shape(const spect_geom& g) {
  SepShape s{};
  s.nx = g.nx; s.ny = g.ny; s.nz = g.nz; s.px = g.px; s.pz = g.pz;
  s.ha = (g.px - 1) / 2; s.hb = (g.pz - 1) / 2;
  s.NBx = (g.px + 3) / 4 * 4;
  s.NBz = (g.pz + 3) / 4 * 4;
  s.nx8 = (g.nx + kOct - 1) / kOct * kOct;
  s.ok = false;
  // largest strip (multiple of 8 rows) that fits LDS, the forward's
  // register-held outputs and its prefetched rows, then balanced over the
  // strips it takes
  int zs = (g.nz + kOct - 1) / kOct * kOct;
  for (; zs >= kOct; zs -= kOct) {
    s.ZS = zs;
    if (sep_lds_bytes(s, false) <= kLdsBytes && sep_lds_bytes(s, true) <= kLdsBytes &&
        zs * (s.nx8 / kOct) <= kSepThreads * (kSepOcts) &&
        zs + s.NBz <= (kSepThreads / 64) * kPfRows && g.nx <= 64 * kPfCols)
      break;
  }
  if (zs < kOct) return s;
  s.nstrip = (g.nz + zs - 1) / zs;
  s.ZS = ((g.nz + s.nstrip - 1) / s.nstrip + kOct - 1) / kOct * kOct;
  s.nchunk = 1;
  s.nchunk_back = 1;
  s.ok = true;
  return s;
}

void tune_sep_chunks(SepShape& s, int views) {
  int dev = 0, cus = 0;
  if (!s.ok || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    return;
  const int fw = sep_wgs_per_cu((const void*)conv_fwd_sep, sep_lds_bytes(s, false));
  const int bw = sep_wgs_per_cu((const void*)conv_back_sep, sep_lds_bytes(s, true));
  const long long units = (long long)s.nstrip * views;
  s.nchunk = sep_pick_chunks(s.ny, units, (long long)cus * fw);
  s.nchunk_back = sep_pick_chunks(s.ny, units, (long long)cus * bw);
}

hipError_t launch_conv_sep(const Plan& p, bool back, const float* in, float* out, int view0,
                           int nvb, hipStream_t st) {
  const SepShape& s = p.sep;
  const size_t sm = sep_lds_bytes(s, back);
  const void* fn = back ? (const void*)conv_back_sep : (const void*)conv_fwd_sep;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e != hipSuccess) return e;
  const dim3 grid(s.nstrip * (back ? s.nchunk_back : s.nchunk) * nvb);
  if (back)
    hipLaunchKernelGGL(conv_back_sep, grid, dim3(kSepThreads), sm, st, in, p.psf, out, s, view0, nvb);
  else
    hipLaunchKernelGGL(conv_fwd_sep, grid, dim3(kSepThreads), sm, st, in, p.psf, out, s, view0, nvb);
  return hipGetLastError();
}

}  // namespace spect
