// PSF convolution through the FFT (Sec. II-A convolves every depth plane with
// its PSF by FFT, with replicate padding), and its exact adjoint.
//
// The operator is the direct one,
//   c[i,k] = sum_{a,b} p[b][a] w[clamp(k - b + hb)][clamp(i - a + ha)],
// written as a linear convolution of the replicate-padded plane wt (size
// (nz + 2 hb) x (nx + 2 ha)) with p, of which the bins (k + 2 hb, i + 2 ha)
// are kept.  A circular convolution of size Lz x Lx with Lz >= nz + 2 hb and
// Lx >= nx + 2 ha equals the linear one on those bins (the taps never reach
// past the start of the padded plane), so c = crop(IDFT(DFT(p) DFT(wt))), and
// the depth sum of Alg. 1 is taken on the spectra: one inverse transform per
// view.  The adjoint (Alg. 2) places the projection at (2 hb, 2 ha),
// multiplies its spectrum by conj(DFT(p)) (a circular correlation, which for
// the same sizes equals the zero-padded one on the whole padded plane), and
// folds the padded plane onto the edge rows and columns (the adjoint of
// replicate padding).  Lx and Lz are the smallest even products of 2, 3 and 5
// that hold the padded plane.
//
// Transforms run in LDS, one plane per workgroup at a time, as mixed-radix
// Stockham passes (radix 2, 3, 4, 5): all butterflies of a pass read their
// operands into registers, the workgroup synchronises, and they write back.
// A real plane of Lz rows is transformed as Lz/2 complex rows (row k plus i
// times row k + Lz/2) along x; unpacking the pair gives each row's spectrum
// for x frequencies 0..Lx/2, stored in place: frequency f of the first row
// at column f, of the second at column Lx - f; the two real columns of
// frequencies 0 and Lx/2 share column 0 / Lx/2 as one complex column.  The z
// transforms then run down these Lx/2 virtual columns.  Spectra leave LDS as
// "slots": the (Lx/2 - 1) x Lz complex bins of frequencies 1..Lx/2-1, then
// for z frequencies 0..Lz/2 the bins of the two real columns (unpacked).
// The PSF spectra (scaled by 1 / (Lx Lz), so no other normalisation is
// needed) are computed once per plan and read per plane in slot order, each
// thread owning a fixed set of slots.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "fft_core.h"
#include "internal.h"

namespace spect {
namespace {

using namespace fft;

constexpr int kFftThreads = 512;
constexpr int kMaxPlane = 12288;  // complex elements of the LDS plane (Lz / 2 x Lx) at most
constexpr int kMaxSlots = 24;     // regular slots a thread owns
constexpr int kMaxPlaneRegs = 24; // raw plane values a thread prefetches (forward)
constexpr int kMaxFftLen = 1024;   // transform length along x at most

// One in-place pass of radix R over `batch` transforms of length N, stage of
// sub-transform length Ns (S = Ns / R).  Forward (decimation in frequency):
// for block o and offset k < S, the R elements o Ns + k + r S go through an
// R-point DFT and output r' is multiplied by exp(-2 pi i r' k / Ns).  Inverse:
// the exact reverse (conjugate twiddles first, then the inverse R-point
// DFT).  Every butterfly writes back where it read, so a thread can finish
// one butterfly before it reads the next.  tw[t] = exp(-2 pi i t / N).
// `bmajor`: consecutive threads take consecutive transforms (columns).
template <int R, bool kInv, class Addr>
__device__ __forceinline__ void ct_pass(float2* A, Addr addr, int N, int batch, int Ns,
                                        const float2* tw, bool bmajor) {
  const int S = Ns / R, Nb = N / R, B = batch * Nb, step = N / Ns;
  const int outer = bmajor ? batch : Nb;
  const float r_outer = 1.0f / (float)outer, r_s = 1.0f / (float)S;
#pragma unroll 1
  for (int b = threadIdx.x; b < B; b += kFftThreads) {
    const int hi = fdiv(b, r_outer), lo = b - hi * outer;
    const int tb = bmajor ? lo : hi, j = bmajor ? hi : lo;
    const int o = fdiv(j, r_s), k = j - o * S;
    const int base = o * Ns + k;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = A[addr(tb, base + r * S)];
    // the last pass (S = 1) has no twiddles
    if (kInv) {
      if (S > 1) {
        float2 w[R];
        stage_twiddles<R>(w, tw, k * step);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmulc(v[r], w[r]);
      }
      dft_any<R, true>(v);
    } else {
      dft_any<R, false>(v);
      if (S > 1) {
        float2 w[R];
        stage_twiddles<R>(w, tw, k * step);
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) A[addr(tb, base + r * S)] = v[r];
  }
  __syncthreads();
}

// Passes [p0, p1) of a transform (of npass): forward in the order of the
// radices, inverse in the reverse order.
template <bool kInv, class Addr>
__device__ __forceinline__ void transforms(float2* A, Addr addr, int N, int batch, const int* rad,
                                           int npass, const float2* tw, bool bmajor, int p0 = 0,
                                           int p1 = -1) {
  if (p1 < 0) p1 = npass;
  for (int i = p0; i < p1; ++i) {
    const int q = kInv ? npass - 1 - i : i;
    int Ns = N;
    for (int t = 0; t < q; ++t) Ns /= rad[t];
    switch (rad[q]) {
#define SPECT_FFT_RADIX(R) \
      case R: ct_pass<R, kInv>(A, addr, N, batch, Ns, tw, bmajor); break;
      SPECT_FFT_RADIX(2) SPECT_FFT_RADIX(3) SPECT_FFT_RADIX(4) SPECT_FFT_RADIX(5)
      SPECT_FFT_RADIX(6) SPECT_FFT_RADIX(8) SPECT_FFT_RADIX(9) SPECT_FFT_RADIX(10)
      SPECT_FFT_RADIX(12) SPECT_FFT_RADIX(15)
#undef SPECT_FFT_RADIX
      default: break;
    }
  }
}

// Row pairs after the forward x transforms: Z = DFT(r1 + i r2) gives
// R1[f] = (Z[f] + conj Z[-f]) / 2 and R2[f] = -i (Z[f] - conj Z[-f]) / 2,
// stored at Z's own positions: R1[f] where Z[f] was, R2[f] where Z[-f] was;
// R1 and R2 at frequencies 0 and Lx/2 (real) as the pairs (R1[0], R1[Lx/2])
// and (R2[0], R2[Lx/2]).
__device__ __forceinline__ void unpack_rows(float2* A, const FftShape& s, const Tabs& t) {
  const int items = s.H * s.Lh;
  for (int e = threadIdx.x; e < items; e += kFftThreads) {
    const int p = fdiv(e, s.r_lh), f = e - p * s.Lh;
    float2* row = A + p * s.stride;
    if (f == 0) {
      const int cn = t.posx[s.Lh];
      const float2 z0 = row[0], zn = row[cn];
      row[0] = make_float2(z0.x, zn.x);
      row[cn] = make_float2(z0.y, zn.y);
    } else {
      const int cf = t.posx[f], cm = t.posx[s.Lx - f];
      const float2 zf = row[cf], zm = cconj(row[cm]);
      row[cf] = cscale(cadd(zf, zm), 0.5f);
      row[cm] = cimul(csub(zf, zm), -0.5f);
    }
  }
  __syncthreads();
}

// The inverse of unpack_rows, before the inverse x transforms:
// Z[f] = R1[f] + i R2[f], Z[-f] = conj R1[f] + i conj R2[f].
__device__ __forceinline__ void repack_rows(float2* A, const FftShape& s, const Tabs& t) {
  const int items = s.H * s.Lh;
  for (int e = threadIdx.x; e < items; e += kFftThreads) {
    const int p = fdiv(e, s.r_lh), f = e - p * s.Lh;
    float2* row = A + p * s.stride;
    if (f == 0) {
      const int cn = t.posx[s.Lh];
      const float2 a = row[0], b = row[cn];
      row[0] = make_float2(a.x, b.x);
      row[cn] = make_float2(a.y, b.y);
    } else {
      const int cf = t.posx[f], cm = t.posx[s.Lx - f];
      const float2 r1 = row[cf], r2 = row[cm];
      row[cf] = cadd(r1, cimul(r2, 1.0f));
      row[cm] = cadd(cconj(r1), cimul(cconj(r2), 1.0f));
    }
  }
  __syncthreads();
}

// Real plane (staged as row pairs in A) -> spectrum (virtual columns, z
// frequencies at posz).  before_last() runs before the last pass (the caller
// issues the loads it needs right after the transform there).
template <class F>
__device__ __forceinline__ void fft2_forward(float2* A, const FftShape& s, const Tabs& t,
                                             const float2* twx, const float2* twz, F&& before_last) {
  transforms<false>(A, RowAddr{s.stride}, s.Lx, s.H, s.rx, s.nrx, twx, false);
  unpack_rows(A, s, t);
  const ColAddr ca{s.stride, s.H, t.vc1, t.vc2};
  transforms<false>(A, ca, s.Lz, s.Lh, s.rz, s.nrz, twz, true, 0, s.nrz - 1);
  before_last();
  transforms<false>(A, ca, s.Lz, s.Lh, s.rz, s.nrz, twz, true, s.nrz - 1, s.nrz);
}
__device__ __forceinline__ void fft2_forward(float2* A, const FftShape& s, const Tabs& t,
                                             const float2* twx, const float2* twz) {
  fft2_forward(A, s, t, twx, twz, [] {});
}

// Spectrum -> real plane as row pairs in A (times Lx Lz).
__device__ __forceinline__ void fft2_inverse(float2* A, const FftShape& s, const Tabs& t,
                                             const float2* twx, const float2* twz) {
  transforms<true>(A, ColAddr{s.stride, s.H, t.vc1, t.vc2}, s.Lz, s.Lh, s.rz, s.nrz, twz, true);
  repack_rows(A, s, t);
  transforms<true>(A, RowAddr{s.stride}, s.Lx, s.H, s.rx, s.nrx, twx, false);
}

// LDS position of regular slot q: virtual column 1 + q mod (Lx/2 - 1), the
// element at row q / (Lx/2 - 1) of that column (whatever frequency sits
// there; every spectrum is laid out the same way).
__device__ __forceinline__ int slot_pos(const FftShape& s, const Tabs& t, int q) {
  const int r = fdiv(q, s.r_lh1), v = 1 + q - r * (s.Lh - 1);
  return r < s.H ? r * s.stride + t.vc1[v] : (r - s.H) * s.stride + t.vc2[v];
}
// LDS position of the packed real-column pair at z frequency zq.
__device__ __forceinline__ int col0_pos(const FftShape& s, const Tabs& t, int zq) {
  const int r = t.posz[zq];
  return r < s.H ? r * s.stride + t.vc1[0] : (r - s.H) * s.stride + t.vc2[0];
}

// Real plane value at (row k, column c) of the row-pair layout.
__device__ __forceinline__ float plane_at(const float2* A, const FftShape& s, int k, int c) {
  return k < s.H ? A[k * s.stride + c].x : A[(k - s.H) * s.stride + c].y;
}

// The two real columns' spectra at z frequency zq (0..Lz/2) from the packed
// column Y = X0 + i XN: X0 = (Y[zq] + conj Y[-zq]) / 2, XN = -i (Y[zq] - conj Y[-zq]) / 2.
__device__ __forceinline__ void unpack_col0(const float2* A, const FftShape& s, const Tabs& t,
                                            int zq, float2* x0, float2* xn) {
  const float2 y = A[col0_pos(s, t, zq)];
  const float2 ym = cconj(A[col0_pos(s, t, zq == 0 ? 0 : s.Lz - zq)]);
  *x0 = cscale(cadd(y, ym), 0.5f);
  *xn = cimul(csub(y, ym), -0.5f);
}

// Write the two real columns' spectra (z frequency zq in 0..Lz/2) into the
// packed column: Y[zq] = X0 + i XN and Y[-zq] = conj X0 + i conj XN; at
// zq = 0 and Lz/2 both spectra are real.
__device__ __forceinline__ void pack_col0(float2* A, const FftShape& s, const Tabs& t, int zq,
                                          float2 x0, float2 xn) {
  if (zq == 0 || zq == s.H) {
    A[col0_pos(s, t, zq)] = make_float2(x0.x, xn.x);
  } else {
    A[col0_pos(s, t, zq)] = cadd(x0, cimul(xn, 1.0f));
    A[col0_pos(s, t, s.Lz - zq)] = cadd(cconj(x0), cimul(cconj(xn), 1.0f));
  }
}

// tw[t] = exp(-2 pi i t / N), t < N, from FP64.
__device__ __forceinline__ void init_twiddles(float2* tw, int N) {
  for (int t = threadIdx.x; t < N; t += kFftThreads) {
    double sn, cs;
    sincospi(-2.0 * (double)t / (double)N, &sn, &cs);
    tw[t] = make_float2((float)cs, (float)sn);
  }
}


__device__ __forceinline__ void chunk_range(int c, int nchunk, int ny, int& j0, int& j1) {
  j0 = (int)(((long long)c * ny) / nchunk);
  j1 = (int)(((long long)(c + 1) * ny) / nchunk);
}

__device__ __forceinline__ int clampi(int q, int lo, int hi) { return q < lo ? lo : (q > hi ? hi : q); }

// LDS of the transform kernels: the plane (Lz/2 x Lx complex), twiddles of
// both lengths, the index tables and (forward) the raw plane being staged.
struct Smem {
  float2* A;
  float2* twx;
  float2* twz;
  int* tab;
  float* raw;
  Tabs t;
};
__device__ __forceinline__ int tab_ints(const FftShape& s) { return 2 * s.Lx + s.Lz; }
__device__ __forceinline__ Smem carve(float2* sm, const FftShape& s) {
  Smem m;
  m.A = sm;
  m.twx = sm + s.H * s.stride;
  m.twz = m.twx + s.Lx;
  m.tab = reinterpret_cast<int*>(m.twz + s.Lz);
  m.raw = reinterpret_cast<float*>(m.tab + tab_ints(s));
  m.t.posx = m.tab;
  m.t.posz = m.tab + s.Lx;
  m.t.vc1 = m.tab + s.Lx + s.Lz;
  m.t.vc2 = m.tab + s.Lx + s.Lz + s.Lh;
  return m;
}
// Twiddles and index tables into LDS (the caller synchronises before use).
__device__ __forceinline__ void setup(const Smem& m, const FftShape& s, const int* __restrict__ gtab) {
  init_twiddles(m.twx, s.Lx);
  init_twiddles(m.twz, s.Lz);
  for (int e = threadIdx.x; e < tab_ints(s); e += kFftThreads) m.tab[e] = gtab[e];
}

// Spectrum slots of the plane in A (after fft2_forward) scaled by `scale`,
// written to out[0 .. NS).
__device__ __forceinline__ void store_slots(const float2* A, const FftShape& s, const Tabs& t,
                                            float2* out, float scale) {
  for (int q = threadIdx.x; q < s.NR; q += kFftThreads)
    out[q] = cscale(A[slot_pos(s, t, q)], scale);
  for (int zq = threadIdx.x; zq <= s.H; zq += kFftThreads) {
    float2 x0, xn;
    unpack_col0(A, s, t, zq, &x0, &xn);
    out[s.NR + 2 * zq] = cscale(x0, scale);
    out[s.NR + 2 * zq + 1] = cscale(xn, scale);
  }
}

// ---------------------------------------------------------------- kernels

// Index tables (one workgroup): posx, posz (digit reversal), then vc1 / vc2.
__global__ __launch_bounds__(kFftThreads) void fft_index_tables(int* __restrict__ out, FftShape s) {
  __shared__ int inv[kMaxFftLen];
  int* posx = out;
  int* posz = out + s.Lx;
  int* vc1 = out + s.Lx + s.Lz;
  int* vc2 = vc1 + s.Lh;
  for (int f = threadIdx.x; f < s.Lx + s.Lz; f += kFftThreads) {
    const bool isx = f < s.Lx;
    const int N = isx ? s.Lx : s.Lz, npass = isx ? s.nrx : s.nrz;
    const int* rad = isx ? s.rx : s.rz;
    int rem = isx ? f : f - s.Lx, mult = N, pos = 0;
    for (int q = 0; q < npass; ++q) {
      mult /= rad[q];
      pos += (rem % rad[q]) * mult;
      rem /= rad[q];
    }
    if (isx) {
      posx[f] = pos;
      inv[pos] = f;
    } else {
      posz[f - s.Lx] = pos;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int n = 0;
    for (int c = 0; c < s.Lx; ++c) {
      const int f = inv[c];
      if (f < s.Lh) {
        vc1[n] = c;
        n += 0;
        int cm = 0;
        const int g = f == 0 ? s.Lh : s.Lx - f;
        // position of frequency g (digit reversal, as above)
        int rem = g, mult = s.Lx;
        for (int q = 0; q < s.nrx; ++q) {
          mult /= s.rx[q];
          cm += (rem % s.rx[q]) * mult;
          rem /= s.rx[q];
        }
        vc2[n] = cm;
        ++n;
      }
    }
  }
}

// PSF spectra, one workgroup per (plane j, view l): p[b][a] at row b, column
// a of an Lz x Lx plane, transformed and scaled by 1 / (Lx Lz).
__global__ __launch_bounds__(kFftThreads) void fft_psf_spectra(const float* __restrict__ psf,
                                                               const int* __restrict__ gtab,
                                                               float2* __restrict__ P, FftShape s) {
  extern __shared__ float2 sm2[];
  const Smem m = carve(sm2, s);
  const int jl = blockIdx.x;                       // l * ny + j
  const float* p = psf + (size_t)jl * s.pz * s.px;
  setup(m, s, gtab);
  for (int e = threadIdx.x; e < s.H * s.Lx; e += kFftThreads) {
    const int r = fdiv(e, s.r_lx), c = e - r * s.Lx;
    const float lo = (r < s.pz && c < s.px) ? p[r * s.px + c] : 0.0f;
    const float hi = (r + s.H < s.pz && c < s.px) ? p[(r + s.H) * s.px + c] : 0.0f;
    m.A[r * s.stride + c] = make_float2(lo, hi);
  }
  __syncthreads();
  fft2_forward(m.A, s, m.t, m.twx, m.twz);
  store_slots(m.A, s, m.t, P + (size_t)jl * s.NS, 1.0f / ((float)s.Lx * (float)s.Lz));
}

// Forward: the depth planes [j0, j1) of view l (chunk c), each staged with
// replicate padding, transformed and multiplied by its PSF spectrum; the sum
// over the chunk's planes is written as slots to part[c][lb].
template <int KS>
__global__ __launch_bounds__(kFftThreads) void conv_fwd_fft(const float* __restrict__ W,
                                                            const float2* __restrict__ P,
                                                            const int* __restrict__ gtab,
                                                            float2* __restrict__ part, FftShape s,
                                                            int view0, int nvb) {
  extern __shared__ float2 sm2[];
  const Smem m = carve(sm2, s);
  const int c = blockIdx.x % s.nchunk, lb = blockIdx.x / s.nchunk, l = view0 + lb;
  int j0, j1;
  chunk_range(c, s.nchunk, s.ny, j0, j1);
  setup(m, s, gtab);
  const int tid = threadIdx.x, plane = s.nz * s.nx;
  const size_t rs = (size_t)s.ny * s.nx;           // stride between z rows of a plane
  const float* Wl = W + (size_t)lb * s.nz * rs;
  float2 acc[KS], a0 = make_float2(0.f, 0.f), an = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < KS; ++q) acc[q] = make_float2(0.f, 0.f);
  // plane j of W straight into the raw LDS region (no registers): lane L of
  // a wave writes the wave's base + 4 L bytes, so the wave covers 64
  // consecutive elements of the flattened [nz][nx] plane
  auto load_plane = [&](int j) {
    const int lane = tid & 63, wbase = tid - lane;
#pragma unroll
    for (int q = 0; q < kMaxPlaneRegs; ++q) {
      const int e0 = wbase + q * kFftThreads, e = e0 + lane;
      if (e < plane) {
        const int k = fdiv(e, s.r_nx), i = e - k * s.nx;
        __builtin_amdgcn_global_load_lds(Wl + (size_t)k * rs + (size_t)j * s.nx + i,
                                         (__attribute__((address_space(3))) void*)(m.raw + e0), 4, 0,
                                         0);
      }
    }
  };
  if (j0 < j1) load_plane(j0);
  const int KZ = s.nz + 2 * s.hb, IX = s.nx + 2 * s.ha;
  for (int j = j0; j < j1; ++j) {
    const float2* Pj = P + ((size_t)l * s.ny + j) * s.NS;
    float2 pr[KS], p0 = make_float2(0.f, 0.f), pn = make_float2(0.f, 0.f);
    // this plane's PSF spectrum, loaded during the transform's last pass
    auto load_p = [&] {
#pragma unroll
      for (int q = 0; q < KS; ++q) {
        const int sl = tid + q * kFftThreads;
        if (sl < s.NR) pr[q] = Pj[sl];
      }
      if (tid <= s.H) {
        p0 = Pj[s.NR + 2 * tid];
        pn = Pj[s.NR + 2 * tid + 1];
      }
    };
    __builtin_amdgcn_s_waitcnt(0);                 // this plane's loads into raw landed
    __syncthreads();                               // raw complete, A free, tables ready
    // padded plane wt[k][i] = w[clamp(k - hb)][clamp(i - ha)] on the
    // (nz + 2 hb) x (nx + 2 ha) corner, zero elsewhere; rows k and k + H paired
    for (int e = tid; e < s.H * s.Lx; e += kFftThreads) {
      const int r = fdiv(e, s.r_lx), cc = e - r * s.Lx;
      float lo = 0.0f, hi = 0.0f;
      if (cc < IX) {
        const int ii = clampi(cc - s.ha, 0, s.nx - 1);
        if (r < KZ) lo = m.raw[clampi(r - s.hb, 0, s.nz - 1) * s.nx + ii];
        if (r + s.H < KZ) hi = m.raw[clampi(r + s.H - s.hb, 0, s.nz - 1) * s.nx + ii];
      }
      m.A[r * s.stride + cc] = make_float2(lo, hi);
    }
    __syncthreads();                               // raw consumed
    if (j + 1 < j1) load_plane(j + 1);
    fft2_forward(m.A, s, m.t, m.twx, m.twz, load_p);
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int sl = tid + q * kFftThreads;
      if (sl < s.NR) {
        const float2 f = m.A[slot_pos(s, m.t, sl)];
        acc[q].x += pr[q].x * f.x - pr[q].y * f.y;
        acc[q].y += pr[q].x * f.y + pr[q].y * f.x;
      }
    }
    if (tid <= s.H) {
      float2 x0, xn;
      unpack_col0(m.A, s, m.t, tid, &x0, &xn);
      a0 = cadd(a0, cmul(p0, x0));
      an = cadd(an, cmul(pn, xn));
    }
  }
  float2* out = part + ((size_t)c * nvb + lb) * s.NS;
#pragma unroll
  for (int q = 0; q < KS; ++q) {
    const int sl = tid + q * kFftThreads;
    if (sl < s.NR) out[sl] = acc[q];
  }
  if (tid <= s.H) {
    out[s.NR + 2 * tid] = a0;
    out[s.NR + 2 * tid + 1] = an;
  }
}

// Forward, per view: the chunks' spectra summed in a fixed order, inverse
// transform, and the bins (k + 2 hb, i + 2 ha) written to v[l][k][i].
template <int KS>
__global__ __launch_bounds__(kFftThreads) void fwd_fft_finish(const float2* __restrict__ part,
                                                              const int* __restrict__ gtab,
                                                              float* __restrict__ v, FftShape s,
                                                              int view0, int nvb) {
  extern __shared__ float2 sm2[];
  const Smem m = carve(sm2, s);
  const int lb = blockIdx.x, l = view0 + lb, tid = threadIdx.x;
  setup(m, s, gtab);
  float2 acc[KS], a0 = make_float2(0.f, 0.f), an = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < KS; ++q) acc[q] = make_float2(0.f, 0.f);
  for (int c = 0; c < s.nchunk; ++c) {
    const float2* src = part + ((size_t)c * nvb + lb) * s.NS;
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int sl = tid + q * kFftThreads;
      if (sl < s.NR) acc[q] = cadd(acc[q], src[sl]);
    }
    if (tid <= s.H) {
      a0 = cadd(a0, src[s.NR + 2 * tid]);
      an = cadd(an, src[s.NR + 2 * tid + 1]);
    }
  }
  __syncthreads();                                 // tables ready
#pragma unroll
  for (int q = 0; q < KS; ++q) {
    const int sl = tid + q * kFftThreads;
    if (sl < s.NR) m.A[slot_pos(s, m.t, sl)] = acc[q];
  }
  if (tid <= s.H) pack_col0(m.A, s, m.t, tid, a0, an);
  __syncthreads();
  fft2_inverse(m.A, s, m.t, m.twx, m.twz);
  for (int e = tid; e < s.nz * s.nx; e += kFftThreads) {
    const int k = fdiv(e, s.r_nx), i = e - k * s.nx;
    v[((size_t)l * s.nz + k) * s.nx + i] = plane_at(m.A, s, k + 2 * s.hb, i + 2 * s.ha);
  }
}

// Adjoint, per view: the projection placed at (2 hb, 2 ha) of an Lz x Lx
// plane (zero elsewhere), transformed; slots to V[lb].
__global__ __launch_bounds__(kFftThreads) void back_fft_prep(const float* __restrict__ v,
                                                             const int* __restrict__ gtab,
                                                             float2* __restrict__ V, FftShape s,
                                                             int view0) {
  extern __shared__ float2 sm2[];
  const Smem m = carve(sm2, s);
  const int lb = blockIdx.x, l = view0 + lb;
  setup(m, s, gtab);
  const float* vl = v + (size_t)l * s.nz * s.nx;
  for (int e = threadIdx.x; e < s.H * s.Lx; e += kFftThreads) {
    const int r = fdiv(e, s.r_lx), cc = e - r * s.Lx;
    const int i = cc - 2 * s.ha, k1 = r - 2 * s.hb, k2 = r + s.H - 2 * s.hb;
    const bool in_i = i >= 0 && i < s.nx;
    const float lo = (in_i && k1 >= 0 && k1 < s.nz) ? vl[k1 * s.nx + i] : 0.0f;
    const float hi = (in_i && k2 >= 0 && k2 < s.nz) ? vl[k2 * s.nx + i] : 0.0f;
    m.A[r * s.stride + cc] = make_float2(lo, hi);
  }
  __syncthreads();
  fft2_forward(m.A, s, m.t, m.twx, m.twz);
  store_slots(m.A, s, m.t, V + (size_t)lb * s.NS, 1.0f);
}

// Adjoint: for each depth plane of chunk c of view l, the projection's
// spectrum times conj(PSF spectrum), inverse transform (the zero-padded
// correlation on the padded plane), and the fold of the padding onto the
// edges: u[k][i] = sum of the padded plane over the rows whose clamped
// source is k and the columns whose clamped source is i.  Written to
// U[lb][k][j][i].
template <int KS>
__global__ __launch_bounds__(kFftThreads) void conv_back_fft(const float2* __restrict__ V,
                                                             const float2* __restrict__ P,
                                                             const int* __restrict__ gtab,
                                                             float* __restrict__ U, FftShape s,
                                                             int view0, int nvb) {
  extern __shared__ float2 sm2[];
  const Smem m = carve(sm2, s);
  const int c = blockIdx.x % s.nchunk_back, lb = blockIdx.x / s.nchunk_back, l = view0 + lb;
  int j0, j1;
  chunk_range(c, s.nchunk_back, s.ny, j0, j1);
  setup(m, s, gtab);
  const int tid = threadIdx.x;
  const float2* Vl = V + (size_t)lb * s.NS;
  float2 vr[KS], v0 = make_float2(0.f, 0.f), vn = make_float2(0.f, 0.f);
  float2 pr[KS], p0 = make_float2(0.f, 0.f), pn = make_float2(0.f, 0.f);
  auto load_p = [&](int j) {
    const float2* Pj = P + ((size_t)l * s.ny + j) * s.NS;
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int sl = tid + q * kFftThreads;
      if (sl < s.NR) pr[q] = Pj[sl];
    }
    if (tid <= s.H) {
      p0 = Pj[s.NR + 2 * tid];
      pn = Pj[s.NR + 2 * tid + 1];
    }
  };
#pragma unroll
  for (int q = 0; q < KS; ++q) {
    const int sl = tid + q * kFftThreads;
    if (sl < s.NR) vr[q] = Vl[sl];
  }
  if (tid <= s.H) {
    v0 = Vl[s.NR + 2 * tid];
    vn = Vl[s.NR + 2 * tid + 1];
  }
  if (j0 < j1) load_p(j0);
  const size_t rs = (size_t)s.ny * s.nx;
  float* Ul = U + (size_t)lb * s.nz * rs;
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                               // A free, tables ready
#pragma unroll
    for (int q = 0; q < KS; ++q) {
      const int sl = tid + q * kFftThreads;
      if (sl < s.NR) m.A[slot_pos(s, m.t, sl)] = cmulc(vr[q], pr[q]);
    }
    if (tid <= s.H) pack_col0(m.A, s, m.t, tid, cmulc(v0, p0), cmulc(vn, pn));
    __syncthreads();
    if (j + 1 < j1) load_p(j + 1);
    fft2_inverse(m.A, s, m.t, m.twx, m.twz);
    fold_store(m.A, m.raw, s.nx, s.nz, s.ha, s.hb, Ul + (size_t)j * s.nx, rs,
               [&](const float2* A, int k, int c) { return plane_at(A, s, k, c); }, kFftThreads);
  }
}

int smallest_235_even(int n) {
  for (int L = std::max(2, n + (n & 1));; L += 2) {
    int r = L;
    for (int f : {2, 3, 5})
      while (r % f == 0) r /= f;
    if (r == 1) return L;
  }
}

// Radices of one transform: L as a product of the fewest radices the passes
// implement (2, 3, 4, 5 and the composites 6, 8, 9, 10, 12, 15), then the smallest
// largest radix.  Returns the number of passes (0 if L has no such split).
int radices(int L, int* out) {
  static const int kRad[] = {15, 12, 10, 9, 8, 6, 5, 4, 3, 2};
  int best_n = 0, best_max = 0, best[kMaxFftPass];
  int cur[kMaxFftPass];
  // depth-first over non-increasing sequences of radices
  auto search = [&](auto&& self, int rem, int depth, int maxr, int largest) -> void {
    if (rem == 1) {
      if (best_n == 0 || depth < best_n || (depth == best_n && largest < best_max)) {
        best_n = depth;
        best_max = largest;
        for (int i = 0; i < depth; ++i) best[i] = cur[i];
      }
      return;
    }
    if (depth == kMaxFftPass || (best_n && depth >= best_n)) return;
    for (int r : kRad)
      if (r <= maxr && rem % r == 0) {
        cur[depth] = r;
        self(self, rem / r, depth + 1, r, largest > r ? largest : r);
      }
  };
  search(search, L, 0, 15, 0);
  for (int i = 0; i < best_n; ++i) out[i] = best[i];
  return best_n;
}

// LDS bytes: the plane, twiddles and tables, then (kind 1) the forward's raw
// plane or (kind 2) the adjoint's column-folded padded plane.
size_t fft_smem(const FftShape& s, int kind) {
  const size_t extra = kind == 1 ? (size_t)s.nz * s.nx
                     : kind == 2 ? (size_t)(s.nz + 2 * s.hb) * s.nx
                                 : 0;
  return ((size_t)s.H * s.stride + s.Lx + s.Lz) * sizeof(float2) +
         (size_t)(2 * s.Lx + s.Lz) * sizeof(int) + extra * sizeof(float);
}

hipError_t set_fft_smem(const void* fn, size_t sm) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
}

const float2* spectra(const Plan& p) {
  return reinterpret_cast<const float2*>(p.ws + p.lay.fft_spectra);
}

const int* fft_tables(const Plan& p) { return reinterpret_cast<const int*>(p.ws + p.lay.fft_tables); }

template <int KS>
hipError_t launch_fwd_ks(const Plan& p, const float* W, int view0, int nvb, hipStream_t st) {
  const FftShape& s = p.fft;
  const size_t sm = fft_smem(s, 1);
  hipError_t e = set_fft_smem((const void*)conv_fwd_fft<KS>, sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(conv_fwd_fft<KS>, dim3((unsigned)(nvb * s.nchunk)), dim3(kFftThreads), sm, st,
                     W, spectra(p), fft_tables(p), reinterpret_cast<float2*>(p.ws + p.lay.fft_part),
                     s, view0, nvb);
  return hipGetLastError();
}

template <int KS>
hipError_t launch_finish_ks(const Plan& p, float* v, int view0, int nvb, hipStream_t st) {
  const FftShape& s = p.fft;
  const size_t sm = fft_smem(s, 0);
  hipError_t e = set_fft_smem((const void*)fwd_fft_finish<KS>, sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fwd_fft_finish<KS>, dim3((unsigned)nvb), dim3(kFftThreads), sm, st,
                     reinterpret_cast<const float2*>(p.ws + p.lay.fft_part), fft_tables(p), v, s,
                     view0, nvb);
  return hipGetLastError();
}

template <int KS>
hipError_t launch_back_ks(const Plan& p, float* U, int view0, int nvb, hipStream_t st) {
  const FftShape& s = p.fft;
  const size_t sm = fft_smem(s, 2);
  hipError_t e = set_fft_smem((const void*)conv_back_fft<KS>, sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(conv_back_fft<KS>, dim3((unsigned)(nvb * s.nchunk_back)), dim3(kFftThreads),
                     sm, st, reinterpret_cast<const float2*>(p.ws + p.lay.fft_vproj), spectra(p),
                     fft_tables(p), U, s, view0, nvb);
  return hipGetLastError();
}

// Instantiations by the number of slots a thread owns.
bool small_slots(const FftShape& s) { return (s.NR + kFftThreads - 1) / kFftThreads <= 8; }

int fft_pick_chunks(int ny, long long views, long long slots, bool prefer_more) {
  int best = 1;
  long long best_cost = -1;
  for (int n = 1; n <= kMaxChunks && n <= ny; ++n) {
    const long long rounds = (views * n + slots - 1) / slots;
    const long long cost = rounds * ((ny + n - 1) / n);
    if (best_cost < 0 || cost < best_cost || (prefer_more && cost == best_cost)) {
      best_cost = cost;
      best = n;
    }
  }
  return best;
}

}  // namespace

FftShape make_fft_shape(const spect_geom& g) {
  FftShape s{};
  s.nx = g.nx; s.ny = g.ny; s.nz = g.nz; s.px = g.px; s.pz = g.pz;
  s.ha = (g.px - 1) / 2; s.hb = (g.pz - 1) / 2;
  s.Lx = smallest_235_even(g.nx + g.px - 1);
  s.Lz = smallest_235_even(g.nz + g.pz - 1);
  s.Lh = s.Lx / 2;
  s.H = s.Lz / 2;
  s.stride = s.Lx;
  s.nrx = radices(s.Lx, s.rx);
  s.nrz = radices(s.Lz, s.rz);
  s.r_lx = 1.0f / (float)s.Lx;
  s.r_lh = 1.0f / (float)s.Lh;
  s.r_lh1 = s.Lh > 1 ? 1.0f / (float)(s.Lh - 1) : 0.0f;
  s.r_nx = 1.0f / (float)s.nx;
  s.NR = (s.Lh - 1) * s.Lz;
  s.NS = s.NR + 2 * (s.H + 1);
  s.nchunk = 1;
  s.nchunk_back = 1;
  // every pass fits the registers a thread holds, the slots and the
  // prefetched plane fit theirs, and the plane, raw plane and twiddles fit LDS
  bool ok = s.nrx > 0 && s.nrz > 0 && s.H * s.Lx <= kMaxPlane &&
            s.Lx <= kMaxFftLen &&
            (s.NR + kFftThreads - 1) / kFftThreads <= kMaxSlots && s.H + 1 <= kFftThreads &&
            g.nx <= kFftThreads &&
            g.nz * g.nx <= kMaxPlaneRegs * kFftThreads && fft_smem(s, 1) <= kLdsBytes &&
            fft_smem(s, 2) <= kLdsBytes;
  s.cfg = fft_fixed_config(s);
  s.ok = ok || s.cfg != 0;
  s.real = s.cfg != 0 && (g.flags & SPECT_PSF_SYMMETRIC_X) && (g.flags & SPECT_PSF_SYMMETRIC_Z);
  return s;
}

void tune_fft_chunks(FftShape& s, int views) {
  int dev = 0, cus = 0, nb = 0;
  if (!s.ok || hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    return;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)conv_fwd_fft<kMaxSlots>,
                                                   kFftThreads, fft_smem(s, 1)) != hipSuccess ||
      nb < 1)
    nb = 1;
  s.nchunk = fft_pick_chunks(s.ny, views, (long long)cus * nb, false);
  s.nchunk_back = fft_pick_chunks(s.ny, views, (long long)cus * nb, false);
}

hipError_t launch_fft_psf_spectra(const Plan& p, hipStream_t st) {
  const FftShape& s = p.fft;
  if (s.cfg) return launch_fft_fixed(p, kFftSpectra, nullptr, nullptr, 0, 0, st);
  hipLaunchKernelGGL(fft_index_tables, dim3(1), dim3(kFftThreads), 0, st,
                     reinterpret_cast<int*>(p.ws + p.lay.fft_tables), s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t sm = fft_smem(s, 0);
  e = hipFuncSetAttribute((const void*)fft_psf_spectra, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fft_psf_spectra, dim3((unsigned)(p.g.nview * p.g.ny)), dim3(kFftThreads), sm,
                     st, p.psf, fft_tables(p), reinterpret_cast<float2*>(p.ws + p.lay.fft_spectra), s);
  return hipGetLastError();
}

hipError_t launch_conv_fwd_fft(const Plan& p, const float* W, int view0, int nvb, hipStream_t st) {
  if (p.fft.cfg) return launch_fft_fixed(p, kFftForward, W, nullptr, view0, nvb, st);
  return small_slots(p.fft) ? launch_fwd_ks<8>(p, W, view0, nvb, st)
                            : launch_fwd_ks<kMaxSlots>(p, W, view0, nvb, st);
}

hipError_t launch_fwd_fft_finish(const Plan& p, float* v, int view0, int nvb, hipStream_t st) {
  if (p.fft.cfg) return launch_fft_fixed(p, kFftFinish, nullptr, v, view0, nvb, st);
  return small_slots(p.fft) ? launch_finish_ks<8>(p, v, view0, nvb, st)
                            : launch_finish_ks<kMaxSlots>(p, v, view0, nvb, st);
}

hipError_t launch_back_fft_prep(const Plan& p, const float* v, int view0, int nvb, hipStream_t st) {
  if (p.fft.cfg) return launch_fft_fixed(p, kFftBackPrep, v, nullptr, view0, nvb, st);
  const FftShape& s = p.fft;
  const size_t sm = fft_smem(s, 0);
  hipError_t e = set_fft_smem((const void*)back_fft_prep, sm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(back_fft_prep, dim3((unsigned)nvb), dim3(kFftThreads), sm, st, v,
                     fft_tables(p), reinterpret_cast<float2*>(p.ws + p.lay.fft_vproj), s, view0);
  return hipGetLastError();
}

hipError_t launch_conv_back_fft(const Plan& p, float* U, int view0, int nvb, hipStream_t st) {
  if (p.fft.cfg) return launch_fft_fixed(p, kFftBack, nullptr, U, view0, nvb, st);
  return small_slots(p.fft) ? launch_back_ks<8>(p, U, view0, nvb, st)
                            : launch_back_ks<kMaxSlots>(p, U, view0, nvb, st);
}

}  // namespace spect
