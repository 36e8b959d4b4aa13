// The FFT convolution of conv_fft.hip for transform sizes fixed at compile
// time (Sec. II-A: each depth plane convolved with its PSF by FFT, replicate
// padding; the adjoint with the padding's fold).  Same operator, same data
// flow and the same slot semantics (regular bins, then the two real columns'
// bins for z frequencies 0..Lz/2) as the runtime-size kernels; only the order
// of the regular slots differs (here: LDS order), and every spectrum a plan
// uses comes from the same kernels.  With the sizes and the two radices per
// axis known to the compiler, every index -- butterfly, twiddle, digit
// reversal, slot position -- is constant arithmetic instead of table lookups
// and divisions, and the LDS row stride is odd (Lx + 1 complex values), so
// that the transform-major passes read and write without bank conflicts.
//
// A configuration: Lx = Rx0 Rx1 (Rx1 even), Lz = Rz0 Rz1, each axis two
// in-place passes (decimation in frequency forward, the exact reverse
// inverse).  Frequency f along x sits at column (f mod Rx0) (Lx / Rx0) +
// f / Rx0; the frequencies below Lx/2 are those with f / Rx0 < Rx1 / 2, so
// virtual column v (x frequency v / (Rx1/2) + Rx0 (v mod Rx1/2)) starts at
// column (v / (Rx1/2)) (Lx / Rx0) + v mod (Rx1/2), and columns 0 and Rx1/2
// hold frequencies 0 and Lx/2.
#include "fft_core.h"
#include "internal.h"

namespace spect {
namespace {

using namespace fft;

__device__ __forceinline__ int clampi(int q, int lo, int hi) { return q < lo ? lo : (q > hi ? hi : q); }

// Threads of the forward convolution kernel.
constexpr int kFwdThreads = 768;

// Row stride (floats) of the raw W plane in LDS: odd when whole waves load
// whole row segments (nx a multiple of 64; fits() then also requires that the
// forward's waves split evenly over a row's segments), so that the lanes of
// the first x pass, on consecutive rows, read distinct banks; packed
// otherwise.
__host__ __device__ __forceinline__ int raw_stride(int nx) { return nx % 64 == 0 ? nx + 1 : nx; }


template <int LX, int LZ, int RX0, int RX1, int RZ0, int RZ1, int THREADS>
struct Cfg {
  static constexpr int T = THREADS;
  static constexpr int Lx = LX, Lz = LZ, Lh = LX / 2, H = LZ / 2, ST = LX + 1;
  static constexpr int Rx0 = RX0, Rx1 = RX1, Rz0 = RZ0, Rz1 = RZ1;
  static constexpr int Sx = LX / RX0, Sz = LZ / RZ0;
  static constexpr int HR = RX1 / 2;               // also the column of frequency Lx/2
  static constexpr int NR = H * (LX - 2), NS = NR + 2 * (H + 1);
  static constexpr int KS = (NR + T - 1) / T;
  static_assert(RX0 * RX1 == LX && RZ0 * RZ1 == LZ && RX1 % 2 == 0 && LZ % 2 == 0, "config");
  __device__ static int posx(int f) { return (f % RX0) * Sx + f / RX0; }
  __device__ static int posz(int q) { return (q % RZ0) * Sz + q / RZ0; }
  __device__ static int c1(int v) { return (v / HR) * Sx + v % HR; }
  __device__ static int c2(int v) {
    const int f = v / HR + RX0 * (v % HR);
    return posx(f == 0 ? Lh : LX - f);
  }
  // LDS index of regular slot q: row pair q / (Lx - 2), columns other than 0 and HR
  __device__ static int slot(int q) {
    const int p = q / (LX - 2), c = q - p * (LX - 2) + 1;
    return p * ST + c + (c >= HR ? 1 : 0);
  }
  // LDS index of the packed real-column pair at z frequency zq
  __device__ static int col0(int zq) {
    const int r = posz(zq);
    return r < H ? r * ST : (r - H) * ST + HR;
  }
};

// 128 x 80 planes with 37 x 37 PSFs, and 64 x 40 planes with 19 x 19 PSFs.
// The convolution kernels keep spectra per thread in registers (the forward
// its accumulators and the next PSF spectrum, the adjoint the next PSF
// spectrum), so they run 768 threads (170 registers per lane); the
// once-per-view kernels run 1024.
template <int T> using Cfg180x120 = Cfg<180, 120, 15, 12, 12, 10, T>;
template <int T> using Cfg90x60 = Cfg<90, 60, 9, 10, 10, 6, T>;

template <int T>
__device__ __forceinline__ void init_tw(float2* tw, int N) {
  for (int t = threadIdx.x; t < N; t += T) {
    double sn, cs;
    sincospi(-2.0 * (double)t / (double)N, &sn, &cs);
    tw[t] = make_float2((float)cs, (float)sn);
  }
}

// One in-place pass (see ct_pass in conv_fft.hip): radix R, sub-transform
// length Ns, rows (along x) or virtual columns (along z).  Lanes take
// consecutive transforms when the butterflies' stride S is short (then the
// odd row stride or the virtual-column order spreads them over the banks),
// consecutive butterflies otherwise.
template <class C, int R, int Ns, bool kCol, bool kInv>
__device__ __forceinline__ void pass(float2* A, const float2* tw) {
  constexpr int N = kCol ? C::Lz : C::Lx;
  constexpr int batch = kCol ? C::Lh : C::H;
  constexpr int S = Ns / R, Nb = N / R, B = batch * Nb, step = N / Ns;
  constexpr bool tmajor = S < 16;
#pragma unroll 1
  for (int b = threadIdx.x; b < B; b += C::T) {
    int tb, j;
    if (tmajor) { j = b / batch; tb = b - j * batch; }
    else { tb = b / Nb; j = b - tb * Nb; }
    const int o = j / S, k = j - o * S;
    const int t0 = o * Ns + k;
    int ad[R];
    if constexpr (!kCol) {
#pragma unroll
      for (int r = 0; r < R; ++r) ad[r] = tb * C::ST + t0 + r * S;
    } else {
      const int b1 = t0 * C::ST + C::c1(tb), b2 = (t0 - C::H) * C::ST + C::c2(tb);
#pragma unroll
      for (int r = 0; r < R; ++r) ad[r] = (t0 + r * S < C::H ? b1 : b2) + r * S * C::ST;
    }
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = A[ad[r]];
    // the last pass of an axis (S = 1) has no twiddles
    float2 w[R];
    if constexpr (S > 1) stage_twiddles<R>(w, tw, k * step);
    if constexpr (kInv) {
      if constexpr (S > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmulc(v[r], w[r]);
      }
      dft_any<R, true>(v);
    } else {
      dft_any<R, false>(v);
      if constexpr (S > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) A[ad[r]] = v[r];
  }
  __syncthreads();
}

// The last x pass (radix Rx1, no twiddles) fused with the unpack of the row
// pairs (see unpack_rows in conv_fft.hip), and its inverse fused with the
// repack.  After the pass, column o Rx1 + r of a row pair holds x frequency
// f = o + Rx0 r; for o >= 1 its mirror Lx - f sits at (Rx0 - o, Rx1 - 1 - r),
// and for o = 0 at (0, Rx1 - r).  So one thread takes butterflies u and
// Rx0 - u of a row pair (Rx0 odd) and unpacks every pair in registers: the
// member below Lx/2 (r < Rx1/2) gets R1 = (Z[f] + conj Z[-f]) / 2, the mirror
// R2 = -i (Z[f] - conj Z[-f]) / 2; frequencies 0 and Lx/2 (column 0 and
// Rx1/2) hold the two rows' real DC and Nyquist values.  Lanes take
// consecutive row pairs.
template <class C>
__device__ __forceinline__ void unpack_pair(float2& a, float2& b) {
  const float2 zf = a, zm = cconj(b);
  a = cscale(cadd(zf, zm), 0.5f);
  b = cimul(csub(zf, zm), -0.5f);
}

template <class C>
__device__ __forceinline__ void repack_pair(float2& a, float2& b) {
  const float2 r1 = a, r2 = b;
  a = cadd(r1, cimul(r2, 1.0f));
  b = cadd(cconj(r1), cimul(cconj(r2), 1.0f));
}

template <class C, bool kInv>
__device__ __forceinline__ void xpass_last_rows(float2* A) {
  constexpr int R = C::Rx1, U = (C::Rx0 + 1) / 2, B = C::H * U, HR = R / 2;
  static_assert(C::Rx0 % 2 == 1 && R % 2 == 0 && C::Rx1 * C::Rx0 == C::Lx, "row-pair split");
#pragma unroll 1
  for (int b = threadIdx.x; b < B; b += C::T) {
    const int u = b / C::H, tb = b - u * C::H;
    float2* row = A + tb * C::ST;
    if (u == 0) {
      float2 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = row[r];
      if constexpr (!kInv) {
        dft_any<R, false>(v);
        const float2 z0 = v[0], zn = v[HR];
        v[0] = make_float2(z0.x, zn.x);
        v[HR] = make_float2(z0.y, zn.y);
#pragma unroll
        for (int r = 1; r < HR; ++r) unpack_pair<C>(v[r], v[R - r]);
      } else {
        const float2 a = v[0], c = v[HR];
        v[0] = make_float2(a.x, c.x);
        v[HR] = make_float2(a.y, c.y);
#pragma unroll
        for (int r = 1; r < HR; ++r) repack_pair<C>(v[r], v[R - r]);
        dft_any<R, true>(v);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) row[r] = v[r];
    } else {
      float2* p1 = row + u * R;
      float2* p2 = row + (C::Rx0 - u) * R;
      float2 v1[R], v2[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        v1[r] = p1[r];
        v2[r] = p2[r];
      }
      if constexpr (!kInv) {
        dft_any<R, false>(v1);
        dft_any<R, false>(v2);
#pragma unroll
        for (int r = 0; r < HR; ++r) {
          unpack_pair<C>(v1[r], v2[R - 1 - r]);
          unpack_pair<C>(v2[r], v1[R - 1 - r]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < HR; ++r) {
          repack_pair<C>(v1[r], v2[R - 1 - r]);
          repack_pair<C>(v2[r], v1[R - 1 - r]);
        }
        dft_any<R, true>(v1);
        dft_any<R, true>(v2);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        p1[r] = v1[r];
        p2[r] = v2[r];
      }
    }
  }
  __syncthreads();
}

// The first x pass of the forward transform (radix Rx0, stride Lx / Rx0,
// twiddle exp(-2 pi i r k / Lx)) with its input read straight from a raw
// nz x nx plane in LDS (rows of `rs` floats): element (row q, column c) of
// the replicate-padded plane is raw[clamp(q - hb)][clamp(c - ha)] for
// q < nz + 2 hb and c < nx + 2 ha, and 0 beyond; row pair tb holds rows tb
// and tb + H.  Lanes take consecutive row pairs.
template <class C>
__device__ __forceinline__ void xpass_first_from_raw(float2* A, const float2* tw, const float* raw,
                                                     int rs, int nx, int nz, int ha, int hb) {
  constexpr int R = C::Rx0, S = C::Lx / R, B = C::H * S;
  const int KZ = nz + 2 * hb, IX = nx + 2 * ha;
#pragma unroll 1
  for (int b = threadIdx.x; b < B; b += C::T) {
    const int k = b / C::H, tb = b - k * C::H;
    const bool lo_ok = tb < KZ, hi_ok = tb + C::H < KZ;
    const float* rlo = raw + clampi(tb - hb, 0, nz - 1) * rs;
    const float* rhi = raw + clampi(tb + C::H - hb, 0, nz - 1) * rs;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = k + r * S;
      const int i = clampi(c - ha, 0, nx - 1);
      const bool in_c = c < IX;
      v[r] = make_float2(lo_ok && in_c ? rlo[i] : 0.0f, hi_ok && in_c ? rhi[i] : 0.0f);
    }
    float2 w[R];
    stage_twiddles<R>(w, tw, k);
    dft_any<R, false>(v);
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
    float2* row = A + tb * C::ST + k;
#pragma unroll
    for (int r = 0; r < R; ++r) row[r * S] = v[r];
  }
  __syncthreads();
}

// Forward 2-D transform after the first x pass; `before_last` runs before
// the last z pass (the callers prefetch there).
template <class C, class F>
__device__ __forceinline__ void fft2_fwd_rest(float2* A, const float2* twz, F&& before_last) {
  xpass_last_rows<C, false>(A);
  pass<C, C::Rz0, C::Lz, true, false>(A, twz);
  before_last();
  pass<C, C::Rz1, C::Rz1, true, false>(A, twz);
}

template <class C, class F>
__device__ __forceinline__ void fft2_fwd(float2* A, const float2* twx, const float2* twz,
                                         F&& before_last) {
  pass<C, C::Rx0, C::Lx, false, false>(A, twx);
  fft2_fwd_rest<C>(A, twz, before_last);
}

template <class C>
__device__ __forceinline__ void fft2_inv(float2* A, const float2* twx, const float2* twz) {
  pass<C, C::Rz1, C::Rz1, true, true>(A, twz);
  pass<C, C::Rz0, C::Lz, true, true>(A, twz);
  xpass_last_rows<C, true>(A);
  pass<C, C::Rx0, C::Lx, false, true>(A, twx);
}

template <class C>
__device__ __forceinline__ float plane_at(const float2* A, int k, int c) {
  return k < C::H ? A[k * C::ST + c].x : A[(k - C::H) * C::ST + c].y;
}

template <class C>
__device__ __forceinline__ void unpack_col0(const float2* A, int zq, float2* x0, float2* xn) {
  const float2 y = A[C::col0(zq)];
  const float2 ym = cconj(A[C::col0(zq == 0 ? 0 : C::Lz - zq)]);
  *x0 = cscale(cadd(y, ym), 0.5f);
  *xn = cimul(csub(y, ym), -0.5f);
}

template <class C>
__device__ __forceinline__ void pack_col0(float2* A, int zq, float2 x0, float2 xn) {
  if (zq == 0 || zq == C::H) {
    A[C::col0(zq)] = make_float2(x0.x, xn.x);
  } else {
    A[C::col0(zq)] = cadd(x0, cimul(xn, 1.0f));
    A[C::col0(C::Lz - zq)] = cadd(cconj(x0), cimul(cconj(xn), 1.0f));
  }
}

// Real spectra (PSFs symmetric in x and z, centred on the origin): the real
// parts, one float per slot.
template <class C>
__device__ __forceinline__ void store_slots_real(const float2* A, float* out, float scale) {
  for (int q = threadIdx.x; q < C::NR; q += C::T) out[q] = A[C::slot(q)].x * scale;
  for (int zq = threadIdx.x; zq <= C::H; zq += C::T) {
    float2 x0, xn;
    unpack_col0<C>(A, zq, &x0, &xn);
    out[C::NR + 2 * zq] = x0.x * scale;
    out[C::NR + 2 * zq + 1] = xn.x * scale;
  }
}

template <class C>
__device__ __forceinline__ void store_slots(const float2* A, float2* out, float scale) {
  for (int q = threadIdx.x; q < C::NR; q += C::T) out[q] = cscale(A[C::slot(q)], scale);
  for (int zq = threadIdx.x; zq <= C::H; zq += C::T) {
    float2 x0, xn;
    unpack_col0<C>(A, zq, &x0, &xn);
    out[C::NR + 2 * zq] = cscale(x0, scale);
    out[C::NR + 2 * zq + 1] = cscale(xn, scale);
  }
}


__device__ __forceinline__ void chunk_range(int c, int nchunk, int ny, int& j0, int& j1) {
  j0 = (int)(((long long)c * ny) / nchunk);
  j1 = (int)(((long long)(c + 1) * ny) / nchunk);
}

// LDS: plane (H x ST complex), twiddles (Lx + Lz), then the raw plane
// (forward) or the column-folded plane (adjoint).
template <class C>
struct Lds {
  float2* A;
  float2* twx;
  float2* twz;
  float* extra;
  __device__ explicit Lds(float2* sm) {
    A = sm;
    twx = sm + C::H * C::ST;
    twz = twx + C::Lx;
    extra = reinterpret_cast<float*>(twz + C::Lz);
  }
  __device__ void setup() const {
    init_tw<C::T>(twx, C::Lx);
    init_tw<C::T>(twz, C::Lz);
  }
};

template <class C>
constexpr size_t smem_bytes(int extra_floats) {
  return ((size_t)C::H * C::ST + C::Lx + C::Lz) * sizeof(float2) + (size_t)extra_floats * sizeof(float);
}

// Plane shape of the convolution kernels: read at run time (RunShape) or
// fixed at compile time for the common workloads (FixShape), so that the
// clamps of the replicate padding, the fold's loops and the plane loads work
// on constants.
struct RunShape {
  __device__ static int nx(const FftShape& s) { return s.nx; }
  __device__ static int nz(const FftShape& s) { return s.nz; }
  __device__ static int ha(const FftShape& s) { return s.ha; }
  __device__ static int hb(const FftShape& s) { return s.hb; }
};
template <int NX, int NZ, int HA, int HB>
struct FixShape {
  __device__ static constexpr int nx(const FftShape&) { return NX; }
  __device__ static constexpr int nz(const FftShape&) { return NZ; }
  __device__ static constexpr int ha(const FftShape&) { return HA; }
  __device__ static constexpr int hb(const FftShape&) { return HB; }
};

// ---------------------------------------------------------------- kernels
// kReal: the PSFs are symmetric in x and in z.  Their spectra are then taken
// of the PSF centred on the origin (tap (b, a) at ((b - hb) mod Lz,
// (a - ha) mod Lx)), which are real and even, and kept as one float per
// slot; the centring moves the kept bins of the forward from
// (k + 2 hb, i + 2 ha) to (k + hb, i + ha) and the adjoint's projection
// from (2 hb, 2 ha) to (hb, ha).  Otherwise complex spectra of the PSF at
// the corner.
template <bool kReal> using Spec = std::conditional_t<kReal, float, float2>;
__device__ __forceinline__ float2 spec_mul(float p, float2 a) { return cscale(a, p); }
__device__ __forceinline__ float2 spec_mul(float2 p, float2 a) { return cmul(p, a); }
// a * conj(p)
__device__ __forceinline__ float2 spec_mulc(float2 a, float p) { return cscale(a, p); }
__device__ __forceinline__ float2 spec_mulc(float2 a, float2 p) { return cmulc(a, p); }

template <class C, bool kReal>
__global__ __launch_bounds__(C::T) void psf_spectra_c(const float* __restrict__ psf,
                                                    Spec<kReal>* __restrict__ P, FftShape s) {
  extern __shared__ float2 sm2[];
  const Lds<C> m(sm2);
  const int jl = blockIdx.x;
  const float* p = psf + (size_t)jl * s.pz * s.px;
  m.setup();
  // tap row (column) of plane row q (column c): q itself, or (q + hb) mod Lz centred
  auto tap = [](int q, int h, int L) { return kReal ? (q + h < L ? q + h : q + h - L) : q; };
  for (int e = threadIdx.x; e < C::H * C::Lx; e += C::T) {
    const int r = e / C::Lx, c = e - r * C::Lx;
    const int a = tap(c, s.ha, C::Lx), b1 = tap(r, s.hb, C::Lz), b2 = tap(r + C::H, s.hb, C::Lz);
    const float lo = (b1 < s.pz && a < s.px) ? p[b1 * s.px + a] : 0.0f;
    const float hi = (b2 < s.pz && a < s.px) ? p[b2 * s.px + a] : 0.0f;
    m.A[r * C::ST + c] = make_float2(lo, hi);
  }
  __syncthreads();
  fft2_fwd<C>(m.A, m.twx, m.twz, [] {});
  const float scale = 1.0f / ((float)C::Lx * (float)C::Lz);
  if constexpr (kReal) store_slots_real<C>(m.A, P + (size_t)jl * C::NS, scale);
  else store_slots<C>(m.A, P + (size_t)jl * C::NS, scale);
}

template <class C, bool kReal, class SH>
__global__ __launch_bounds__(C::T) void conv_fwd_fft_c(const float* __restrict__ W,
                                                     const Spec<kReal>* __restrict__ P,
                                                     float2* __restrict__ part, FftShape s,
                                                     int view0, int nvb) {
  extern __shared__ float2 sm2[];
  const Lds<C> m(sm2);
  const int c = blockIdx.x % s.nchunk, lb = blockIdx.x / s.nchunk, l = view0 + lb;
  int j0, j1;
  chunk_range(c, s.nchunk, s.ny, j0, j1);
  m.setup();
  const int tid = threadIdx.x, nx = SH::nx(s), nz = SH::nz(s), plane = nz * nx;
  const int ha = SH::ha(s), hb = SH::hb(s);
  const size_t rs = (size_t)s.ny * nx;
  const float* Wl = W + (size_t)lb * nz * rs;
  const float rnx = 1.0f / (float)nx;
  float2 acc[C::KS], a0 = make_float2(0.f, 0.f), an = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < C::KS; ++q) acc[q] = make_float2(0.f, 0.f);
  const int rrs = raw_stride(nx);
  // plane j of W straight into the raw LDS region (lane L of a wave writes
  // the wave's base + 4 L bytes: 64 consecutive elements of the [nz][nx] plane)
  // nx a multiple of 64: every wave keeps one 64-element segment of a row
  // (nx / 64 divides the wave count, which fits() checks) and walks its rows
  // with uniform pointer steps, rows rrs floats apart in LDS; otherwise the
  // plane is packed and each lane finds its element
  const int segs = nx >> 6, nwv = C::T / 64;
  const bool walk = nx % 64 == 0;
  auto load_plane = [&](int j) {
    const int lane = tid & 63, wbase = tid - lane;
    if (walk) {
      const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
      const int seg = wv % segs, k0 = wv / segs, kstep = nwv / segs;
      const float* g = Wl + (size_t)k0 * rs + (size_t)j * nx + seg * 64 + lane;
      float* l = m.extra + k0 * rrs + seg * 64;
      const size_t gstep = (size_t)kstep * rs;
      const int lstep = kstep * rrs;
      for (int k = k0; k < nz; k += kstep, g += gstep, l += lstep)
        __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)l, 4, 0, 0);
    } else {
      for (int e0 = wbase; e0 < plane; e0 += C::T) {
        const int e = e0 + lane;
        if (e < plane) {
          const int k = fdiv(e, rnx), i = e - k * nx;
          __builtin_amdgcn_global_load_lds(Wl + (size_t)k * rs + (size_t)j * nx + i,
                                           (__attribute__((address_space(3))) void*)(m.extra + e0),
                                           4, 0, 0);
        }
      }
    }
  };
  if (j0 < j1) load_plane(j0);
  for (int j = j0; j < j1; ++j) {
    const Spec<kReal>* Pj = P + ((size_t)l * s.ny + j) * C::NS;
    Spec<kReal> pr[C::KS], p0 = Spec<kReal>{}, pn = Spec<kReal>{};
    auto load_p = [&] {
#pragma unroll
      for (int q = 0; q < C::KS; ++q) {
        const int sl = tid + q * C::T;
        if (sl < C::NR) pr[q] = Pj[sl];
      }
      if (tid <= C::H) {
        p0 = Pj[C::NR + 2 * tid];
        pn = Pj[C::NR + 2 * tid + 1];
      }
    };
    __builtin_amdgcn_s_waitcnt(0);                 // this plane's loads into raw landed
    __syncthreads();                               // raw complete, A free, twiddles ready
    xpass_first_from_raw<C>(m.A, m.twx, m.extra, rrs, nx, nz, ha, hb);  // ends with a barrier
    if (j + 1 < j1) load_plane(j + 1);             // raw consumed
    fft2_fwd_rest<C>(m.A, m.twz, load_p);
#pragma unroll
    for (int q = 0; q < C::KS; ++q) {
      const int sl = tid + q * C::T;
      if (sl < C::NR) {
        const float2 f = m.A[C::slot(sl)];
        if constexpr (kReal) {
          acc[q].x += pr[q] * f.x;
          acc[q].y += pr[q] * f.y;
        } else {
          acc[q].x += pr[q].x * f.x - pr[q].y * f.y;
          acc[q].y += pr[q].x * f.y + pr[q].y * f.x;
        }
      }
    }
    if (tid <= C::H) {
      float2 x0, xn;
      unpack_col0<C>(m.A, tid, &x0, &xn);
      a0 = cadd(a0, spec_mul(p0, x0));
      an = cadd(an, spec_mul(pn, xn));
    }
  }
  float2* out = part + ((size_t)c * nvb + lb) * C::NS;
#pragma unroll
  for (int q = 0; q < C::KS; ++q) {
    const int sl = tid + q * C::T;
    if (sl < C::NR) out[sl] = acc[q];
  }
  if (tid <= C::H) {
    out[C::NR + 2 * tid] = a0;
    out[C::NR + 2 * tid + 1] = an;
  }
}

template <class C, bool kReal>
__global__ __launch_bounds__(C::T) void fwd_fft_finish_c(const float2* __restrict__ part,
                                                       float* __restrict__ v, FftShape s,
                                                       int view0, int nvb) {
  extern __shared__ float2 sm2[];
  const Lds<C> m(sm2);
  const int lb = blockIdx.x, l = view0 + lb, tid = threadIdx.x;
  m.setup();
  for (int q = tid; q < C::NR; q += C::T) {
    float2 a = make_float2(0.f, 0.f);
    for (int c = 0; c < s.nchunk; ++c) a = cadd(a, part[((size_t)c * nvb + lb) * C::NS + q]);
    m.A[C::slot(q)] = a;
  }
  for (int zq = tid; zq <= C::H; zq += C::T) {
    float2 a0 = make_float2(0.f, 0.f), an = make_float2(0.f, 0.f);
    for (int c = 0; c < s.nchunk; ++c) {
      const float2* src = part + ((size_t)c * nvb + lb) * C::NS + C::NR + 2 * zq;
      a0 = cadd(a0, src[0]);
      an = cadd(an, src[1]);
    }
    pack_col0<C>(m.A, zq, a0, an);
  }
  __syncthreads();
  fft2_inv<C>(m.A, m.twx, m.twz);
  const float rnx = 1.0f / (float)s.nx;
  for (int e = tid; e < s.nz * s.nx; e += C::T) {
    const int k = fdiv(e, rnx), i = e - k * s.nx;
    v[((size_t)l * s.nz + k) * s.nx + i] =
        plane_at<C>(m.A, k + (kReal ? 1 : 2) * s.hb, i + (kReal ? 1 : 2) * s.ha);
  }
}

template <class C, bool kReal>
__global__ __launch_bounds__(C::T) void back_fft_prep_c(const float* __restrict__ v,
                                                      float2* __restrict__ V, FftShape s,
                                                      int view0) {
  extern __shared__ float2 sm2[];
  const Lds<C> m(sm2);
  const int lb = blockIdx.x, l = view0 + lb;
  m.setup();
  const float* vl = v + (size_t)l * s.nz * s.nx;
  for (int e = threadIdx.x; e < C::H * C::Lx; e += C::T) {
    const int r = e / C::Lx, cc = e - r * C::Lx;
    const int oa = (kReal ? 1 : 2) * s.ha, ob = (kReal ? 1 : 2) * s.hb;
    const int i = cc - oa, k1 = r - ob, k2 = r + C::H - ob;
    const bool in_i = i >= 0 && i < s.nx;
    const float lo = (in_i && k1 >= 0 && k1 < s.nz) ? vl[k1 * s.nx + i] : 0.0f;
    const float hi = (in_i && k2 >= 0 && k2 < s.nz) ? vl[k2 * s.nx + i] : 0.0f;
    m.A[r * C::ST + cc] = make_float2(lo, hi);
  }
  __syncthreads();
  fft2_fwd<C>(m.A, m.twx, m.twz, [] {});
  store_slots<C>(m.A, V + (size_t)lb * C::NS, 1.0f);
}

template <class C, bool kReal, class SH>
__global__ __launch_bounds__(C::T) void conv_back_fft_c(const float2* __restrict__ V,
                                                      const Spec<kReal>* __restrict__ P,
                                                      float* __restrict__ U, FftShape s, int view0,
                                                      int nvb) {
  extern __shared__ float2 sm2[];
  const Lds<C> m(sm2);
  const int c = blockIdx.x % s.nchunk_back, lb = blockIdx.x / s.nchunk_back, l = view0 + lb;
  int j0, j1;
  chunk_range(c, s.nchunk_back, s.ny, j0, j1);
  m.setup();
  const int tid = threadIdx.x, nx = SH::nx(s), nz = SH::nz(s);
  // the PSF spectrum of the next plane is loaded into registers during this
  // plane's transform; the view's projection spectrum (86 KB at 180 x 120)
  // is read per plane, from L2 after the first
  const float2* Vl = V + (size_t)lb * C::NS;
  float2 v0 = make_float2(0.f, 0.f), vn = make_float2(0.f, 0.f);
  if (tid <= C::H) {
    v0 = Vl[C::NR + 2 * tid];
    vn = Vl[C::NR + 2 * tid + 1];
  }
  const size_t rs = (size_t)s.ny * nx;
  float* Ul = U + (size_t)lb * nz * rs;
  Spec<kReal> pr[C::KS], p0 = Spec<kReal>{}, pn = Spec<kReal>{};
  auto load_p = [&](int j) {
    const Spec<kReal>* Pj = P + ((size_t)l * s.ny + j) * C::NS;
#pragma unroll
    for (int q = 0; q < C::KS; ++q) {
      const int sl = tid + q * C::T;
      if (sl < C::NR) pr[q] = Pj[sl];
    }
    if (tid <= C::H) {
      p0 = Pj[C::NR + 2 * tid];
      pn = Pj[C::NR + 2 * tid + 1];
    }
  };
  if (j0 < j1) load_p(j0);
  for (int j = j0; j < j1; ++j) {
    __syncthreads();                               // A and the folded plane free
#pragma unroll
    for (int q = 0; q < C::KS; ++q) {
      const int sl = tid + q * C::T;
      if (sl < C::NR) m.A[C::slot(sl)] = spec_mulc(Vl[sl], pr[q]);
    }
    if (tid <= C::H) pack_col0<C>(m.A, tid, spec_mulc(v0, p0), spec_mulc(vn, pn));
    __syncthreads();
    if (j + 1 < j1) load_p(j + 1);                 // the next plane's spectrum, during this one
    fft2_inv<C>(m.A, m.twx, m.twz);
    fold_store(m.A, m.extra, nx, nz, SH::ha(s), SH::hb(s), Ul + (size_t)j * nx, rs,
               [](const float2* A, int k, int c) { return plane_at<C>(A, k, c); }, C::T);
  }
}

hipError_t set_smem(const void* fn, size_t sm) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
}

// The plane shapes compiled in: 128 x 80 with 37 x 37 PSFs on the 180 x 120
// transforms, 64 x 40 with 19 x 19 PSFs on the 90 x 60 ones; others at run time.
template <class C, class F>
hipError_t with_plane_shape(const FftShape& s, F&& f) {
  if constexpr (C::Lx == 180 && C::Lz == 120) {
    if (s.nx == 128 && s.nz == 80 && s.ha == 18 && s.hb == 18) return f(FixShape<128, 80, 18, 18>());
  } else if constexpr (C::Lx == 90 && C::Lz == 60) {
    if (s.nx == 64 && s.nz == 40 && s.ha == 9 && s.hb == 9) return f(FixShape<64, 40, 9, 9>());
  }
  return f(RunShape());
}

template <template <int> class CF, bool kReal>
hipError_t launch_cr(const Plan& p, int which, const void* in, void* out, int view0, int nvb,
                     hipStream_t st) {
  using CW = CF<1024>;   // transforms of one plane per workgroup pass
  using CFW = CF<kFwdThreads>;   // forward convolution
  using CB = CF<768>;    // adjoint
  const FftShape& s = p.fft;
  char* ws = p.ws;
  Spec<kReal>* P = reinterpret_cast<Spec<kReal>*>(ws + p.lay.fft_spectra);
  float2* part = reinterpret_cast<float2*>(ws + p.lay.fft_part);
  float2* V = reinterpret_cast<float2*>(ws + p.lay.fft_vproj);
  hipError_t e = hipSuccess;
  switch (which) {
    case kFftSpectra: {
      const size_t sm = smem_bytes<CW>(0);
      if ((e = set_smem((const void*)psf_spectra_c<CW, kReal>, sm)) != hipSuccess) return e;
      hipLaunchKernelGGL((psf_spectra_c<CW, kReal>), dim3((unsigned)(p.g.nview * p.g.ny)),
                         dim3(CW::T), sm, st, p.psf, P, s);
      break;
    }
    case kFftForward: {
      const size_t sm = smem_bytes<CFW>(s.nz * raw_stride(s.nx));
      return with_plane_shape<CFW>(s, [&](auto sh) {
        using SH = decltype(sh);
        hipError_t r = set_smem((const void*)conv_fwd_fft_c<CFW, kReal, SH>, sm);
        if (r != hipSuccess) return r;
        hipLaunchKernelGGL((conv_fwd_fft_c<CFW, kReal, SH>), dim3((unsigned)(nvb * s.nchunk)),
                           dim3(CFW::T), sm, st, static_cast<const float*>(in), P, part, s, view0,
                           nvb);
        return hipGetLastError();
      });
    }
    case kFftFinish: {
      const size_t sm = smem_bytes<CW>(0);
      if ((e = set_smem((const void*)fwd_fft_finish_c<CW, kReal>, sm)) != hipSuccess) return e;
      hipLaunchKernelGGL((fwd_fft_finish_c<CW, kReal>), dim3((unsigned)nvb), dim3(CW::T), sm, st,
                         part, static_cast<float*>(out), s, view0, nvb);
      break;
    }
    case kFftBackPrep: {
      const size_t sm = smem_bytes<CW>(0);
      if ((e = set_smem((const void*)back_fft_prep_c<CW, kReal>, sm)) != hipSuccess) return e;
      hipLaunchKernelGGL((back_fft_prep_c<CW, kReal>), dim3((unsigned)nvb), dim3(CW::T), sm, st,
                         static_cast<const float*>(in), V, s, view0);
      break;
    }
    case kFftBack: {
      const size_t sm = smem_bytes<CB>((s.nz + 2 * s.hb) * s.nx);
      return with_plane_shape<CB>(s, [&](auto sh) {
        using SH = decltype(sh);
        hipError_t r = set_smem((const void*)conv_back_fft_c<CB, kReal, SH>, sm);
        if (r != hipSuccess) return r;
        hipLaunchKernelGGL((conv_back_fft_c<CB, kReal, SH>), dim3((unsigned)(nvb * s.nchunk_back)),
                           dim3(CB::T), sm, st, V, P, static_cast<float*>(out), s, view0, nvb);
        return hipGetLastError();
      });
    }
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <template <int> class CF>
hipError_t launch_c(const Plan& p, int which, const void* in, void* out, int view0, int nvb,
                    hipStream_t st) {
  return p.fft.real ? launch_cr<CF, true>(p, which, in, out, view0, nvb, st)
                    : launch_cr<CF, false>(p, which, in, out, view0, nvb, st);
}

template <class C>
bool fits(const FftShape& s) {
  return s.Lx == C::Lx && s.Lz == C::Lz && s.nz * s.nx <= 16384 &&
         (s.nx % 64 != 0 || (kFwdThreads / 64) % (s.nx / 64) == 0) &&
         smem_bytes<C>(s.nz * raw_stride(s.nx)) <= kLdsBytes &&
         smem_bytes<C>((s.nz + 2 * s.hb) * s.nx) <= kLdsBytes;
}

}  // namespace

int fft_fixed_config(const FftShape& s) {
  if (fits<Cfg180x120<512>>(s)) return 1;
  if (fits<Cfg90x60<512>>(s)) return 2;
  return 0;
}

hipError_t launch_fft_fixed(const Plan& p, int which, const void* in, void* out, int view0, int nvb,
                            hipStream_t st) {
  switch (p.fft.cfg) {
    case 1: return launch_c<Cfg180x120>(p, which, in, out, view0, nvb, st);
    case 2: return launch_c<Cfg90x60>(p, which, in, out, view0, nvb, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace spect
