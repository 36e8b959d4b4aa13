// Building blocks of the FFT convolution kernels (conv_fft.hip,
// conv_fft_fixed.hip): complex arithmetic, R-point DFTs in registers for
// R = 2, 3, 4, 5 and the composites 6, 8, 9, 10, 12, 15, and the stage
// twiddles of one in-place pass.  The arithmetic helpers are host-callable
// too, so that the DFTs can be checked on the CPU.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace spect {
namespace fft {

// q / d and q mod d for 0 <= q < 2^16 and 1 <= d < 2^16 through the FP32
// reciprocal rd = 1 / d: (q + 1/2) / d lies at least 1 / (2 d) from an
// integer, and the rounding error of (q + 1/2) rd is below 2^-22 (q + 1/2) / d,
// far less.
__device__ __forceinline__ int fdiv(int q, float rd) { return (int)(((float)q + 0.5f) * rd); }

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__host__ __device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// i s a
__host__ __device__ __forceinline__ float2 cimul(float2 a, float s) { return make_float2(-s * a.y, s * a.x); }
__host__ __device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// R-point DFT in place, X[m] = sum_r v[r] exp(sg 2 pi i r m / R), sg = -1
// (forward) or +1 (inverse).
template <int R, bool kInv>
__host__ __device__ __forceinline__ void dft(float2 (&v)[R]) {
  constexpr float sg = kInv ? 1.0f : -1.0f;
  if constexpr (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const float h = 0.86602540378443864676f;   // sin(2 pi / 3)
    const float2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const float2 t = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
    const float2 u = cimul(d, sg * h);
    v[0] = cadd(v[0], s);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
  } else if constexpr (R == 4) {
    const float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const float2 c = cadd(v[1], v[3]), d = cimul(csub(v[1], v[3]), sg);
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  } else {
    static_assert(R == 5, "radix 2, 3, 4 or 5");
    const float c1 = 0.30901699437494742410f;    // cos(2 pi / 5)
    const float c2 = -0.80901699437494742410f;   // cos(4 pi / 5)
    const float s1 = 0.95105651629515357212f;    // sin(2 pi / 5)
    const float s2 = 0.58778525229247312917f;    // sin(4 pi / 5)
    const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const float2 x0 = v[0];
    const float2 r1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    const float2 r2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    const float2 i1 = cimul(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y), sg);
    const float2 i2 = cimul(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y), sg);
    v[0] = cadd(x0, cadd(a1, a2));
    v[1] = cadd(r1, i1);
    v[4] = csub(r1, i1);
    v[2] = cadd(r2, i2);
    v[3] = csub(r2, i2);
  }
}

// Index tables of one plan's transforms (in LDS):
//   posx[f], posz[q]: where frequency f (q) of a transform along x (z) sits
//     after the in-place decimation-in-frequency passes (mixed-radix digit
//     reversal);
//   vc1[v], vc2[v]: the columns of virtual column v (x frequency f < Lx/2) in
//     the first and the second half of the row pairs, in increasing vc1; v = 0
//     is frequency 0 (with Lx/2 in the second half: the two real columns).
struct Tabs {
  const int* posx;
  const int* posz;
  const int* vc1;
  const int* vc2;
};

// Twiddle constants of the composite radices, evaluated at compile time
// (Taylor series in FP64 on [-pi, pi]).
constexpr double kTwoPi = 6.28318530717958647692528676655900577;
constexpr double csin(double x) {
  while (x > kTwoPi / 2) x -= kTwoPi;
  while (x < -kTwoPi / 2) x += kTwoPi;
  double term = x, sum = x;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double ccos(double x) { return csin(x + kTwoPi / 4); }

template <class F, int... I>
__host__ __device__ __forceinline__ void unroll_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>()), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void unroll(F&& f) {
  unroll_seq(f, std::make_integer_sequence<int, N>());
}

// Factors of the composite radices: R = Ra Rb.
template <int R> struct Split;
template <> struct Split<6> { static constexpr int a = 2, b = 3; };
template <> struct Split<8> { static constexpr int a = 2, b = 4; };
template <> struct Split<9> { static constexpr int a = 3, b = 3; };
template <> struct Split<10> { static constexpr int a = 2, b = 5; };
template <> struct Split<12> { static constexpr int a = 3, b = 4; };
template <> struct Split<15> { static constexpr int a = 3, b = 5; };

constexpr int gcd(int a, int b) { return b == 0 ? a : gcd(b, a % b); }
// a^-1 mod m for gcd(a, m) = 1 (0 when m = 1).
constexpr int modinv(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 0;
}

template <int R, bool kInv>
__host__ __device__ __forceinline__ void dft_any(float2 (&v)[R]);

// a exp(sg 2 pi i e / R) for a constant e, sg = -1 (forward) or +1 (inverse);
// multiples of a quarter turn are exact sign changes and swaps.
template <int e, int R, bool kInv>
__host__ __device__ __forceinline__ float2 crot(float2 a) {
  constexpr int q = e % R;
  constexpr float sg = kInv ? 1.0f : -1.0f;
  if constexpr (q == 0) {
    return a;
  } else if constexpr ((4 * q) % R == 0) {
    constexpr int quarter = 4 * q / R;             // the angle is sg quarter pi / 2
    if constexpr (quarter == 2) return make_float2(-a.x, -a.y);
    else return cimul(a, quarter == 1 ? sg : -sg);
  } else {
    constexpr float c = (float)ccos(kTwoPi * q / R);
    constexpr float sn = (float)csin((kInv ? 1.0 : -1.0) * kTwoPi * q / R);
    return cmul(a, make_float2(c, sn));
  }
}

// R-point DFT for R = Ra Rb in registers (Cooley-Tukey): input n = Rb n1 + n2,
// Ra-point DFTs over n1, twiddles exp(sg 2 pi i n2 k1 / R), Rb-point DFTs over
// n2, output k = k1 + Ra k2 (natural order).
template <int Ra, int Rb, bool kInv>
__host__ __device__ __forceinline__ void dft_comp(float2 (&v)[Ra * Rb]) {
  float2 y[Ra][Rb];
  unroll<Rb>([&](auto n2c) {
    constexpr int n2 = decltype(n2c)::value;
    float2 t[Ra];
    unroll<Ra>([&](auto n1c) { t[decltype(n1c)::value] = v[Rb * decltype(n1c)::value + n2]; });
    dft_any<Ra, kInv>(t);
    unroll<Ra>([&](auto k1c) {
      constexpr int k1 = decltype(k1c)::value;
      y[k1][n2] = crot<n2 * k1, Ra * Rb, kInv>(t[k1]);
    });
  });
  unroll<Ra>([&](auto k1c) {
    constexpr int k1 = decltype(k1c)::value;
    float2 t[Rb];
    unroll<Rb>([&](auto n2c) { t[decltype(n2c)::value] = y[k1][decltype(n2c)::value]; });
    dft_any<Rb, kInv>(t);
    unroll<Rb>([&](auto k2c) { v[k1 + Ra * decltype(k2c)::value] = t[decltype(k2c)::value]; });
  });
}

// R-point DFT for R = Ra Rb with coprime factors (Good-Thomas prime-factor
// algorithm): input n = (Rb n1 + Ra n2) mod R, Ra-point DFTs over n1,
// Rb-point DFTs over n2, output k = (Rb (Rb^-1 mod Ra) k1 + Ra (Ra^-1 mod Rb)
// k2) mod R.  exp(2 pi i n k / R) then factors into exp(2 pi i n1 k1 / Ra)
// exp(2 pi i n2 k2 / Rb): no twiddles between the two sets of DFTs.
template <int Ra, int Rb, bool kInv>
__host__ __device__ __forceinline__ void dft_pfa(float2 (&v)[Ra * Rb]) {
  constexpr int R = Ra * Rb;
  constexpr int ia = modinv(Rb % Ra, Ra), ib = modinv(Ra % Rb, Rb);
  float2 y[Ra][Rb];
  unroll<Rb>([&](auto n2c) {
    constexpr int n2 = decltype(n2c)::value;
    float2 t[Ra];
    unroll<Ra>([&](auto n1c) {
      constexpr int n1 = decltype(n1c)::value;
      t[n1] = v[(Rb * n1 + Ra * n2) % R];
    });
    dft_any<Ra, kInv>(t);
    unroll<Ra>([&](auto k1c) { y[decltype(k1c)::value][n2] = t[decltype(k1c)::value]; });
  });
  unroll<Ra>([&](auto k1c) {
    constexpr int k1 = decltype(k1c)::value;
    float2 t[Rb];
    unroll<Rb>([&](auto n2c) { t[decltype(n2c)::value] = y[k1][decltype(n2c)::value]; });
    dft_any<Rb, kInv>(t);
    unroll<Rb>([&](auto k2c) {
      constexpr int k2 = decltype(k2c)::value;
      v[(Rb * ia * k1 + Ra * ib * k2) % R] = t[k2];
    });
  });
}

template <int R, bool kInv>
__host__ __device__ __forceinline__ void dft_any(float2 (&v)[R]) {
  if constexpr (R <= 5) {
    dft<R, kInv>(v);
  } else {
    constexpr int a = Split<R>::a, b = Split<R>::b;
    if constexpr (gcd(a, b) == 1) dft_pfa<a, b, kInv>(v);
    else dft_comp<a, b, kInv>(v);
  }
}

// Element t of transform b: rows (b = row pair, along x) or virtual columns
// (b = virtual column, along z).
struct RowAddr {
  int stride;
  __device__ __forceinline__ int operator()(int b, int t) const { return b * stride + t; }
};
struct ColAddr {
  int stride, H;
  const int* vc1;
  const int* vc2;
  __device__ __forceinline__ int operator()(int b, int t) const {
    return t < H ? t * stride + vc1[b] : (t - H) * stride + vc2[b];
  }
};

// Stage twiddles w[r] = tw[r d] = exp(-2 pi i r d / N) for r < R (w[0] unused),
// read from the table (r d < N for every stage of a length-N transform).
template <int R>
__device__ __forceinline__ void stage_twiddles(float2 (&w)[R], const float2* tw, int d) {
#pragma unroll
  for (int r = 1; r < R; ++r) w[r] = tw[r * d];
}


// The adjoint of replicate padding on one inverse-transformed plane:
// u[k][i] = sum of the padded plane g over the padded rows that clamp onto k
// and the padded columns that clamp onto i, written to out[k * rs + i].
// Columns first (into `fold`, (nz + 2 hb) x nx floats), then rows.  Interior
// bins are copies: a thread keeps one column (lanes on consecutive columns)
// and steps over the rows, T / nx rows apart, so no index needs a division.
// The edge sums (ha + 1 or hb + 1 terms) run on lanes of their own so that
// no wave waits on one long sum.  Requires nx <= T.
template <class G>
__device__ __forceinline__ void fold_store(const float2* A, float* fold, int nx, int nz, int ha,
                                           int hb, float* out, size_t rs, G&& g, int T) {
  const int KZ = nz + 2 * hb;
  const int RG = T / nx, c = threadIdx.x % nx, r0 = threadIdx.x / nx;
  const bool mine = r0 < RG;                       // threads past RG * nx idle in the copies
  if (mine && c >= 1 && c < nx - 1)
    for (int zz = r0; zz < KZ; zz += RG) fold[zz * nx + c] = g(A, zz, c + ha);
  const int edges_x = nx > 1 ? 2 : 1;
  for (int e = threadIdx.x; e < KZ * edges_x; e += T) {
    const int zz = e / edges_x, side = e - zz * edges_x;
    const int i = side ? nx - 1 : 0;
    const int xl = side ? nx - 1 + ha : 0;
    const int xh = (side || nx == 1) ? nx - 1 + 2 * ha : ha;
    float a = 0.0f;
    for (int xx = xl; xx <= xh; ++xx) a += g(A, zz, xx);
    fold[zz * nx + i] = a;
  }
  __syncthreads();
  if (mine)
    for (int k = 1 + r0; k < nz - 1; k += RG) out[(size_t)k * rs + c] = fold[(k + hb) * nx + c];
  const int edges_z = nz > 1 ? 2 : 1;
  for (int e = threadIdx.x; e < edges_z * nx; e += T) {
    const int side = e / nx, i = e - side * nx;
    const int k = side ? nz - 1 : 0;
    const int zl = side ? nz - 1 + hb : 0;
    const int zh = (side || nz == 1) ? nz - 1 + 2 * hb : hb;
    float a = 0.0f;
    for (int zz = zl; zz <= zh; ++zz) a += fold[zz * nx + i];
    out[(size_t)k * rs + i] = a;
  }
}

}  // namespace fft
}  // namespace spect
