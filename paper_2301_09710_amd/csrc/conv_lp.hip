// PSF convolution as BF16 / FP16 matrix-core contractions with FP32
// accumulation (v_mfma_f32_16x16x32_{bf16,f16}): the reduced-precision form of
// the replicate-padded convolution and its adjoint (Sec. II-A, Alg. 1 and 2).
// Rotation, attenuation, the depth-sum reduction and the edge fold of the
// adjoint stay FP32; the inputs of the contraction (the weighted planes or
// the projection, and the PSF) are rounded to nearest-even at staging.
//
// Mapping (one M-block of 16 output z positions per wave, NN N-blocks of 16
// output x positions per wave, the whole x range of a tile in one wave):
//   C[m][n] += sum_r A[m][r] B[r][n]   for every x-tap a, with
//   forward  A[m][r] = p[a][m - r + 2hb],  B[r][n] = R[16 w + r][16 u + n - a + 2ha]
//   adjoint  A[m][r] = p[a][r - m],        B[r][n] = R[16 w + r][16 u + n + a]
// where r runs over the 16 + pz - 1 region rows of the M-block's band.  The
// K dimension of one MFMA (32) is four lanes groups of 8 consecutive rows;
// each group takes its own (tap, 8-row chunk) pair from the flattened list of
// px * C7 chunks (C7 = ceil((15 + pz) / 8)), so k-steps do not end at tap
// boundaries and only the 8-row rounding of the band is wasted
// (8 C7 / pz = 1.51x for pz = 37, against 64 / 37 for whole-tap k-steps).
//
// Operands come from LDS:
//   B: the region is staged transposed (z contiguous, column stride RS =
//      8 (mod 16) elements), so a lane's 8 rows are one aligned 16-byte read
//      and eight consecutive columns cover all banks;
//   A: each PSF row is stored reversed (forward) or shifted (adjoint) as
//      overlapping element pairs, one 32-bit word per position, so the 8
//      values a lane needs from an arbitrary start are four word reads.
// A is shared by the NN N-blocks of a k-step.
#include "internal.h"

namespace spect {

hipError_t lp_launch_fwd_bf16(const LpShape&, const float*, const float*, float*, int, int, hipStream_t);
hipError_t lp_launch_back_bf16(const LpShape&, const float*, const float*, float*, int, int, hipStream_t);
int lp_occupancy_bf16(const LpShape&, bool);
hipError_t lp_launch_fwd_fp16(const LpShape&, const float*, const float*, float*, int, int, hipStream_t);
hipError_t lp_launch_back_fp16(const LpShape&, const float*, const float*, float*, int, int, hipStream_t);
int lp_occupancy_fp16(const LpShape&, bool);
hipError_t lp_launch_fwd_bf16x3(const LpShape&, const float*, const float*, float*, int, int, hipStream_t);
hipError_t lp_launch_back_bf16x3(const LpShape&, const float*, const float*, float*, int, int, hipStream_t);
int lp_occupancy_bf16x3(const LpShape&, bool);

namespace {
// Depth chunks per (tile, view): minimise rounds * planes per workgroup.
int lp_pick_chunks(int ny, long long tiles_views, long long slots) {
  int best = 1;
  long long best_cost = -1;
  for (int c = 1; c <= kMaxChunks && c <= ny; ++c) {
    const long long rounds = (tiles_views * c + slots - 1) / slots;
    const long long cost = rounds * ((ny + c - 1) / c);
    if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = c; }
  }
  return best;
}

}  // namespace

static int odd8_stride(int rows) {      // >= rows, multiple of 8, odd multiple of 8
  int s = (rows + 7) / 8;
  if (s % 2 == 0) ++s;
  return 8 * s;
}

LpShape make_lp_shape(const spect_geom& g) {
  LpShape s;
  s.nx = g.nx; s.ny = g.ny; s.nz = g.nz; s.px = g.px; s.pz = g.pz;
  s.ha = (g.px - 1) / 2; s.hb = (g.pz - 1) / 2;
  const int nmb = (g.nz + 15) / 16;
  s.tiles_k = (nmb + kLpMaxWaves - 1) / kLpMaxWaves;
  s.WKm = (nmb + s.tiles_k - 1) / s.tiles_k;        // M-blocks per workgroup tile
  const int nwv = (g.nx + 31) / 32;
  s.NN = nwv < 4 ? nwv : 4;                          // waves per workgroup, 32 x bins each
  s.tiles_i = (nwv + s.NN - 1) / s.NN;
  s.C7 = (15 + g.pz + 7) / 8;
  s.ntq = (g.px + 3) / 4;
  s.NR = 2 * (s.WKm - 1) + s.C7;
  s.RR = 16 * (s.WKm - 1) + 8 * s.C7;
  s.RS = odd8_stride(s.RR);
  s.RC = 32 * s.NN + g.px - 1;
  s.dx = (4 - s.ha % 4) % 4;                         // region origin i0 - ha - dx is 4-aligned
  s.RCa = (s.RC + s.dx + 3) / 4 * 4;
  s.QL = 8 * s.C7 + 15;
  s.nchunk = 1;
  s.nchunk_back = 1;
  return s;
}

size_t lp_lds_bytes(const LpShape& s, bool split) {
  // region and PSF pair table; the split form holds leading parts and remainders
  return (split ? 2 : 1) * ((size_t)s.RCa * s.RS * 2 + (size_t)(s.px + 1) * s.QL * 4);
}

bool lp_supported(const spect_geom& g) {
  const LpShape s = make_lp_shape(g);
  return s.C7 >= 2 && s.C7 <= 8 &&
         lp_lds_bytes(s, g.conv_precision == SPECT_CONV_BF16X3) <= kLdsBytes;
}

void tune_lp_chunks(LpShape& s, int views, int precision) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    return;
  int fw, bw;
  if (precision == SPECT_CONV_FP16) {
    fw = lp_occupancy_fp16(s, false);
    bw = lp_occupancy_fp16(s, true);
  } else if (precision == SPECT_CONV_BF16X3) {
    fw = lp_occupancy_bf16x3(s, false);
    bw = lp_occupancy_bf16x3(s, true);
  } else {
    fw = lp_occupancy_bf16(s, false);
    bw = lp_occupancy_bf16(s, true);
  }
  const long long tv = (long long)s.tiles_k * s.tiles_i * views;
  s.nchunk = lp_pick_chunks(s.ny, tv, (long long)cus * fw);
  s.nchunk_back = lp_pick_chunks(s.ny, tv, (long long)cus * bw);
}

hipError_t launch_conv_fwd_lp(const Plan& p, const float* W, float* partial, int view0, int nvb,
                              hipStream_t st) {
  switch (p.conv_precision) {
    case SPECT_CONV_FP16: return lp_launch_fwd_fp16(p.lp, W, p.psf, partial, view0, nvb, st);
    case SPECT_CONV_BF16X3: return lp_launch_fwd_bf16x3(p.lp, W, p.psf, partial, view0, nvb, st);
    default: return lp_launch_fwd_bf16(p.lp, W, p.psf, partial, view0, nvb, st);
  }
}

hipError_t launch_conv_back_lp(const Plan& p, const float* v, float* U, int view0, int nvb,
                               hipStream_t st) {
  switch (p.conv_precision) {
    case SPECT_CONV_FP16: return lp_launch_back_fp16(p.lp, v, p.psf, U, view0, nvb, st);
    case SPECT_CONV_BF16X3: return lp_launch_back_bf16x3(p.lp, v, p.psf, U, view0, nvb, st);
    default: return lp_launch_back_bf16(p.lp, v, p.psf, U, view0, nvb, st);
  }
}

}  // namespace spect
