// Split-BF16 (three products per FP32 product) instantiations of the reduced-precision PSF convolution.
#include "conv_lp_impl.h"

namespace spect {

hipError_t lp_launch_fwd_bf16x3(const LpShape& s, const float* W, const float* psf, float* partial,
                              int view0, int nvb, hipStream_t st) {
  return launch_fwd_t<__bf16, true>(s, W, psf, partial, view0, nvb, st);
}

hipError_t lp_launch_back_bf16x3(const LpShape& s, const float* v, const float* psf, float* U,
                               int view0, int nvb, hipStream_t st) {
  return launch_back_t<__bf16, true>(s, v, psf, U, view0, nvb, st);
}

int lp_occupancy_bf16x3(const LpShape& s, bool back) { return lp_wgs_per_cu<__bf16, true>(s, back); }

}  // namespace spect
