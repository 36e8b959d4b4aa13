// FP16 instantiations of the reduced-precision PSF convolution.
#include "conv_lp_impl.h"

namespace spect {

hipError_t lp_launch_fwd_fp16(const LpShape& s, const float* W, const float* psf, float* partial,
                              int view0, int nvb, hipStream_t st) {
  return launch_fwd_t<_Float16, false>(s, W, psf, partial, view0, nvb, st);
}

hipError_t lp_launch_back_fp16(const LpShape& s, const float* v, const float* psf, float* U,
                               int view0, int nvb, hipStream_t st) {
  return launch_back_t<_Float16, false>(s, v, psf, U, view0, nvb, st);
}

int lp_occupancy_fp16(const LpShape& s, bool back) { return lp_wgs_per_cu<_Float16, false>(s, back); }

}  // namespace spect
