"""FP64 CPU oracle for the rotation-based SPECT projector pair.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library: it computes its own angle split, shear parameters, attenuation,
convolution and transposes from the paper's definitions, in float64, as plain
and slow as is still practical.

Paper: Z. Li, Y. K. Dewaraja, J. A. Fessler, "Training End-to-End Unrolled
Iterative Neural Networks for SPECT Image Reconstruction".

Modules
  geometry    view angles, quarter-turn / residual split, shear parameters
              (Sec. II-A, rotation by theta_l with 3-pass 1-D interpolation)
  rotation    exact quarter turns, gather shears, rotation and its transpose
  attenuation accumulated attenuation factor, Eq. (1)
  convolution replicate-padded 2-D convolution, its transpose, FFT form
  projector   forward projector (Alg. 1), back projector (Alg. 2 / Eq. (2))
  em          Poisson model and EM updates, Eq. (3)-(4), (7)-(8), and their
              reverse-mode derivatives (unrolled EM, Sec. II-B)
  precision   rounding to BF16 / FP16 for the reduced-precision convolution
  dense       explicit system matrices for tiny problems (Sec. III-A-3)

Index conventions: arrays come in the C-ABI storage layout
(volumes [nz][ny][nx], projections [nview][nz][nx], PSFs
[nview][ny][pz][px]); internally the code uses the paper's x[i, j, k] order
(i along x, j along y = depth, k along z).  Indices are 0-based, so the
paper's plane j = ny (nearest the detector) is j = ny-1 here.

Readings of the paper where it is silent (all shared with the GPU path as
conventions, not code): rotation centre c = (n-1)/2; gather
out(p) = in(R(theta)^-1 (p - c) + c); theta = M*pi/2 + phi with
M = floor(theta/(pi/2) + 1/2), phi in [-pi/4, pi/4); quarter turn first, then
the shears X(tan(phi/2)) Y(-sin phi) X(tan(phi/2)); zero outside the grid for
interpolation; replicate padding of width (p-1)/2 for odd kernels.
"""
from . import geometry, rotation, attenuation, convolution, projector, em, dense, precision  # noqa: F401
from .projector import forward, back, Geometry  # noqa: F401
