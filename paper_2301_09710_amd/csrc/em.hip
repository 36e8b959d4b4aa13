// Element-wise EM kernels (Sec. II-B, Eq. (7)-(8) with beta -> 0) and the
// FP64 inner product used by adjoint checks.
#include "internal.h"

namespace spect {
namespace {

// rho = y / (v + r), 0 where the mean v + r <= 0.  rho may be v (the EM step
// overwrites its projection in place): each element is read before it is
// written by the same thread, so v and rho carry no __restrict__.
__global__ void em_ratio_kernel(const float* v, const float* __restrict__ y,
                                const float* __restrict__ r, float* rho, size_t m) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const float ybar = v[q] + (r ? r[q] : 0.0f);
  rho[q] = ybar > 0.0f ? y[q] / ybar : 0.0f;
}

// x <- x * e / sens, 0 where sens <= 0.
__global__ void em_update_kernel(float* __restrict__ x, const float* __restrict__ e,
                                 const float* __restrict__ sens, size_t n) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float s = sens[q];
  x[q] = s > 0.0f ? x[q] * e[q] / s : 0.0f;
}

// Regularised update of Eq. (7)-(8): the root of beta x^2 + d x - x_k e = 0
// with d = sens - beta u, evaluated as 2 x_k e / (d + sqrt(d^2 + 4 beta x_k e))
// when d > 0 (no cancellation) and as (-d + sqrt(...)) / (2 beta) otherwise;
// beta = 0 is the ML-EM update (0 where sens <= 0).
__global__ void em_reg_update_kernel(float* __restrict__ x, const float* __restrict__ e,
                                     const float* __restrict__ sens, const float* __restrict__ u,
                                     float beta, size_t n) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float xe = x[q] * e[q];
  const float d = sens[q] - beta * u[q];
  if (beta == 0.0f) {
    x[q] = d > 0.0f ? xe / d : 0.0f;
    return;
  }
  const float root = sqrtf(fmaf(d, d, 4.0f * beta * xe));
  x[q] = d > 0.0f ? 2.0f * xe / (d + root) : (root - d) / (2.0f * beta);
}

// Vector-Jacobian product of one EM update x+ = x * A'(y / (A x + r)) / s
// (Eq. (7)-(8), beta -> 0), with g = dL/dx+ and b = A'rho:
//   dL/dx = g b / s + A'(gq),   gq = -(t / q)(y / q),   t = A (g x / s),
//   dL/dy = t / q,              q = A x + r,
// where the guarded branches (s <= 0, q <= 0) are constants and pass no
// gradient.  The projections t and A'(gq) run on the projector kernels; the
// steps below are the element-wise parts.

// gb = g x / s and gx = g b / s (0 where s <= 0).  gx may be g (the C ABI
// allows the gradient to be updated in place), so those two are not
// __restrict__; each element of g is read before gx is written.
__global__ void em_vjp_prep_kernel(const float* g, const float* __restrict__ x,
                                   const float* __restrict__ b, const float* __restrict__ sens,
                                   float* __restrict__ gb, float* gx, size_t n) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float s = sens[q];
  const float gq = g[q];
  const bool ok = s > 0.0f;
  gb[q] = ok ? gq * x[q] / s : 0.0f;
  gx[q] = ok ? gq * b[q] / s : 0.0f;
}

// From t = A gb and the mean q = v + r: gy = t / q and gq = -(t / q)(y / q),
// both 0 where q <= 0; gq overwrites t.
__global__ void em_vjp_ratio_kernel(float* __restrict__ t, const float* __restrict__ v,
                                    const float* __restrict__ y, const float* __restrict__ r,
                                    float* __restrict__ gy, size_t m) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const float ybar = v[q] + (r ? r[q] : 0.0f);
  const bool ok = ybar > 0.0f;
  const float tq = ok ? t[q] / ybar : 0.0f;
  if (gy) gy[q] = tq;
  t[q] = ok ? -tq * (y[q] / ybar) : 0.0f;
}

// a += b
__global__ void add_kernel(float* __restrict__ a, const float* __restrict__ b, size_t n) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  a[q] += b[q];
}

constexpr int kDotThreads = 1024;

// Single workgroup, fixed order: thread t sums elements t, t+T, ... in FP64,
// then a tree reduction in LDS.  Deterministic for a given n.
__global__ __launch_bounds__(kDotThreads) void dot_f64_kernel(const float* __restrict__ a,
                                                              const float* __restrict__ b,
                                                              size_t n, double* __restrict__ out) {
  __shared__ double red[kDotThreads];
  double s = 0.0;
  for (size_t q = threadIdx.x; q < n; q += kDotThreads) s += (double)a[q] * (double)b[q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

hipError_t launch_em_ratio(const float* v, const float* y, const float* r, float* rho, size_t m,
                           hipStream_t s) {
  hipLaunchKernelGGL(em_ratio_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, v, y, r,
                     rho, m);
  return hipGetLastError();
}

hipError_t launch_em_update(float* x, const float* e, const float* sens, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(em_update_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, e,
                     sens, n);
  return hipGetLastError();
}

hipError_t launch_em_vjp_prep(const float* g, const float* x, const float* b, const float* sens,
                              float* gb, float* gx, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(em_vjp_prep_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, x, b,
                     sens, gb, gx, n);
  return hipGetLastError();
}

hipError_t launch_em_vjp_ratio(float* t, const float* v, const float* y, const float* r, float* gy,
                               size_t m, hipStream_t s) {
  hipLaunchKernelGGL(em_vjp_ratio_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, t, v,
                     y, r, gy, m);
  return hipGetLastError();
}

hipError_t launch_add(float* a, const float* b, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t launch_em_reg_update(float* x, const float* e, const float* sens, const float* u,
                                float beta, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(em_reg_update_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, e,
                     sens, u, beta, n);
  return hipGetLastError();
}

hipError_t launch_dot_f64(const float* a, const float* b, size_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(dot_f64_kernel, dim3(1), dim3(kDotThreads), 0, s, a, b, n, out);
  return hipGetLastError();
}

}  // namespace spect
