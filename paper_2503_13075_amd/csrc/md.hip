// Leapfrog steps around the constraint solve (the MD step of the main
// text's section on constrained dynamics, with the constraint solved for the
// new positions at every step):
//   v_{k+1/2} = v_{k-1/2} + h M^-1 f_k,   r_u = r_k + h v_{k+1/2}     (kick, drift)
//   r_{k+1}   = solve(r_k, r_u)                                          (constraints)
//   v_{k+1/2} = (r_{k+1} - r_k) / h,      r_k <- r_{k+1}               (finish)
// so the velocities carried to the next step are those of the constrained
// positions.  One thread per atom, SoA [3][n] FP64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "md.hpp"

namespace {

__global__ void __launch_bounds__(256) kick_drift_kernel(const double* __restrict__ r, double* __restrict__ v,
                                                         const double* __restrict__ f,
                                                         const double* __restrict__ mass, double h, int32_t n,
                                                         double* __restrict__ r_u) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double s = h / mass[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double vv = v[c * n + i] + s * f[c * n + i];
    v[c * n + i] = vv;
    r_u[c * n + i] = r[c * n + i] + h * vv;
  }
}

__global__ void __launch_bounds__(256) finish_kernel(double* __restrict__ r, const double* __restrict__ r_new,
                                                     double inv_h, int32_t n, double* __restrict__ v) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double x = r_new[c * n + i];
    v[c * n + i] = (x - r[c * n + i]) * inv_h;
    r[c * n + i] = x;
  }
}

}  // namespace

namespace ilves_md {

hipError_t launch_kick_drift(const double* r, double* v, const double* f, const double* mass, double h, int32_t n,
                             double* r_u, hipStream_t stream) {
  (void)hipGetLastError();  // no stale error from an earlier call
  hipLaunchKernelGGL(kick_drift_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, r, v, f, mass, h, n, r_u);
  return hipGetLastError();
}

hipError_t launch_finish(double* r, const double* r_new, double h, int32_t n, double* v, hipStream_t stream) {
  (void)hipGetLastError();  // no stale error from an earlier call
  hipLaunchKernelGGL(finish_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, r, r_new, 1.0 / h, n, v);
  return hipGetLastError();
}

}  // namespace ilves_md
