// Leapfrog kernels around the constraint solve.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ilves_md {

// v += h f / m; r_u = r + h v   (SoA [3][n] FP64, mass [n])
hipError_t launch_kick_drift(const double* r, double* v, const double* f, const double* mass, double h, int32_t n,
                             double* r_u, hipStream_t stream);

// v = (r_new - r) / h; r = r_new
hipError_t launch_finish(double* r, const double* r_new, double h, int32_t n, double* v, hipStream_t stream);

}  // namespace ilves_md
