// Device generation of perturbed positions for repeated solves:
// r_u = r + sigma * z with z standard normal, drawn from the counter-based
// generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011) and the Box-Muller transform.
// The step index is read from device memory, so that a captured HIP graph
// that also advances it draws fresh inputs on every replay.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include "inputs.hpp"

namespace {

// Philox4x32 round constants: the two multipliers and the Weyl key
// increments of the published generator.
constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;

__device__ inline uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(kMul0) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(kMul1) * c.z;
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += kWeyl0;
    k.y += kWeyl1;
  }
  return c;
}

// two 32-bit words -> uniform double in (0, 1) with 53 random bits
__device__ inline double uniform53(uint32_t lo, uint32_t hi) {
  const uint64_t x = ((static_cast<uint64_t>(hi) << 32) | lo) >> 11;
  return (static_cast<double>(x) + 0.5) * 0x1.0p-53;
}

__device__ inline double2 box_muller(uint4 w) {
  const double u1 = uniform53(w.x, w.y), u2 = uniform53(w.z, w.w);
  const double rho = sqrt(-2.0 * log(u1));
  const double th = 6.283185307179586476925287 * u2;
  return make_double2(rho * cos(th), rho * sin(th));
}

__global__ void __launch_bounds__(256) perturb_kernel(const double* __restrict__ r, int32_t n, double sigma,
                                                      uint2 key, const uint64_t* __restrict__ step,
                                                      double* __restrict__ ru) {
  const int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t s = *step;
  const uint32_t s_lo = static_cast<uint32_t>(s), s_hi = static_cast<uint32_t>(s >> 32);
  const double2 zxy = box_muller(philox4x32_10(make_uint4(static_cast<uint32_t>(i), 0u, s_lo, s_hi), key));
  const double2 zz = box_muller(philox4x32_10(make_uint4(static_cast<uint32_t>(i), 1u, s_lo, s_hi), key));
  ru[i] = r[i] + sigma * zxy.x;
  ru[n + i] = r[n + i] + sigma * zxy.y;
  ru[2 * n + i] = r[2 * n + i] + sigma * zz.x;
}

__global__ void counter_add_kernel(uint64_t* c, uint64_t d) {
  if (threadIdx.x == 0) *c += d;
}

}  // namespace

namespace ilves_in {

hipError_t launch_perturb(const double* r, int32_t n_atoms, double sigma, uint64_t seed, const uint64_t* step,
                          double* r_u, hipStream_t stream) {
  const uint2 key = make_uint2(static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  (void)hipGetLastError();  // no stale error from an earlier call
  hipLaunchKernelGGL(perturb_kernel, dim3((n_atoms + 255) / 256), dim3(256), 0, stream, r, n_atoms, sigma, key,
                     step, r_u);
  return hipGetLastError();
}

hipError_t launch_counter_add(uint64_t* counter, uint64_t delta, hipStream_t stream) {
  (void)hipGetLastError();  // no stale error from an earlier call
  hipLaunchKernelGGL(counter_add_kernel, dim3(1), dim3(64), 0, stream, counter, delta);
  return hipGetLastError();
}

}  // namespace ilves_in
