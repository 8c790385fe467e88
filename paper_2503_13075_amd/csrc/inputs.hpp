// Device generation of perturbed inputs (Philox4x32-10 + Box-Muller).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ilves_in {

// r_u = r + sigma * z for every atom, z from Philox4x32-10 with key = seed
// and counter {atom, 0 | 1, step (two words)}; *step is read on the device.
hipError_t launch_perturb(const double* r, int32_t n_atoms, double sigma, uint64_t seed, const uint64_t* step,
                          double* r_u, hipStream_t stream);

// *counter += delta on the device.
hipError_t launch_counter_add(uint64_t* counter, uint64_t delta, hipStream_t stream);

}  // namespace ilves_in
