// Allocation-free variants: their scratch is a file-scope device array of
// fixed size (noalloc.hip), whose device address is taken once per device.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace kpme {

// Doubles in the scratch array: the kSumBlocks (sum q pot, sum q, sum q^2)
// triples of the energy reduction.
constexpr int kNoallocScratchDoubles = 3 * kSumBlocks;

// Device address of the scratch array on `device` (looked up on first use).
hipError_t noalloc_scratch(int device, double** out);

// launch_energy with the scratch array in place of a workspace.
hipError_t launch_energy_noalloc(int device, int prec, int64_t n, const void* q,
                                 const void* pot, double beta, double volume,
                                 double* energy4, hipStream_t st);

}  // namespace kpme
