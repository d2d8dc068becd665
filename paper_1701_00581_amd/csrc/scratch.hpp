// Device scratch array of nvsm_reconstruct_noalloc (see scratch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace nvsm {

// Size of the array on each GPU: 256 MiB.
constexpr size_t SCRATCH_BYTES = (size_t)256 << 20;
constexpr int SCRATCH_MAX_DEVICES = 64;

// Looks up `device`'s copy of the array (once; later calls return at once).
hipError_t scratch_setup(int device);
// The device address scratch_setup found for `device`, or null.
void *scratch_address(int device);

}  // namespace nvsm
