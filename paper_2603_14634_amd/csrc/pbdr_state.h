// Per-body state read-out of a single scene (not on the solver's hot path).
// Internal to libpbdr.
#pragma once
#include "pbdr_device.h"

namespace pbdr {

// Writes the per-body state of the current (x, v) into out ([B][18] doubles:
// centre of mass, rotation, linear and angular momentum).
hipError_t enqueue_body_state(const Scene& s, double* out, hipStream_t stream);

}  // namespace pbdr
