// Shared host-side helpers of the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>

#include "gsr.h"
#include "kernels.hpp"

namespace gsr {

extern thread_local std::string g_last_error;

// Record a message for gsr_last_error() and return `s`.
gsr_status fail(gsr_status s, const char* fmt, ...);
gsr_status hip_fail(hipError_t e, const char* what);
// Current device must be a gfx950; returns its compute-unit count.
gsr_status check_device(int* dev, int* n_cu);
gsr_status check_dims(const gsr_dims* d);
Geo make_geo(const gsr_dims* d);
int grid_for(int64_t items, int per_block, int max_blocks);
// Device memory for the library's arrays (hipMalloc semantics; free with hipFree).
hipError_t device_alloc(void** p, size_t bytes);

}  // namespace gsr
