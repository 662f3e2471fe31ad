// Process-wide cache of device allocations (devpool.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>

namespace raspml {

// hipMalloc through the cache: reuses an idle block of this device whose
// rounded size fits within 1/8, else maps a new one.
hipError_t pool_alloc(void **p, size_t bytes);
// Returns a block obtained from pool_alloc to the cache (or to the driver
// beyond the cache limit).  The caller guarantees that no queued or running
// work still uses it.
void pool_free(void *p);

}  // namespace raspml
