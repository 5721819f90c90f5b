// Fixed device scratch of the allocation-free apply (noalloc.hip).
#pragma once

#include <cstddef>

#include "dcommon.h"

namespace diaf {

// Bytes of the per-device scratch array: 256 for the control words, the
// rest for the intermediate vector (n doubles or n complex doubles).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
constexpr size_t NOALLOC_CTL_BYTES = 256;

// Take the scratch array's address on `device` (which must be current),
// once per device; later calls return at once.
Err noalloc_init(int device);
// The address taken by noalloc_init on `device`.
Err noalloc_scratch(int device, void** ptr);
// Zero `bytes` at p (rounded up to whole 32-bit words) with a kernel on st.
Err noalloc_clear(void* p, size_t bytes, hipStream_t st);

}  // namespace diaf
