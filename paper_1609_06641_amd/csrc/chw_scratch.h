// chw_scratch.h -- the static device scratch of chw_forward_noalloc (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace chw {

// Bytes of the scratch array: 64 MiB, the intermediate of 2^24 FP32 / int32
// elements (2^23 FP64) of two-pass signals.
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;

// Device address of the scratch array on device `dev`, which must be the
// current device.  The first call on a device asks hipGetSymbolAddress and
// keeps the address; later calls return the kept one.
hipError_t scratch_address(int dev, void **ptr);

}  // namespace chw
