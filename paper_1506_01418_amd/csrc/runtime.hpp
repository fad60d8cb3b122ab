// Host-side helpers shared by the context runtime and the serving loop.
#pragma once
#include <hip/hip_runtime.h>

namespace psgld {

// hipSetDevice(dev) unless dev is already the calling thread's device.
hipError_t use_device(int dev);

}  // namespace psgld
