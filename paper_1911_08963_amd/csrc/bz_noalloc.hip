// Device scratch of bz_min_distance_noalloc: one file-scope array, of which
// every device the library runs on holds its own copy until the process ends.
// Host code must not pass the array's name to a kernel (in host code it is a
// host-side stand-in, not a device address); the address comes from
// hipGetSymbolAddress, called with the device current.
#include <hip/hip_runtime.h>

#include "bz_host.h"

static __device__ __align__(256) unsigned char scratch[bz::kNoAllocScratchBytes];

namespace bz {

hipError_t noalloc_scratch_address(void **ptr) {
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

}  // namespace bz
