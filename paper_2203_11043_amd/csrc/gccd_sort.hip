// Radix sort of the 64-bit curve/index keys that order the Eq. (6)
// targets spatially (rocPRIM device radix sort; temporary storage is
// allocated once per load by the caller, so a step allocates nothing).
#include "gccd_internal.h"

#include <rocprim/device/device_radix_sort.hpp>

namespace gccd {

hipError_t sort_keys_storage(uint32_t n, uint32_t end_bit, size_t* bytes) {
    size_t b = 0;
    hipError_t e = rocprim::radix_sort_keys(nullptr, b, static_cast<const uint64_t*>(nullptr),
                                            static_cast<uint64_t*>(nullptr), n, 0u, end_bit);
    *bytes = b;
    return e;
}

hipError_t sort_keys(void* tmp, size_t tmp_bytes, const uint64_t* in, uint64_t* out, uint32_t n,
                     uint32_t end_bit, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t b = tmp_bytes;
    return rocprim::radix_sort_keys(tmp, b, in, out, n, 0u, end_bit, s);
}

}  // namespace gccd
