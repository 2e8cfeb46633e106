// Device radix sort of the comparator's (tile << 32 | depth bits, id) pairs.
// The paper's baseline sorts its tile-depth keys with a library device
// radix sort; rocPRIM's onesweep radix sort is the equivalent library
// primitive here. The sort is stable, so equal keys keep emission order,
// which is ascending Gaussian id.
#include <rocprim/device/device_radix_sort.hpp>

#include "common.hpp"

namespace tgs {

size_t global_sort_tmp_bytes(int64_t capacity, int end_bit) {
    size_t bytes = 0;
    if (capacity <= 0) return 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, bytes, static_cast<uint64_t*>(nullptr), static_cast<uint64_t*>(nullptr),
                              static_cast<uint32_t*>(nullptr), static_cast<uint32_t*>(nullptr), (size_t)capacity, 0,
                              end_bit);
    return e == hipSuccess ? bytes : 0;
}

hipError_t launch_global_sort(void* tmp, size_t tmp_bytes, uint64_t* keys_in, uint64_t* keys_out, uint32_t* vals_in,
                              uint32_t* vals_out, int64_t m, int end_bit, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    size_t need = 0;
    hipError_t e = rocprim::radix_sort_pairs(nullptr, need, keys_in, keys_out, vals_in, vals_out, (size_t)m, 0,
                                             end_bit, s);
    if (e != hipSuccess) return e;
    if (need > tmp_bytes) return hipErrorInvalidValue;
    return rocprim::radix_sort_pairs(tmp, need, keys_in, keys_out, vals_in, vals_out, (size_t)m, 0, end_bit, s);
}

}  // namespace tgs
