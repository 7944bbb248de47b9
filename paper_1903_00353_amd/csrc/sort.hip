// Stable device radix sort of (key, value) pairs (hipCUB / rocPRIM), used to
// group triangle corners by vertex.
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace csc {

size_t sort_pairs_tmp_bytes(int64_t n, int bits) {
  size_t tmp = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                                    (const int32_t*)nullptr, (int32_t*)nullptr, (int)n, 0, bits,
                                                    (hipStream_t)0);
  return e == hipSuccess ? tmp : 0;
}

hipError_t sort_pairs(void* tmp, size_t tmp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                      const int32_t* vals_in, int32_t* vals_out, int64_t n, int bits, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys_in, keys_out, vals_in, vals_out, (int)n, 0, bits, s);
}

}  // namespace csc
