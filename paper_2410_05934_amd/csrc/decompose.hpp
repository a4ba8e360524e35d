// decompose.hpp -- signed gadget digits: the Decompose step of the TFHE external
// product (Sec. II-B, Sec. IV-A).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nttk {

// Digit j (of `levels`) of the word x in base B = 2^log_base, as a residue mod q.
// The digits are the balanced ones: from the remainder r (initially x), each
// lower digit is r mod B moved to [-B/2, B/2) and r becomes (r - d) / B; the top
// digit is the last remainder, so x = sum_j d_j B^j exactly.  They are read off
// y = x + offset, offset = (B/2)(1 + B + ... + B^(levels-2)): adding B/2 at
// every lower position turns each balanced digit d_j into the plain base-B
// digit d_j + B/2 of y (the carries are the same), and the top digit is
// y >> (log_base (levels - 1)).  levels * log_base <= 64 keeps y below 2^64
// (x < 2^62, offset < 2^(log_base (levels - 1))); the top digit lies in
// [0, B/2] when q <= 2^(levels * log_base - 1).  Both bounds are checked by
// the caller.
template <class W>
__host__ __device__ __forceinline__ W signed_digit(W x, uint32_t j, uint32_t levels,
                                                   uint32_t log_base, uint64_t offset, uint64_t q) {
  const uint64_t y = (uint64_t)x + offset;
  int64_t d;
  if (j + 1 >= levels) {
    d = (int64_t)(y >> (log_base * j));
  } else {
    const uint64_t mask = (1ull << log_base) - 1;
    d = (int64_t)((y >> (log_base * j)) & mask) - (int64_t)(1ull << (log_base - 1));
  }
  return (W)(d < 0 ? (int64_t)q + d : d);
}

// The offset above: B/2 at each of the levels - 1 lower digit positions.
__host__ __device__ inline uint64_t digit_offset(uint32_t levels, uint32_t log_base) {
  uint64_t c = 0;
  for (uint32_t j = 0; j + 1 < levels; ++j) c += (1ull << (log_base - 1)) << (log_base * j);
  return c;
}

}  // namespace nttk
