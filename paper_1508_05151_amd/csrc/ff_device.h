// Device helpers shared by the HIP translation units of libff (the searches
// with the census and with the SIFT-flow data term draw the same random
// offsets).  Included by .hip sources only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ff {

// Philox4x32-10 (Salmon et al., SC 2011): 10 rounds of the two multiplier
// S-boxes with Weyl-sequence key schedule.  Returns the first two words.
__device__ __forceinline__ void philox2(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                        uint32_t& o0, uint32_t& o1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  o0 = c0;
  o1 = c1;
}

}  // namespace ff
