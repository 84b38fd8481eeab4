// Device helpers shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

namespace gsw {

// Position of the k-th (from 0) set bit of m; k < popcount(m).  A binary
// search over the halves, quarters, ... of the word by their popcounts.
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int k) {
  int pos = 0;
  int c = __popc((unsigned)m);
  if (k >= c) { k -= c; m >>= 32; pos += 32; }
  c = __popc((unsigned)(m & 0xffffull));
  if (k >= c) { k -= c; m >>= 16; pos += 16; }
  c = __popc((unsigned)(m & 0xffull));
  if (k >= c) { k -= c; m >>= 8; pos += 8; }
  c = __popc((unsigned)(m & 0xfull));
  if (k >= c) { k -= c; m >>= 4; pos += 4; }
  c = __popc((unsigned)(m & 0x3ull));
  if (k >= c) { k -= c; m >>= 2; pos += 2; }
  if (k >= (int)(m & 1ull)) pos += 1;
  return pos;
}

}  // namespace gsw
