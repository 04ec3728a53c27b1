// rx_comb.hpp -- comb-pilot interpolation shared by the estimate kernel and
// the training-channel generator (device code).
#pragma once

#include <hip/hip_runtime.h>

namespace rx {

// Value of used subcarrier d from the LS values pil[j] of the pilot
// subcarriers j*ps: the straight line in signed frequency (d - U/2 below the
// DC gap, d - U/2 + 1 above it) between the pilot at or below d and the next
// pilot; past the last pilot its value is held.
__device__ __forceinline__ float2 comb_value(const float2* pil, int d, int U, int ps) {
  const int j0 = d / ps, last = (U - 1) / ps;
  if (j0 >= last) return pil[last];
  const int d0 = j0 * ps;
  if (d == d0) return pil[j0];
  const int h = U >> 1;
  auto fr = [h](int x) { return x < h ? x - h : x - h + 1; };
  const float t = (float)(fr(d) - fr(d0)) / (float)(fr(d0 + ps) - fr(d0));
  const float2 a = pil[j0], b = pil[j0 + 1];
  return make_float2(a.x + t * (b.x - a.x), a.y + t * (b.y - a.y));
}

}  // namespace rx
