// Device helpers shared by the complex64 and complex-half kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "desc.h"

namespace matnc {

__device__ __forceinline__ uint32_t tlook(const uint32_t* __restrict__ T, uint32_t x) {
  return T[x & 255u] + T[256 + ((x >> 8) & 255u)] + T[512 + ((x >> 16) & 255u)] + T[768 + (x >> 24)];
}

// offset of coordinate hi * 256 + lo (lo < 256)
__device__ __forceinline__ uint32_t tlook_split(const uint32_t* __restrict__ T, uint32_t hi, uint32_t lo) {
  return T[lo] + T[256 + (hi & 255u)] + T[512 + ((hi >> 8) & 255u)] + T[768 + (hi >> 16)];
}

__device__ __forceinline__ int64_t operand_instance(const OpDesc& o, const int32_t* gmap, int64_t j,
                                                    int64_t s, int64_t sigma) {
  int64_t v = (int64_t)gmap[j] * o.nsv;
  for (int t = 0; t < o.nsb; ++t) v += ((sigma >> o.sbit[t]) & 1) << t;
  if (o.dep) v += s * (int64_t)o.w_child;
  return v;
}

__device__ __forceinline__ void cmac(float2& c, float2 a, float2 b) {
  c.x = fmaf(a.x, b.x, c.x);
  c.x = fmaf(-a.y, b.y, c.x);
  c.y = fmaf(a.x, b.y, c.y);
  c.y = fmaf(a.y, b.x, c.y);
}


// grid size for grid-stride loops
static inline unsigned grid_for(int64_t blocks) {
  const int64_t cap = 256 * 1024;
  return (unsigned)(blocks < 1 ? 1 : (blocks > cap ? cap : blocks));
}

}  // namespace matnc
