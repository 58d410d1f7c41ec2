// Device helpers shared by the complex64 and complex-half kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "desc.h"

namespace matnc {

// Workspace addresses are plain integers; a pointer made from one carries no
// address space, and the compiler then emits FLAT accesses, which also count
// on the LDS wait counter (every LDS wait would drain the outstanding global
// loads as well).  Every access to the workspace goes through a global
// (address space 1) pointer instead.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> gmem(uint64_t a) {
  return (gptr<T>)a;
}

// Offset tables are written when a plan is bound and only read by the
// kernels.  A lookup at a wave-uniform index (a k step) through a constant
// (address space 4) pointer compiles to scalar loads, which count on the
// LDS/scalar wait counter: waiting for its result inside a k loop then does
// not also wait for the operand loads in flight, which complete in order on
// the vector-memory counter.
template <typename T>
using cptr = __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ cptr<T> cmem(uint64_t a) {
  return (cptr<T>)a;
}

// unsigned atomic max on a workspace word (float bits of non-negative values)
__device__ __forceinline__ void gmax_u32(uint64_t a, uint32_t v) { atomicMax((uint32_t*)a, v); }

// element accessors (HIP's float2 / __half2 classes cannot be copied
// through an address-space-qualified reference; plain vectors can)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 ldg_f2(uint64_t base, uint64_t i) {
  const f32x2 v = gmem<const f32x2>(base)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void stg_f2(uint64_t base, uint64_t i, float2 v) { gmem<f32x2>(base)[i] = f32x2{v.x, v.y}; }
__device__ __forceinline__ uint32_t ldg_u32(uint64_t base, uint64_t i) { return gmem<const uint32_t>(base)[i]; }
__device__ __forceinline__ void stg_u32(uint64_t base, uint64_t i, uint32_t v) { gmem<uint32_t>(base)[i] = v; }
__device__ __forceinline__ HalfScale ldg_scale(uint64_t base, int64_t i) {
  const u32x2 v = gmem<const u32x2>(base)[i];
  HalfScale h;
  h.e = (int32_t)v.x;
  h.mx = v.y;
  return h;
}
// exponent word of scale slot i, and an atomic max into its maximum word
__device__ __forceinline__ void stg_scale_e(uint64_t base, int64_t i, int32_t e) {
  gmem<int32_t>(base + (uint64_t)i * sizeof(HalfScale))[0] = e;
}
// The slot was cleared before the launch and only grows while it runs, so a
// value read from it is never above the final maximum: when it already holds
// at least mx_bits the atomic is skipped.  An instance spread over many tiles
// or blocks (a stem tensor) would otherwise send every one of them to the
// same address.
__device__ __forceinline__ void max_scale_mx(uint64_t base, int64_t i, uint32_t mx_bits) {
  uint32_t* p = (uint32_t*)(base + (uint64_t)i * sizeof(HalfScale) + offsetof(HalfScale, mx));
  if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < mx_bits) atomicMax(p, mx_bits);
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  A grid-stride index vid (grid size a multiple of 8, or a single
// pass) maps to a logical tile so that XCD x works through the contiguous
// logical range [start(x), start(x) + count(x)): neighbouring tiles, which
// share operand data, then meet in the same L2.  A bijection on [0, total).
__device__ __forceinline__ int64_t xcd_tile(int64_t vid, int64_t total) {
  const int64_t q = total >> 3, r = total & 7;
  const int64_t x = vid & 7, k = vid >> 3;
  return x * q + (x < r ? x : r) + k;
}

// Logical (unit, tile) of a logical tile index.  Units (output instances,
// or fan-table rows) are taken in blocks of R; inside a block the tile
// index is outermost, so that the R tiles at one position of the R units
// run next to each other on one XCD.  Units that read the same A instance
// are adjacent (fan tables are grouped by A instance, plain instances are
// in key order), so the later reads of each A tile hit the L2.  R = 1
// (plain steps) is the unit-major order; fan-out steps, whose A instances
// are shared by about two rows, take R = 2; a unit group sharing an A
// instance far larger than the caches takes R = its size, so that the
// instance streams from HBM once while the group's B instances are re-read
// from the caches.  A bijection on [0, units * tiles) for any R >= 1 (a
// short last block keeps the same order over its units).
__device__ __forceinline__ void unit_tile(int64_t lt, int64_t units, int64_t tiles, int64_t R, int64_t& u,
                                          int64_t& t) {
  const int64_t blk = lt / (R * tiles);
  const int64_t r = lt - blk * R * tiles;
  const int64_t rows = units - blk * R < R ? units - blk * R : R;  // units in this block
  u = blk * R + r % rows;
  t = r / rows;
}

template <typename P>
__device__ __forceinline__ uint32_t tlook(P T, uint32_t x) {
  return T[x & 255u] + T[256 + ((x >> 8) & 255u)] + T[512 + ((x >> 16) & 255u)] + T[768 + (x >> 24)];
}

// offset of coordinate hi * 256 + lo (lo < 256)
template <typename P>
__device__ __forceinline__ uint32_t tlook_split(P T, uint32_t hi, uint32_t lo) {
  return T[lo] + T[256 + (hi & 255u)] + T[512 + ((hi >> 8) & 255u)] + T[768 + (hi >> 16)];
}

template <typename P>
__device__ __forceinline__ int64_t operand_instance(const OpDesc& o, P gmap, int64_t j, int64_t s, int64_t sigma) {
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
