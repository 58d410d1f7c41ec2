// Streaming (VALU) kernels of one pairwise step C[m, n] = sum_k A[m, k] B[k, n],
// for both storage precisions.  These steps move more bytes than they
// compute (a big tensor times a gate-sized one, or a batched matrix-vector
// product), so the kernels are built for HBM bandwidth:
//
//  * k_wide<FL, KB, R>     small K (<= 16) and N (<= 16): every lane owns R
//    values of m spaced 256 apart (R x KB loads in flight), B is staged once
//    per block in LDS, all offset tables that do not depend on m are hoisted.
//    A block covers 256*R consecutive m of one instance, so instance
//    decoding and B are block-uniform.
//  * k_narrow<FL, KB>      the same for instances smaller than 256 elements:
//    one lane per (instance, m).
//  * k_kred<FL, NB>        large K: lanes own m (coalesced reads of A along
//    its low bits), groups of lanes split K, partial sums meet in LDS.
//  * k_generic<FL>         anything else (one lane per output element).
//
// Precision policy P: C64 plans store float2 everywhere.  MIX (complex-half
// plans) stores each tensor as __half2 with a per-instance exponent e
// (value = half * 2^e) or as float2 (e = 0), as the plan decided; every
// stored instance also carries its measured maximum mx.  A FP16 output's
// exponent is chosen from the operands' maxima so that |Re|, |Im| of every
// output (bounded by 2^(kbits+1) mx_A mx_B 2^(e_A+e_B)) is stored below
// 2^15 (no FP16 overflow); the maximum of the stored output is measured
// (block reduction + unsigned atomicMax on the float bits, exact because
// all values are non-negative) for the next step.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "desc.h"
#include "device_common.h"
#include "kernels.h"

namespace matnc {

// Storage flags FL (compile-time): bit 3 = complex-half plan (scales
// tracked); bit 0 / 1 / 2 = A / B / C stored as FP16 (else FP32).
constexpr int kMixBit = 8;

template <int FL, int WHICH>
__device__ __forceinline__ float2 ldop(uint64_t base, uint32_t i) {
  if constexpr ((FL & kMixBit) && (FL & WHICH)) {
    const uint32_t u = ldg_u32(base, i);
    __half2 h;
    __builtin_memcpy(&h, &u, 4);
    return __half22float2(h);
  }
  return ldg_f2(base, i);
}

// Output scale of one instance; identity for complex64 plans.
struct OutScale {
  float f;       // multiply the FP32 result by f before storing
  int32_t e;     // exponent recorded for the output instance
};

template <int FL>
__device__ __forceinline__ OutScale out_scale(const NodeDesc& d, uint64_t ws, int64_t ai, int64_t bi) {
  OutScale o{1.f, 0};
  if constexpr ((FL & kMixBit) != 0) {
    const HalfScale sa = ldg_scale(ws + d.A.scale_off, ai);
    const HalfScale sb = ldg_scale(ws + d.B.scale_off, bi);
    if constexpr ((FL & 4) != 0) {
      const float bound = ldexpf(__uint_as_float(sa.mx) * __uint_as_float(sb.mx), d.kbits + 1);
      int ex = 0;
      if (bound > 0.f) frexpf(bound, &ex);  // bound < 2^ex
      o.e = sa.e + sb.e + ex - 15;
      o.f = ldexpf(1.f, 15 - ex);
    } else {
      o.e = 0;
      o.f = ldexpf(1.f, sa.e + sb.e);
    }
  }
  return o;
}

// store one output element; returns the largest stored |component|
template <int FL>
__device__ __forceinline__ float put(uint64_t base, uint32_t i, float2 c, const OutScale& s) {
  if constexpr ((FL & kMixBit) != 0) {
    const float2 v = make_float2(c.x * s.f, c.y * s.f);
    if constexpr ((FL & 4) != 0) {
      const __half2 h = __float22half2_rn(v);
      uint32_t u;
      __builtin_memcpy(&u, &h, 4);
      stg_u32(base, i, u);
      const float2 back = __half22float2(h);
      return fmaxf(fabsf(back.x), fabsf(back.y));
    }
    stg_f2(base, i, v);
    return fmaxf(fabsf(v.x), fabsf(v.y));
  } else {
    stg_f2(base, i, c);
    return 0.f;
  }
}

template <int FL>
__device__ __forceinline__ void record_scale(const NodeDesc& d, uint64_t ws, int64_t inst, const OutScale& s,
                                             float mx, bool writer) {
  if constexpr ((FL & kMixBit) != 0) {
    if (writer) stg_scale_e(ws + d.c_scale_off, inst, s.e);
    if (mx > 0.f) max_scale_mx(ws + d.c_scale_off, inst, __float_as_uint(mx));
  }
}

// max over the 64 lanes of a wave
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// max over lanes whose index agrees above bit log2(seg) (seg <= 64)
__device__ __forceinline__ float segment_max(float v, int seg) {
  for (int o = seg >> 1; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// record the output maximum: at most one atomic per wave, no block barrier;
// the exponent (the same for every block of the instance) is written by the
// first wave of the block that covers the instance's first elements
template <int FL>
__device__ __forceinline__ void block_record(const NodeDesc& d, uint64_t ws, int64_t inst, const OutScale& s, float mx,
                                             float* /*red*/, bool first_block) {
  if constexpr ((FL & kMixBit) != 0) {
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) record_scale<FL>(d, ws, inst, s, mx, first_block && threadIdx.x == 0);
  }
}

struct InstPtrs {
  int64_t inst, ai, bi;
  uint64_t pa, pb, pc;
};

__device__ __forceinline__ InstPtrs instance_ptrs(const NodeDesc& d, uint64_t ws, int64_t inst, int64_t sigma0) {
  InstPtrs r;
  r.inst = inst;
  const int64_t s = d.dep ? inst / d.w : 0;
  const int64_t j = d.dep ? inst - s * d.w : inst;
  const gptr<const int32_t> glA = gmem<const int32_t>(ws + d.A.gmap_off);
  const gptr<const int32_t> glB = gmem<const int32_t>(ws + d.B.gmap_off);
  r.ai = operand_instance(d.A, glA, j, s, sigma0 + s);
  r.bi = operand_instance(d.B, glB, j, s, sigma0 + s);
  r.pa = ws + d.A.off + (uint64_t)r.ai * d.A.inst_bytes;
  r.pb = ws + d.B.off + (uint64_t)r.bi * d.B.inst_bytes;
  r.pc = ws + d.c_off + (uint64_t)inst * d.c_inst_bytes;
  return r;
}

// ---------------------------------------------------------------------------

// N (<= 16) is a runtime bound: outputs are produced one n at a time
template <int FL, int KB, int R>
__global__ __launch_bounds__(256) void k_wide(NodeDesc d, uint64_t ws, const int64_t* __restrict__ sig) {
  constexpr int LR = (R == 1) ? 0 : (R == 2) ? 1 : (R == 4) ? 2 : 3;
  __shared__ float2 Bs[KB * 16];
  __shared__ float red[4];
  const gptr<const uint32_t> tab = gmem<const uint32_t>(ws + d.tab_off);
  const gptr<const uint32_t> TA = tab + TAB_AM * kTabSize;
  const gptr<const uint32_t> TC = tab + TAB_CM * kTabSize;
  const int tid = threadIdx.x;
  const int NB = 1 << d.nbits;
  const uint32_t oa_lo = TA[tid], oc_lo = TC[tid];
  uint32_t tak[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) tak[k] = tab[TAB_AK * kTabSize + k];
  // this lane's B element when staging (KB * NB <= 256)
  uint32_t ob_mine = 0;
  if (tid < KB * NB) ob_mine = tab[TAB_BK * kTabSize + tid / NB] + tab[TAB_BN * kTabSize + tid % NB];
  const int sh = d.mbits - 8 - LR;
  const int64_t bpi = (int64_t)1 << sh;
  const int64_t nblk = d.n_inst << sh;
  const int64_t sigma0 = sig[0];
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const InstPtrs ip = instance_ptrs(d, ws, blk >> sh, sigma0);
    const uint32_t hi0 = (uint32_t)(blk & (bpi - 1)) << LR;
    if (tid < KB * NB) Bs[tid] = ldop<FL, 2>(ip.pb, ob_mine);
    uint32_t oa[R], oc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t hi = hi0 + r;
      oa[r] = oa_lo + TA[256 + (hi & 255u)] + TA[512 + ((hi >> 8) & 255u)] + TA[768 + (hi >> 16)];
      oc[r] = oc_lo + TC[256 + (hi & 255u)] + TC[512 + ((hi >> 8) & 255u)] + TC[768 + (hi >> 16)];
    }
    float2 a[R][KB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < KB; ++k) a[r][k] = ldop<FL, 1>(ip.pa, oa[r] + tak[k]);
    const OutScale s = out_scale<FL>(d, ws, ip.ai, ip.bi);
    __syncthreads();
    float mx = 0.f;
    for (int n = 0; n < NB; ++n) {
      const uint32_t cn = tab[TAB_CN * kTabSize + n];
      float2 b[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k) b[k] = Bs[k * NB + n];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 c = make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < KB; ++k) cmac(c, a[r][k], b[k]);
        mx = fmaxf(mx, put<FL>(ip.pc, oc[r] + cn, c, s));
      }
    }
    block_record<FL>(d, ws, ip.inst, s, mx, red, hi0 == 0);
    __syncthreads();  // Bs is rewritten next iteration
  }
}

template <int FL, int KB>
__global__ __launch_bounds__(256) void k_narrow(NodeDesc d, uint64_t ws, const int64_t* __restrict__ sig) {
  const gptr<const uint32_t> tab = gmem<const uint32_t>(ws + d.tab_off);
  const int NB = 1 << d.nbits;
  uint32_t tak[KB], tbk[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    tak[k] = tab[TAB_AK * kTabSize + k];
    tbk[k] = tab[TAB_BK * kTabSize + k];
  }
  const int64_t total = d.n_inst << d.mbits;
  const uint32_t mmask = (1u << d.mbits) - 1u;
  const int64_t sigma0 = sig[0];
  const int seg = d.mbits >= 6 ? 64 : (1 << d.mbits);
  for (int64_t base = (int64_t)blockIdx.x * 256; base < total; base += (int64_t)gridDim.x * 256) {
    const int64_t g = base + threadIdx.x;
    const bool live = g < total;
    float mx = 0.f;
    OutScale s{1.f, 0};
    int64_t inst = 0;
    if (live) {
      inst = g >> d.mbits;
      const uint32_t m = (uint32_t)g & mmask;
      const InstPtrs ip = instance_ptrs(d, ws, inst, sigma0);
      const uint32_t oa = tab[TAB_AM * kTabSize + m];
      const uint32_t oc = tab[TAB_CM * kTabSize + m];
      float2 a[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k) a[k] = ldop<FL, 1>(ip.pa, oa + tak[k]);
      s = out_scale<FL>(d, ws, ip.ai, ip.bi);
      for (int n = 0; n < NB; ++n) {
        const uint32_t bn = tab[TAB_BN * kTabSize + n];
        float2 c = make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < KB; ++k) cmac(c, a[k], ldop<FL, 2>(ip.pb, bn + tbk[k]));
        mx = fmaxf(mx, put<FL>(ip.pc, oc + tab[TAB_CN * kTabSize + n], c, s));
      }
    }
    if constexpr ((FL & kMixBit) != 0) {
      // lanes of one instance are contiguous; reduce within segments of a wave
      mx = segment_max(mx, seg);
      const int lane = threadIdx.x & 63;
      if (live && (lane & (seg - 1)) == 0) record_scale<FL>(d, ws, inst, s, mx, ((uint32_t)g & mmask) == 0);
    }
  }
}

// large K: block = (instance, 256-wide chunk of m) or, for M < 256, one
// instance with 256 / M groups splitting K
// KS1: M >= 256, every lane of a block walks the same k, so B's offsets are
// made wave-uniform and its loads go through the scalar path
template <int FL, int NB, bool KS1>
__global__ __launch_bounds__(256) void k_kred(NodeDesc d, uint64_t ws, const int64_t* __restrict__ sig) {
  __shared__ uint32_t kofa[256], kofb[256];
  __shared__ float2 part[256 * NB];
  __shared__ float red[4];
  const gptr<const uint32_t> tab = gmem<const uint32_t>(ws + d.tab_off);
  const int tid = threadIdx.x;
  kofa[tid] = tab[TAB_AK * kTabSize + tid];
  kofb[tid] = tab[TAB_BK * kTabSize + tid];
  uint32_t tbn[NB], tcn[NB];
#pragma unroll
  for (int n = 0; n < NB; ++n) {
    tbn[n] = tab[TAB_BN * kTabSize + n];
    tcn[n] = tab[TAB_CN * kTabSize + n];
  }
  __syncthreads();
  const int mb = d.mbits < 8 ? d.mbits : 8;
  const int M = 1 << mb;
  const int KS = 256 >> mb;            // groups splitting K
  const int mloc = tid & (M - 1);
  const int grp = tid >> mb;
  const int chunks_sh = d.mbits - mb;  // 256-wide m chunks per instance
  const int64_t nblk = d.n_inst << chunks_sh;
  const uint32_t kcount = 1u << d.kbits;
  const uint32_t klo_n = kcount < 256u ? kcount : 256u;
  const int64_t sigma0 = sig[0];
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const InstPtrs ip = instance_ptrs(d, ws, blk >> chunks_sh, sigma0);
    const uint32_t chunk = (uint32_t)(blk & (((int64_t)1 << chunks_sh) - 1));
    const uint32_t m = (chunk << mb) + mloc;
    const uint64_t pa = ip.pa, pb = ip.pb;
    const uint32_t om = tlook(tab + TAB_AM * kTabSize, m);
    float2 acc[NB];
#pragma unroll
    for (int n = 0; n < NB; ++n) acc[n] = make_float2(0.f, 0.f);
    for (uint32_t kh = 0; kh < (kcount >> 8) + (kcount < 256u ? 1u : 0u); ++kh) {
      const uint32_t ba = om + tab[TAB_AK * kTabSize + 256 + (kh & 255u)] +
                          tab[TAB_AK * kTabSize + 512 + ((kh >> 8) & 255u)] + tab[TAB_AK * kTabSize + 768 + (kh >> 16)];
      const uint32_t bb = tab[TAB_BK * kTabSize + 256 + (kh & 255u)] +
                          tab[TAB_BK * kTabSize + 512 + ((kh >> 8) & 255u)] + tab[TAB_BK * kTabSize + 768 + (kh >> 16)];
      uint32_t kl = grp;
      for (; kl + 7 * KS < klo_n; kl += 8 * KS) {
        float2 a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = ldop<FL, 1>(pa, ba + kofa[kl + u * KS]);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          uint32_t ob = bb + kofb[kl + u * KS];
          if constexpr (KS1) ob = __builtin_amdgcn_readfirstlane(ob);
#pragma unroll
          for (int n = 0; n < NB; ++n) cmac(acc[n], a[u], ldop<FL, 2>(pb, ob + tbn[n]));
        }
      }
      for (; kl < klo_n; kl += KS) {
        const float2 a = ldop<FL, 1>(pa, ba + kofa[kl]);
        const uint32_t ob = bb + kofb[kl];
#pragma unroll
        for (int n = 0; n < NB; ++n) cmac(acc[n], a, ldop<FL, 2>(pb, ob + tbn[n]));
      }
    }
    const OutScale s = out_scale<FL>(d, ws, ip.ai, ip.bi);
    float mx = 0.f;
    if (KS > 1) {
#pragma unroll
      for (int n = 0; n < NB; ++n) part[tid * NB + n] = acc[n];
      __syncthreads();
      if (grp == 0) {
        for (int g = 1; g < KS; ++g)
#pragma unroll
          for (int n = 0; n < NB; ++n) {
            const float2 v = part[(g * M + mloc) * NB + n];
            acc[n].x += v.x;
            acc[n].y += v.y;
          }
      }
    }
    if (grp == 0) {
      const uint32_t oc = tlook(tab + TAB_CM * kTabSize, m);
#pragma unroll
      for (int n = 0; n < NB; ++n) mx = fmaxf(mx, put<FL>(ip.pc, oc + tcn[n], acc[n], s));
    }
    block_record<FL>(d, ws, ip.inst, s, mx, red, chunk == 0);
    if (KS > 1) __syncthreads();  // part[] is rewritten next iteration
  }
}

template <int FL>
__global__ __launch_bounds__(256) void k_generic(NodeDesc d, uint64_t ws, const int64_t* __restrict__ sig) {
  const gptr<const uint32_t> tab = gmem<const uint32_t>(ws + d.tab_off);
  const int cb = d.mbits + d.nbits;
  const int64_t total = d.n_inst << cb;
  const int64_t sigma0 = sig[0];
  const uint64_t kcount = (uint64_t)1 << d.kbits;
  // lanes of one instance are contiguous: the output maximum is reduced
  // within segments of a wave before its one atomic
  const int seg = cb >= 6 ? 64 : (1 << cb);
  for (int64_t base = (int64_t)blockIdx.x * 256; base < total; base += (int64_t)gridDim.x * 256) {
    const int64_t g = base + threadIdx.x;
    const bool live = g < total;
    float mx = 0.f;
    OutScale s{1.f, 0};
    int64_t inst = 0;
    if (live) {
      inst = g >> cb;
      const uint64_t mn = (uint64_t)g & (((uint64_t)1 << cb) - 1);
      const uint32_t m = (uint32_t)(mn & (((uint64_t)1 << d.mbits) - 1));
      const uint32_t n = (uint32_t)(mn >> d.mbits);
      const InstPtrs ip = instance_ptrs(d, ws, inst, sigma0);
      const uint32_t oa = tlook(tab + TAB_AM * kTabSize, m);
      const uint32_t ob = tlook(tab + TAB_BN * kTabSize, n);
      float2 c = make_float2(0.f, 0.f);
      for (uint64_t k = 0; k < kcount; ++k) {
        const uint32_t kk = (uint32_t)k;
        cmac(c, ldop<FL, 1>(ip.pa, oa + tlook(tab + TAB_AK * kTabSize, kk)),
             ldop<FL, 2>(ip.pb, ob + tlook(tab + TAB_BK * kTabSize, kk)));
      }
      s = out_scale<FL>(d, ws, ip.ai, ip.bi);
      mx = put<FL>(ip.pc, tlook(tab + TAB_CM * kTabSize, m) + tlook(tab + TAB_CN * kTabSize, n), c, s);
    }
    if constexpr ((FL & kMixBit) != 0) {
      mx = segment_max(mx, seg);
      const int lane = threadIdx.x & 63;
      if (live && (lane & (seg - 1)) == 0)
        record_scale<FL>(d, ws, inst, s, mx, ((uint64_t)g & (((uint64_t)1 << cb) - 1)) == 0);
    }
  }
}

// ---------------------------------------------------------------------------
// dispatch

template <int FL, int KB>
static hipError_t launch_small(const NodeDesc& d, uint64_t ws, const int64_t* sig, hipStream_t st) {
  if (d.mbits >= 8) {
    // R m-chunks per lane: as many as the instance allows, up to 4 (2 when
    // K is 16, to bound registers)
    constexpr int RMAX = KB >= 16 ? 2 : 4;
    const int extra = d.mbits - 8;
    if (RMAX >= 4 && extra >= 2) {
      const int64_t blocks = d.n_inst << (d.mbits - 10);
      hipLaunchKernelGGL((k_wide<FL, KB, 4>), dim3(grid_for(blocks)), dim3(256), 0, st, d, ws, sig);
    } else if (extra >= 1) {
      const int64_t blocks = d.n_inst << (d.mbits - 9);
      hipLaunchKernelGGL((k_wide<FL, KB, 2>), dim3(grid_for(blocks)), dim3(256), 0, st, d, ws, sig);
    } else {
      const int64_t blocks = d.n_inst;
      hipLaunchKernelGGL((k_wide<FL, KB, 1>), dim3(grid_for(blocks)), dim3(256), 0, st, d, ws, sig);
    }
  } else {
    const int64_t blocks = ((d.n_inst << d.mbits) + 255) / 256;
    hipLaunchKernelGGL((k_narrow<FL, KB>), dim3(grid_for(blocks)), dim3(256), 0, st, d, ws, sig);
  }
  return hipGetLastError();
}

template <int FL>
static hipError_t launch_kred(const NodeDesc& d, uint64_t ws, const int64_t* sig, hipStream_t st) {
  const int mb = d.mbits < 8 ? d.mbits : 8;
  const int64_t blocks = d.n_inst << (d.mbits - mb);
  const dim3 g(grid_for(blocks)), b(256);
  if (d.mbits >= 8) {
    switch (d.nbits) {
      case 0: hipLaunchKernelGGL((k_kred<FL, 1, true>), g, b, 0, st, d, ws, sig); break;
      case 1: hipLaunchKernelGGL((k_kred<FL, 2, true>), g, b, 0, st, d, ws, sig); break;
      case 2: hipLaunchKernelGGL((k_kred<FL, 4, true>), g, b, 0, st, d, ws, sig); break;
      case 3: hipLaunchKernelGGL((k_kred<FL, 8, true>), g, b, 0, st, d, ws, sig); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (d.nbits) {
      case 0: hipLaunchKernelGGL((k_kred<FL, 1, false>), g, b, 0, st, d, ws, sig); break;
      case 1: hipLaunchKernelGGL((k_kred<FL, 2, false>), g, b, 0, st, d, ws, sig); break;
      case 2: hipLaunchKernelGGL((k_kred<FL, 4, false>), g, b, 0, st, d, ws, sig); break;
      case 3: hipLaunchKernelGGL((k_kred<FL, 8, false>), g, b, 0, st, d, ws, sig); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <int FL>
static hipError_t launch_stream_fl(const NodeDesc& d, uint64_t ws, const int64_t* sig, hipStream_t st) {
  if (d.n_inst == 0) return hipSuccess;
  if (d.kbits <= 4 && d.nbits <= 4) {
    switch (d.kbits) {
      case 0: return launch_small<FL, 1>(d, ws, sig, st);
      case 1: return launch_small<FL, 2>(d, ws, sig, st);
      case 2: return launch_small<FL, 4>(d, ws, sig, st);
      case 3: return launch_small<FL, 8>(d, ws, sig, st);
      case 4: return launch_small<FL, 16>(d, ws, sig, st);
    }
  }
  if (d.nbits <= 3) return launch_kred<FL>(d, ws, sig, st);
  const int64_t blocks = ((d.n_inst << (d.mbits + d.nbits)) + 255) / 256;
  hipLaunchKernelGGL((k_generic<FL>), dim3(grid_for(blocks)), dim3(256), 0, st, d, ws, sig);
  return hipGetLastError();
}

hipError_t launch_stream(const NodeDesc& d, uint64_t ws, const int64_t* sig, hipStream_t st) {
  return launch_stream_fl<0>(d, ws, sig, st);
}

// complex-half plans: the storage combinations a plan produces (an FP32
// output only comes from FP32 operands: the stem)
hipError_t launch_stream_h(const NodeDesc& d, uint64_t ws, const int64_t* sig, hipStream_t st) {
  const int fl = (d.A.half ? 1 : 0) | (d.B.half ? 2 : 0) | (d.c_half ? 4 : 0);
  switch (fl) {
    case 0: return launch_stream_fl<kMixBit | 0>(d, ws, sig, st);
    case 1: return launch_stream_fl<kMixBit | 1>(d, ws, sig, st);
    case 2: return launch_stream_fl<kMixBit | 2>(d, ws, sig, st);
    case 3: return launch_stream_fl<kMixBit | 3>(d, ws, sig, st);
    case 4: return launch_stream_fl<kMixBit | 4>(d, ws, sig, st);
    case 5: return launch_stream_fl<kMixBit | 5>(d, ws, sig, st);
    case 6: return launch_stream_fl<kMixBit | 6>(d, ws, sig, st);
    case 7: return launch_stream_fl<kMixBit | 7>(d, ws, sig, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace matnc
