// complex64 kernels of the contraction path (gfx950).
//
//  * k_mfma: one pairwise step C[m, n] = sum_k A[m, k] B[k, n] with large N
//    and K (the streaming kernels of kernels_stream.hip take the rest): a
//    complex GEMM on
//    v_mfma_f32_32x32x2f32 through the real embedding
//    [Ar Ai] x [[Br, Bi], [-Bi, Br]] = [Cr Ci] (8 real flops per complex
//    MAC, so MFMA flops equal complex flops), LDS-staged, double-buffered
//    tiles, with the bit permutation of each operand folded into its tile
//    loads through the offset tables of desc.h.  M runs along the MFMA
//    column (lane-contiguous) so output stores are coalesced along m.
//    Steps with few columns whose A instance is shared by several output
//    instances (a node of the reuse tree whose operand is gathered for many
//    keys) run as fan-out tiles: the instances that read one A instance
//    fill the columns of one tile, so each A tile is loaded once for all.
//  * k_slice_sum: FP64 accumulation of the root instances into the caller's
//    amplitudes, slices added one by one in slice-id order.
//  * k_xeb: deterministic FP64 sum of |a|^2 and the linear XEB estimate.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "desc.h"
#include "device_common.h"
#include "kernels.h"

namespace matnc {

// ---------------------------------------------------------------------------
// MFMA complex GEMM

typedef float floatx16 __attribute__((ext_vector_type(16)));

// An operand's staged element: an FP32 pair, or (complex-half plans, whose
// FP32 steps may read an FP16-stored child) a half2 word converted exactly to
// FP32 and multiplied by the instance's power of two 2^e.
template <bool H>
struct FStage;
template <>
struct FStage<false> {
  typedef f32x2 type;
  static __device__ __forceinline__ type load(uint64_t base, uint32_t i) { return gmem<const f32x2>(base)[i]; }
  static __device__ __forceinline__ float2 val(type r, float) { return make_float2(r.x, r.y); }
};
template <>
struct FStage<true> {
  typedef uint32_t type;
  static __device__ __forceinline__ type load(uint64_t base, uint32_t i) { return ldg_u32(base, i); }
  static __device__ __forceinline__ float2 val(type r, float c) {
    __half2 h;
    __builtin_memcpy(&h, &r, 4);
    const float2 v = __half22float2(h);
    return make_float2(v.x * c, v.y * c);
  }
};

// Tile: TM = 32*RM*WM values of m, TN = 16*RN*WN complex n, TK complex k.
// FAN: the tile's TN columns are TN >> nbits slots of 2^nbits columns, one
// per output instance of a fan-table row (see NodeDesc); the A tile is
// loaded once for all of them.
// REC (fan tiles only): also record each output instance's largest
// |component| into its scale slot (complex-half plans, whose FP32 branch
// tensors feed FP16 steps): half-wave reductions and one LDS atomic per
// slot column, one global atomic per slot and tile.
// HA, HB (complex-half plans only): A, B stored in FP16 with a per-instance
// exponent; the output is FP32 either way.
template <int RM, int RN, int WM, int WN, int TK, bool FAN, bool REC = false, bool HA = false, bool HB = false>
__global__ __launch_bounds__(64 * WM * WN) void k_mfma(NodeDesc d, uint64_t ws, const int64_t* __restrict__ sig) {
  static_assert(!REC || FAN, "maxima are recorded by fan-out tiles only");
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = 32 * RM * WM;
  constexpr int TN = 16 * RN * WN;
  constexpr int EA = TK * TM / NT;
  constexpr int EB = TK * TN / NT;
  static_assert(EA * NT == TK * TM && EB * NT == TK * TN, "tile must split evenly over threads");
  constexpr int APL = TK * TM + 32;        // plane stride (floats), padded
  constexpr int BPL = TK * TN + 16;
  // third B plane (-Bi) at 16 words mod 32 like the second, so that the two
  // planes a half-wave reads (0 and BPL, or BP2 and 0) sit in different banks
  constexpr int BP2 = 2 * BPL + 16;
  __shared__ float As[2][2 * APL];
  __shared__ float Bs[2][BP2 + BPL];  // planes Br, Bi, -Bi
  // per-tile column data, shared by the waves instead of held per lane:
  // the C offset of each of the tile's TN columns, and for fan tiles the
  // B instance (byte offset) and output instance base of each slot
  __shared__ uint32_t s_cn[TN];
  __shared__ uint64_t s_bb[FAN ? TN : 1];
  __shared__ uint64_t s_cb[FAN ? TN : 1];
  __shared__ uint32_t s_mx[REC ? TN : 1];  // per-slot maxima (float bits)
  __shared__ float s_fb[(FAN && HB) ? TN : 1];  // per-slot factor 2^e of an FP16 B

  const gptr<const uint32_t> tab = gmem<const uint32_t>(ws + d.tab_off);
  const cptr<const uint32_t> ctab = cmem<const uint32_t>(ws + d.tab_off);  // k-step lookups
  const gptr<const int32_t> glA = gmem<const int32_t>(ws + d.A.gmap_off);
  const gptr<const int32_t> glB = gmem<const int32_t>(ws + d.B.gmap_off);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM;
  const int wn = wave / WM;

  const int64_t mt_count = (int64_t)1 << (d.mbits - __builtin_ctz(TM));
  const int64_t nt_count = FAN ? 1 : (int64_t)1 << (d.nbits - __builtin_ctz(TN));
  const int64_t tiles = mt_count * nt_count;
  const int ksteps = 1 << (d.kbits - __builtin_ctz(TK));
  const int64_t sigma0 = sig[0];
  // work units: output instances, or (slice, fan row) pairs
  const int64_t units = FAN ? (d.n_inst / d.w) * d.n_fan : d.n_inst;
  const gptr<const int32_t> fan = gmem<const int32_t>(ws + d.fan_off);
  const uint32_t nmask = (1u << d.nbits) - 1u;
  const int slots = FAN ? (TN >> d.nbits) : 1;

  for (int64_t blk = blockIdx.x; blk < units * tiles; blk += gridDim.x) {
    // logical tile order: n tiles innermost (they share the A tile), then m
    // tiles, then instances / fan rows (fan rows in blocks, see unit_tile);
    // each XCD takes a contiguous range
    const int64_t lt = xcd_tile(blk, units * tiles);
    int64_t u, t;
    unit_tile(lt, units, tiles, d.fan_rows > 0 ? (int64_t)d.fan_rows : (FAN ? 2 : 1), u, t);
    const uint32_t m0 = (uint32_t)((t / nt_count) * TM);
    const uint32_t n0 = (uint32_t)((t % nt_count) * TN);
    int64_t s, j;
    gptr<const int32_t> fj = nullptr;
    if (FAN) {
      s = d.dep ? u / d.n_fan : 0;
      fj = fan + (u - s * d.n_fan) * slots;
      j = fj[0];
    } else {
      s = d.dep ? u / d.w : 0;
      j = d.dep ? u - s * d.w : u;
    }
    const int64_t inst = s * d.w + j;  // output instance (slot 0 for fan tiles)
    const int64_t sigma = sigma0 + s;
    const int64_t ai = operand_instance(d.A, glA, j, s, sigma);
    const int64_t bi = operand_instance(d.B, glB, j, s, sigma);
    const uint64_t pa = ws + d.A.off + ai * d.A.inst_bytes;
    const uint64_t pb = ws + d.B.off + bi * d.B.inst_bytes;
    const gptr<f32x2> pc = gmem<f32x2>(ws + d.c_off + inst * d.c_inst_bytes);
    const float ca = HA ? ldexpf(1.f, ldg_scale(ws + d.A.scale_off, ai).e) : 1.f;
    const float cb = HB ? ldexpf(1.f, ldg_scale(ws + d.B.scale_off, bi).e) : 1.f;
    if (tid < TN) s_cn[tid] = tlook(tab + TAB_CN * kTabSize, FAN ? (tid & nmask) : n0 + tid);
    if (FAN && tid < slots) {
      // an empty slot reads slot 0's B into columns that are never stored
      const int jg = fj[tid];
      const int64_t bg = operand_instance(d.B, glB, jg < 0 ? j : jg, s, sigma);
      s_bb[tid] = d.B.off + bg * d.B.inst_bytes;
      s_cb[tid] = jg < 0 ? 0 : d.c_off + (uint64_t)(s * d.w + jg) * d.c_inst_bytes;
      if (REC) s_mx[tid] = 0u;
      if (HB) s_fb[tid] = ldexpf(1.f, ldg_scale(ws + d.B.scale_off, bg).e);
    }
    __syncthreads();  // the column data above is read by every wave

    // per-thread load coordinates (fixed across k steps)
    uint32_t aoff[EA], boff[EB];
    int akk[EA], bkk[EB], amm[EA], bnn[EB];
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int flat = e * NT + tid;
      amm[e] = flat % TM;
      akk[e] = flat / TM;
      aoff[e] = tlook(tab + TAB_AM * kTabSize, m0 + amm[e]) + tab[TAB_AK * kTabSize + akk[e]];
    }
    uint64_t pbe[EB];  // B instance of each element (fan tiles: its slot's)
    float cbe[EB];     // and its factor (FP16 B)
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int flat = e * NT + tid;
      bnn[e] = flat % TN;
      bkk[e] = flat / TN;
      if (FAN) {
        pbe[e] = ws + s_bb[bnn[e] >> d.nbits];
        cbe[e] = HB ? s_fb[bnn[e] >> d.nbits] : 1.f;
        boff[e] = tlook(tab + TAB_BN * kTabSize, bnn[e] & nmask) + tab[TAB_BK * kTabSize + bkk[e]];
      } else {
        pbe[e] = pb;
        cbe[e] = cb;
        boff[e] = tlook(tab + TAB_BN * kTabSize, n0 + bnn[e]) + tab[TAB_BK * kTabSize + bkk[e]];
      }
    }
    typename FStage<HA>::type ra[EA];
    typename FStage<HB>::type rb[EB];
    auto gload = [&](uint32_t kba, uint32_t kbb) {
#pragma unroll
      for (int e = 0; e < EA; ++e) ra[e] = FStage<HA>::load(pa, aoff[e] + kba);
#pragma unroll
      for (int e = 0; e < EB; ++e) rb[e] = FStage<HB>::load(pbe[e], boff[e] + kbb);
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        const float2 v = FStage<HA>::val(ra[e], ca);
        As[buf][akk[e] * TM + amm[e]] = v.x;
        As[buf][APL + akk[e] * TM + amm[e]] = v.y;
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        const float2 v = FStage<HB>::val(rb[e], cbe[e]);
        Bs[buf][bkk[e] * TN + bnn[e]] = v.x;
        Bs[buf][BPL + bkk[e] * TN + bnn[e]] = v.y;
        Bs[buf][BP2 + bkk[e] * TN + bnn[e]] = -v.y;
      }
    };

    floatx16 acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
      for (int q = 0; q < RN; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][q][r] = 0.f;

    const int half = lane >> 5;     // 0: real part row of the embedding, 1: imaginary
    const int l32 = lane & 31;
    const int dsel = l32 & 1;       // 0: real column, 1: imaginary column
    const int ncol = l32 >> 1;
    // which B plane feeds this lane, and with which sign
    // (half, dsel): (0,0) -> Br, (0,1) -> Bi, (1,0) -> -Bi, (1,1) -> Br, each
    // read from its own plane so that no sign flip sits between the LDS
    // read and the MFMA
    const int bplane = (half ^ dsel) ? (half ? BP2 : BPL) : 0;
    const int aplane = half ? APL : 0;

    // output offsets of this lane's m values, fetched before the k loop
    uint32_t om[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) om[i] = tlook(tab + TAB_CM * kTabSize, m0 + (wm * RM + i) * 32 + l32);

    // k offsets run one step ahead of the loads that use them, so that their
    // table reads are in flight during a whole step of MFMA work
    uint32_t kba = tlook(ctab + TAB_AK * kTabSize, 0u), kbb = tlook(ctab + TAB_BK * kTabSize, 0u);
    gload(kba, kbb);
    if (ksteps > 1) {
      kba = tlook(ctab + TAB_AK * kTabSize, (uint32_t)TK);
      kbb = tlook(ctab + TAB_BK * kTabSize, (uint32_t)TK);
    }
    lstore(0);
    __syncthreads();
    for (int ks = 0; ks < ksteps; ++ks) {
      const int buf = ks & 1;
      if (ks + 1 < ksteps) {
        gload(kba, kbb);
        if (ks + 2 < ksteps) {
          kba = tlook(ctab + TAB_AK * kTabSize, (uint32_t)(ks + 2) * TK);
          kbb = tlook(ctab + TAB_BK * kTabSize, (uint32_t)(ks + 2) * TK);
        }
      }
#pragma unroll
      for (int kk = 0; kk < TK; ++kk) {
        float yv[RM], xv[RN];
#pragma unroll
        for (int i = 0; i < RM; ++i) yv[i] = As[buf][aplane + kk * TM + (wm * RM + i) * 32 + l32];
#pragma unroll
        for (int q = 0; q < RN; ++q) xv[q] = Bs[buf][bplane + kk * TN + (wn * RN + q) * 16 + ncol];
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
          for (int q = 0; q < RN; ++q)
            acc[i][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(xv[q], yv[i], acc[i][q], 0, 0, 0);
      }
      if (ks + 1 < ksteps) lstore(buf ^ 1);
      __syncthreads();
    }

    // epilogue: lane holds C[m][n] (re, im) in registers (r, r+1), r even
#pragma unroll
    for (int q = 0; q < RN; ++q) {
#pragma unroll
      for (int rr = 0; rr < 8; ++rr) {
        const int r = 2 * rr;
        const int row = 8 * (rr >> 1) + 4 * half + 2 * (rr & 1);
        const int nl = (wn * RN + q) * 16 + (row >> 1);  // column within the tile
        gptr<f32x2> dst = pc;
        bool live = true;
        if (FAN) {
          const uint64_t cb = s_cb[nl >> d.nbits];  // uniform over the 32 lanes of a half-wave (one n)
          live = cb != 0;
          dst = gmem<f32x2>(ws + cb);
        }
        const uint32_t ocn = s_cn[nl];
        float v = 0.f;
#pragma unroll
        for (int i = 0; i < RM; ++i) {
          if (live) dst[om[i] + ocn] = f32x2{acc[i][q][r], acc[i][q][r + 1]};
          if (REC) v = fmaxf(v, fmaxf(fabsf(acc[i][q][r]), fabsf(acc[i][q][r + 1])));
        }
        if (REC) {
          // the half-wave's 32 lanes hold 32 values of m of one column
#pragma unroll
          for (int o = 16; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
          if (l32 == 0 && live) atomicMax(&s_mx[nl >> d.nbits], __float_as_uint(v));
        }
      }
    }
    if (REC) {
      __syncthreads();
      if (tid < slots) {
        const int jg = fj[tid];
        if (jg >= 0 && s_mx[tid] > 0u) max_scale_mx(ws + d.c_scale_off, s * d.w + jg, s_mx[tid]);
      }
    }
    __syncthreads();  // the next tile rewrites the column data
  }
}

// ---------------------------------------------------------------------------
// reductions

__global__ __launch_bounds__(256) void k_slice_sum(OpDesc root, uint64_t ws, const int64_t* __restrict__ sig,
                                                   int nb, int64_t nrows, const int32_t* __restrict__ rows,
                                                   int open_bits, double2* __restrict__ amps) {
  const gptr<const int32_t> gmap = gmem<const int32_t>(ws + root.gmap_off);
  const int64_t total = nrows << open_bits;
  const int64_t sigma0 = sig[0];
  const int64_t omask = ((int64_t)1 << open_bits) - 1;
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total; g += (int64_t)gridDim.x * 256) {
    const int64_t rp = g >> open_bits;
    const int64_t o = g & omask;
    const int64_t dst = ((int64_t)rows[rp] << open_bits) + o;
    double2 acc = amps[dst];
    for (int s = 0; s < nb; ++s) {
      const int64_t inst = operand_instance(root, gmap, rp, s, sigma0 + s);
      const float2 v = ldg_f2(ws + root.off + inst * root.inst_bytes, o);
      acc.x += (double)v.x;
      acc.y += (double)v.y;
    }
    amps[dst] = acc;
  }
}

__global__ __launch_bounds__(1024) void k_xeb(const double2* __restrict__ amps, int64_t count, int n_qubits,
                                              double* __restrict__ out) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 1024) {
    const double2 a = amps[i];
    acc += a.x * a.x + a.y * a.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = ldexp(red[0] / (double)count, n_qubits) - 1.0;
}

__global__ void k_set_i64(int64_t* p, int64_t v) {
  if (threadIdx.x == 0) p[0] = v;
}

// ---------------------------------------------------------------------------
// launchers

struct MfmaCfg {
  int tm_bits, tn_bits, tk_bits;
};

static const MfmaCfg kMfmaCfgs[] = {
    {7, 5, 3},  // 0: RM=2 RN=1 WM=2 WN=2, TK=8  -> TM=128, TN=32
    {7, 6, 3},  // 1: RM=2 RN=2 WM=2 WN=2, TK=8  -> TM=128, TN=64
    {6, 5, 3},  // 2: RM=1 RN=1 WM=2 WN=2, TK=8  -> TM=64,  TN=32
    {8, 5, 3},  // 3: RM=4 RN=1 WM=2 WN=2, TK=8  -> TM=256, TN=32
    {8, 6, 3},  // 4: RM=4 RN=2 WM=2 WN=2, TK=8  -> TM=256, TN=64
    {7, 7, 3},  // 5: RM=2 RN=4 WM=2 WN=2, TK=8  -> TM=128, TN=128
};

int mfma_config_count() { return (int)(sizeof(kMfmaCfgs) / sizeof(kMfmaCfgs[0])); }

bool mfma_config_fits(int cfg, int mbits, int nbits, int kbits) {
  if (cfg < 0 || cfg >= mfma_config_count()) return false;
  const MfmaCfg& c = kMfmaCfgs[cfg];
  return mbits >= c.tm_bits && nbits >= c.tn_bits && kbits >= c.tk_bits;
}

int mfma_config_tn(int cfg) { return cfg < 0 || cfg >= mfma_config_count() ? 0 : 1 << kMfmaCfgs[cfg].tn_bits; }

bool mfma_fan_config_fits(int cfg, int mbits, int nbits, int kbits, int fan_tn) {
  if (cfg < 0 || cfg >= mfma_config_count()) return false;
  const MfmaCfg& c = kMfmaCfgs[cfg];
  return (1 << c.tn_bits) == fan_tn && nbits < c.tn_bits && mbits >= c.tm_bits && kbits >= c.tk_bits;
}

template <bool FAN, bool REC, bool HA, bool HB>
static hipError_t launch_mfma_s(const NodeDesc& d, int cfg, unsigned grid, uint64_t ws, const int64_t* sig,
                                hipStream_t st) {
  switch (cfg) {
    case 0: hipLaunchKernelGGL((k_mfma<2, 1, 2, 2, 8, FAN, REC, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 1: hipLaunchKernelGGL((k_mfma<2, 2, 2, 2, 8, FAN, REC, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 2: hipLaunchKernelGGL((k_mfma<1, 1, 2, 2, 8, FAN, REC, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 3: hipLaunchKernelGGL((k_mfma<4, 1, 2, 2, 8, FAN, REC, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 4: hipLaunchKernelGGL((k_mfma<4, 2, 2, 2, 8, FAN, REC, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 5:
      if (FAN) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_mfma<2, 4, 2, 2, 8, false, false, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool FAN, bool REC = false>
static hipError_t launch_mfma_t(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st) {
  if (d.n_inst == 0) return hipSuccess;
  const bool fits = FAN ? mfma_fan_config_fits(cfg, d.mbits, d.nbits, d.kbits, d.fan_tn)
                        : mfma_config_fits(cfg, d.mbits, d.nbits, d.kbits);
  if (!fits || (FAN && (d.w <= 0 || d.n_fan <= 0))) return hipErrorInvalidValue;
  const MfmaCfg& c = kMfmaCfgs[cfg];
  const int64_t units = FAN ? (d.n_inst / d.w) * d.n_fan : d.n_inst;
  const int64_t tiles = ((int64_t)1 << (d.mbits - c.tm_bits)) * (FAN ? 1 : ((int64_t)1 << (d.nbits - c.tn_bits)));
  const unsigned grid = grid_for(units * tiles);
  // FP16-stored operands occur only in complex-half plans
  if (d.A.half) {
    if (d.B.half) return launch_mfma_s<FAN, REC, true, true>(d, cfg, grid, ws, sig, st);
    return launch_mfma_s<FAN, REC, true, false>(d, cfg, grid, ws, sig, st);
  }
  if (d.B.half) return launch_mfma_s<FAN, REC, false, true>(d, cfg, grid, ws, sig, st);
  return launch_mfma_s<FAN, REC, false, false>(d, cfg, grid, ws, sig, st);
}

hipError_t launch_mfma(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st) {
  return launch_mfma_t<false>(d, cfg, ws, sig, st);
}

hipError_t launch_mfma_fan(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st) {
  return launch_mfma_t<true>(d, cfg, ws, sig, st);
}

hipError_t launch_mfma_fan_rec(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st) {
  return launch_mfma_t<true, true>(d, cfg, ws, sig, st);
}

hipError_t launch_slice_sum(const OpDesc& root, uint64_t ws, const int64_t* sig, int nb, int64_t nrows,
                            const int32_t* rows, int open_bits, double* amps, hipStream_t st) {
  const int64_t total = nrows << open_bits;
  if (total == 0 || nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_sum, dim3(grid_for((total + 255) / 256)), dim3(256), 0, st, root, ws, sig, nb, nrows,
                     rows, open_bits, reinterpret_cast<double2*>(amps));
  return hipGetLastError();
}

hipError_t launch_xeb(const double* amps, int64_t count, int n_qubits, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_xeb, dim3(1), dim3(1024), 0, st, reinterpret_cast<const double2*>(amps), count, n_qubits, out);
  return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

}  // namespace matnc
