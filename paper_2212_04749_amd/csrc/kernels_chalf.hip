// complex-half kernels: FP16 (re, im) storage with a per-instance power-of-two
// exponent, FP16 MFMA with FP32 accumulation.
//
//  * k_mfma_h: C[m, n] = sum_k A[m, k] B[k, n] with an FP16 output, on
//    gfx950's v_mfma_f32_32x32x16_f16 through the real embedding
//    [Ar Ai] x [[Br, Bi], [-Bi, Br]]: each instruction covers eight complex
//    k.  For its column m a lane supplies (Ar, Ai) of four consecutive k --
//    exactly four stored half2 values, one 16-byte LDS read -- and for its
//    row 2n + d it supplies (Br, -Bi) (d = 0) or (Bi, Br) (d = 1) of the
//    same four k.  The products of FP16 inputs are exact in the FP32
//    accumulator; the output is multiplied by 2^(15 - ex), ex = ceil of
//    log2 of the bound 2^(kbits+1) mx_A mx_B, stored as FP16 below 2^15, and
//    its measured maximum recorded for the next step.  An operand stored in
//    FP32 (leaves and stem tensors of the plan) is scaled by a power of two
//    and rounded to FP16 as it is loaded.
//  * k_slice_sum_h: FP64 sum of half * 2^e over slices, in slice order.
//  * k_zero: clears the scale slots of a launch sequence (a kernel rather
//    than a memset so that it can live inside a captured graph).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "desc.h"
#include "device_common.h"
#include "kernels.h"

namespace matnc {

bool chalf_available() { return true; }

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint32_t h2bits(__half2 h) {
  uint32_t u;
  __builtin_memcpy(&u, &h, 4);
  return u;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// four output words at word offset i (a multiple of 4) as one 16-byte store
__device__ __forceinline__ void stg_u32x4(uint64_t base, uint64_t i, u32x4 v) { gmem<u32x4>(base)[i >> 2] = v; }
// two output words at word offset i (even) as one 8-byte store
__device__ __forceinline__ void stg_u32x2(uint64_t base, uint64_t i, u32x2 v) { gmem<u32x2>(base)[i >> 1] = v; }

// an FP32 (re, im) pair as half2 bits, scaled by c and rounded to nearest
__device__ __forceinline__ uint32_t f32pair_to_h2bits(u32x2 raw, float c) {
  return h2bits(__float22half2_rn(make_float2(__uint_as_float(raw.x) * c, __uint_as_float(raw.y) * c)));
}

// an operand's staged elements: one half2 word (FP16 storage) or two FP32
// words
template <bool H>
struct AStage;
template <>
struct AStage<true> {
  typedef uint32_t type;
  static __device__ __forceinline__ type load(uint64_t base, uint32_t i) { return ldg_u32(base, i); }
  static __device__ __forceinline__ uint32_t bits(type r, float) { return r; }
};
template <>
struct AStage<false> {
  typedef u32x2 type;
  static __device__ __forceinline__ type load(uint64_t base, uint32_t i) { return gmem<const u32x2>(base)[i]; }
  static __device__ __forceinline__ uint32_t bits(type r, float c) { return f32pair_to_h2bits(r, c); }
};

// TM = 32*RM*WM values of m, TN = 16*RN*WN complex n, TK complex k (multiple of 8)
// FAN: fan-out tiles as in k_mfma (desc.h): the TN columns are slots of
// 2^nbits columns, one per output instance sharing the A instance; every
// slot has its own B scale, output exponent and recorded maximum.
// HA, HB: A, B stored in FP16 (the launcher picks the instance from the
// step, so that the loads carry no storage branches).
// Per-column data (C column offsets; for fan tiles each slot's output base,
// factors and exponent) is kept in LDS, shared by the waves, rather than in
// per-lane registers.
// Operand staging works on quads: a thread loads four consecutive k of one m
// (of A) or of one n (of B) and writes them to LDS as one 16-byte store.
template <int RM, int RN, int WM, int WN, int TK, bool FAN, bool HA, bool HB>
__global__ __launch_bounds__(64 * WM * WN) void k_mfma_h(NodeDesc d, uint64_t ws, const int64_t* __restrict__ sig) {
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = 32 * RM * WM;
  constexpr int TN = 16 * RN * WN;
  static_assert(TK % 8 == 0, "eight complex k per instruction");
  constexpr int QA = (TK / 4) * TM;  // k quads of the A tile
  constexpr int QB = (TK / 4) * TN;  // ... and of the B tile
  static_assert(QA % NT == 0, "A quads must split evenly over threads");
  static_assert(QB % NT == 0 || NT % QB == 0, "B quads must split evenly over threads, or fit in fewer");
  constexpr int EQA = QA / NT;
  constexpr int EQB = QB >= NT ? QB / NT : 1;
  constexpr bool BPART = QB < NT;  // only threads tid < QB stage B
  // LDS tiles in the register layout of the MFMA operands: As[k/4][m][k%4]
  // holds A's half2 (re, im); Bs[k/4][n][d][k%4] holds B's column pair of
  // the real embedding, (re, -im) for d = 0 and (im, re) for d = 1
  constexpr int AQ = 4 * TM + 16;  // u32 per k quad (padded)
  __shared__ __attribute__((aligned(16))) uint32_t As[2][(TK / 4) * AQ];
  __shared__ __attribute__((aligned(16))) uint32_t Bs[2][(TK / 4) * TN * 8];
  // C offset of each of the tile's TN columns; fan-out slots: output base
  // (workspace offset, 0 = empty slot), output factor, output exponent,
  // FP32-load factor of B, recorded maximum (float bits)
  __shared__ uint32_t s_cn[TN];
  __shared__ uint64_t s_cbase[FAN ? TN : 1];
  __shared__ float s_f[FAN ? TN : 1];
  __shared__ int s_e[FAN ? TN : 1];
  __shared__ float s_fb[FAN ? TN : 1];
  __shared__ uint32_t s_mx[FAN ? TN : 1];

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
  const int half = lane >> 5;
  const int l32 = lane & 31;
  const int dsel = l32 & 1;
  const int ncol = l32 >> 1;
  const int64_t units = FAN ? (d.n_inst / d.w) * d.n_fan : d.n_inst;
  const gptr<const int32_t> fan = gmem<const int32_t>(ws + d.fan_off);
  const uint32_t nmask = (1u << d.nbits) - 1u;
  const int slots = FAN ? (TN >> d.nbits) : 1;
  const uint64_t scB = ws + d.B.scale_off;
  const bool bstage = !BPART || tid < QB;

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
    const int64_t inst = s * d.w + j;
    const int64_t sigma = sigma0 + s;
    const int64_t ai = operand_instance(d.A, glA, j, s, sigma);
    const int64_t bi = operand_instance(d.B, glB, j, s, sigma);
    const uint64_t pa = ws + d.A.off + ai * d.A.inst_bytes;
    const uint64_t pb = ws + d.B.off + bi * d.B.inst_bytes;
    const uint64_t pc = ws + d.c_off + inst * d.c_inst_bytes;
    // operand scales; an FP32 operand is converted on load with a power of two
    // that puts its largest component in [2^13, 2^14)
    const HalfScale sa = ldg_scale(ws + d.A.scale_off, ai);
    const HalfScale sb = ldg_scale(ws + d.B.scale_off, bi);
    int ea = sa.e, eb = sb.e;
    float mxa = __uint_as_float(sa.mx), mxb = __uint_as_float(sb.mx);
    float ca = 1.f, cb = 1.f;
    if (!d.A.half && mxa > 0.f) {
      int ex;
      frexpf(mxa, &ex);
      ea = ex - 14;
      ca = ldexpf(1.f, -ea);
      mxa *= ca;
    }
    if (!d.B.half && mxb > 0.f) {
      int ex;
      frexpf(mxb, &ex);
      eb = ex - 14;
      cb = ldexpf(1.f, -eb);
      mxb *= cb;
    }
    if (tid < TN) s_cn[tid] = tlook(tab + TAB_CN * kTabSize, FAN ? (tid & nmask) : n0 + tid);
    if (FAN) {
      // per-slot scales: B's exponent and load factor, the output exponent
      if (tid < slots) {
        const int jg = fj[tid];
        float f = 0.f, cbg = 1.f;
        int e = 0;
        if (jg >= 0) {
          const HalfScale sg = ldg_scale(scB, operand_instance(d.B, glB, jg, s, sigma));
          int ebg = sg.e;
          float mxbg = __uint_as_float(sg.mx);
          if (!HB && mxbg > 0.f) {
            int ex;
            frexpf(mxbg, &ex);
            ebg = ex - 14;
            cbg = ldexpf(1.f, -ebg);
            mxbg *= cbg;
          }
          const float bound = ldexpf(mxa * mxbg, d.kbits + 1);
          int ex = 0;
          if (bound > 0.f) frexpf(bound, &ex);
          f = ldexpf(1.f, 15 - ex);
          e = ea + ebg + ex - 15;
        }
        s_cbase[tid] = jg < 0 ? 0 : d.c_off + (uint64_t)(s * d.w + jg) * d.c_inst_bytes;
        s_f[tid] = f;
        s_e[tid] = e;
        s_fb[tid] = cbg;
        s_mx[tid] = 0u;
      }
    }
    __syncthreads();  // the column data above is read by every wave

    // quad coordinates: A quad e of this thread covers m = amm[e], k =
    // 4 akq[e] .. 4 akq[e] + 3 of the k step; likewise B quads over n
    uint32_t aoff[EQA][4], boff[EQB][4];
    int akq[EQA], amm[EQA], bkq[EQB], bnn[EQB];
#pragma unroll
    for (int e = 0; e < EQA; ++e) {
      const int flat = e * NT + tid;
      amm[e] = flat % TM;
      akq[e] = flat / TM;
      const uint32_t om_ = tlook(tab + TAB_AM * kTabSize, m0 + amm[e]);
#pragma unroll
      for (int q = 0; q < 4; ++q) aoff[e][q] = om_ + tab[TAB_AK * kTabSize + 4 * akq[e] + q];
    }
    uint64_t pbe[EQB];  // B instance of each quad (fan tiles: its slot's)
    float cbe[EQB];
#pragma unroll
    for (int e = 0; e < EQB; ++e) {
      const int flat = bstage ? e * NT + tid : 0;
      bnn[e] = flat % TN;
      bkq[e] = flat / TN;
      uint32_t on_;
      if (FAN) {
        const int g = bnn[e] >> d.nbits;
        const int jg = fj[g];
        // an empty slot reads slot 0's B into columns that are never stored
        pbe[e] = ws + d.B.off + operand_instance(d.B, glB, jg < 0 ? j : jg, s, sigma) * d.B.inst_bytes;
        cbe[e] = s_fb[g];
        on_ = tlook(tab + TAB_BN * kTabSize, bnn[e] & nmask);
      } else {
        pbe[e] = pb;
        cbe[e] = cb;
        on_ = tlook(tab + TAB_BN * kTabSize, n0 + bnn[e]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) boff[e][q] = on_ + tab[TAB_BK * kTabSize + 4 * bkq[e] + q];
    }
    // raw operand words in flight (an FP32 element, or a half2 in .x); the
    // FP32 -> FP16 conversion happens when the tile is written to LDS, after
    // the MFMA work of the current step, so the loads are not waited for
    // inside the load phase.  S register stages: with two, the loads of k
    // step k + 2 are issued before the MFMA work of step k, so that two
    // steps of MFMA work cover their latency.  Two only for the 8-wave tiles
    // whose second stage still fits two waves per SIMD (FP16 operands); the
    // 4-wave tiles would lose half their occupancy to it.
    constexpr int SW = EQA * 4 * (HA ? 1 : 2) + EQB * 4 * (HB ? 1 : 2);  // words per stage
    constexpr int S = (NT == 512 && SW <= 12) ? 2 : 1;
    typename AStage<HA>::type ra[S][EQA][4];
    typename AStage<HB>::type rb[S][EQB][4];
    auto gload = [&](int st, uint32_t kba, uint32_t kbb) {
#pragma unroll
      for (int e = 0; e < EQA; ++e)
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[st][e][q] = AStage<HA>::load(pa, aoff[e][q] + kba);
      if (bstage) {
#pragma unroll
        for (int e = 0; e < EQB; ++e)
#pragma unroll
          for (int q = 0; q < 4; ++q) rb[st][e][q] = AStage<HB>::load(pbe[e], boff[e][q] + kbb);
      }
    };
    auto lstore = [&](int buf, int st) {
#pragma unroll
      for (int e = 0; e < EQA; ++e) {
        uint4 v;
        v.x = AStage<HA>::bits(ra[st][e][0], ca);
        v.y = AStage<HA>::bits(ra[st][e][1], ca);
        v.z = AStage<HA>::bits(ra[st][e][2], ca);
        v.w = AStage<HA>::bits(ra[st][e][3], ca);
        *reinterpret_cast<uint4*>(&As[buf][akq[e] * AQ + 4 * amm[e]]) = v;
      }
      if (bstage) {
#pragma unroll
        for (int e = 0; e < EQB; ++e) {
          uint32_t lo[4], hi[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const uint32_t h = AStage<HB>::bits(rb[st][e][q], cbe[e]);
            const uint32_t re = h & 0xffffu, im = h >> 16;
            lo[q] = re | ((im ^ 0x8000u) << 16);  // (Br, -Bi)
            hi[q] = im | (re << 16);              // (Bi, Br)
          }
          const int base = ((bkq[e] * TN + bnn[e]) * 2) * 4;
          *reinterpret_cast<uint4*>(&Bs[buf][base]) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
          *reinterpret_cast<uint4*>(&Bs[buf][base + 4]) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
        }
      }
    };

    floatx16 acc[RM][RN];
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
      for (int q = 0; q < RN; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][q][r] = 0.f;
    // the MFMA work of one k step from LDS buffer buf
    auto kstep = [&](int buf) {
#pragma unroll
      for (int g = 0; g < TK / 8; ++g) {
        const int kq = 2 * g + half;  // this lane's quad of complex k
        halfx8 yv[RM], xv[RN];
#pragma unroll
        for (int i = 0; i < RM; ++i) {
          const int m = (wm * RM + i) * 32 + l32;
          yv[i] = *reinterpret_cast<const halfx8*>(&As[buf][kq * AQ + 4 * m]);
        }
#pragma unroll
        for (int q = 0; q < RN; ++q) {
          const int n = (wn * RN + q) * 16 + ncol;
          xv[q] = *reinterpret_cast<const halfx8*>(&Bs[buf][((kq * TN + n) * 2 + dsel) * 4]);
        }
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
          for (int q = 0; q < RN; ++q)
            acc[i][q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(xv[q], yv[i], acc[i][q], 0, 0, 0);
      }
    };

    // output offsets of this lane's m values, fetched before the k loop
    uint32_t om[RM];
#pragma unroll
    for (int i = 0; i < RM; ++i) om[i] = tlook(tab + TAB_CM * kTabSize, m0 + (wm * RM + i) * 32 + l32);

    // stages 0 .. S-1 hold k steps 0 .. S-1; kna, knb: k offsets of the next
    // step to load (S), fetched one load ahead of their use
    gload(0, tlook(ctab + TAB_AK * kTabSize, 0u), tlook(ctab + TAB_BK * kTabSize, 0u));
#pragma unroll
    for (int u = 1; u < S; ++u)
      if (u < ksteps)
        gload(u, tlook(ctab + TAB_AK * kTabSize, (uint32_t)(u * TK)),
              tlook(ctab + TAB_BK * kTabSize, (uint32_t)(u * TK)));
    uint32_t kna = 0, knb = 0;
    if (S < ksteps) {
      kna = tlook(ctab + TAB_AK * kTabSize, (uint32_t)(S * TK));
      knb = tlook(ctab + TAB_BK * kTabSize, (uint32_t)(S * TK));
    }
    lstore(0, 0);
    __syncthreads();
    for (int ks = 0; ks < ksteps; ks += S) {
#pragma unroll
      for (int u = 0; u < S; ++u) {
        const int k = ks + u;
        if (k < ksteps) {
          // stage u held step k and was written to LDS at the end of step
          // k - 1: it now takes step k + S
          if (k + S < ksteps) {
            gload(u, kna, knb);
            if (k + S + 1 < ksteps) {
              kna = tlook(ctab + TAB_AK * kTabSize, (uint32_t)(k + S + 1) * TK);
              knb = tlook(ctab + TAB_BK * kTabSize, (uint32_t)(k + S + 1) * TK);
            }
          }
          kstep(k & 1);
          if (k + 1 < ksteps) lstore((k + 1) & 1, (u + 1) % S);
          __syncthreads();
        }
      }
    }

    // output scale of this instance
    const float bound = ldexpf(mxa * mxb, d.kbits + 1);
    int ex = 0;
    if (bound > 0.f) frexpf(bound, &ex);
    const float f = ldexpf(1.f, 15 - ex);
    const int e_out = ea + eb + ex - 15;
    float mx = 0.f;
    // Lane l of half-wave h holds the column pairs 4c + 2h, 4c + 2h + 1 of
    // its m.  Plain tiles pick their stores from the output's lowest storage
    // positions (a test uniform over the workgroup): where columns, or a
    // column and m bit 0, are adjacent in memory, lanes combine values into
    // 8- or 16-byte stores; otherwise (m bits lowest, so that neighbouring
    // lanes already write consecutive words) each value is one 4-byte store.
    // n bits 0 and 1 lowest: the half-waves swap pairs (v_permlane32_swap) so
    // that each lane holds four consecutive columns, one 16-byte store.
    if (!FAN && s_cn[1] - s_cn[0] == 1u && s_cn[2] - s_cn[0] == 2u) {
#pragma unroll
      for (int q = 0; q < RN; ++q) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          // hv: columns 8c + 2h + {0, 1, 4, 5} of this lane's m
          uint32_t hv[RM][4];
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) {
            const int r = 2 * (4 * c + r4);
#pragma unroll
            for (int i = 0; i < RM; ++i) {
              const __half2 h = __float22half2_rn(make_float2(acc[i][q][r] * f, acc[i][q][r + 1] * f));
              hv[i][r4] = h2bits(h);
              const float2 back = __half22float2(h);
              mx = fmaxf(mx, fmaxf(fabsf(back.x), fabsf(back.y)));
            }
          }
          // after the swaps half-wave h holds columns 8c + 4h + {0, 1, 2, 3}
          const uint32_t ocn = s_cn[(wn * RN + q) * 16 + 8 * c + 4 * half];
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            const auto x0 = __builtin_amdgcn_permlane32_swap(hv[i][0], hv[i][2], false, false);
            const auto x1 = __builtin_amdgcn_permlane32_swap(hv[i][1], hv[i][3], false, false);
            stg_u32x4(pc, om[i] + ocn, u32x4{x0[0], x1[0], x0[1], x1[1]});
          }
        }
      }
    } else if (!FAN && s_cn[1] - s_cn[0] == 1u) {
      // n bit 0 alone lowest: each lane's column pair is one 8-byte store
#pragma unroll
      for (int q = 0; q < RN; ++q) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t ocn = s_cn[(wn * RN + q) * 16 + 4 * c + 2 * half];
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            const __half2 h0 = __float22half2_rn(make_float2(acc[i][q][4 * c] * f, acc[i][q][4 * c + 1] * f));
            const __half2 h1 = __float22half2_rn(make_float2(acc[i][q][4 * c + 2] * f, acc[i][q][4 * c + 3] * f));
            stg_u32x2(pc, om[i] + ocn, u32x2{h2bits(h0), h2bits(h1)});
            const float2 b0 = __half22float2(h0), b1 = __half22float2(h1);
            mx = fmaxf(mx, fmaxf(fmaxf(fabsf(b0.x), fabsf(b0.y)), fmaxf(fabsf(b1.x), fabsf(b1.y))));
          }
        }
      }
    } else if (!FAN && s_cn[1] - s_cn[0] == 2u && tlook(tab + TAB_CM * kTabSize, 1u) == 1u) {
      // m bit 0 lowest, n bit 0 next: lanes 2j and 2j + 1 (m bit 0 = 0, 1)
      // exchange column pairs (DPP) so that each holds the 2 x 2 block of one
      // pair -- four consecutive words, one 16-byte store -- the even lane
      // for column pair 4c + 2h (c even), the odd lane for 4(c + 1) + 2h
      const bool odd = (l32 & 1) != 0;
#pragma unroll
      for (int q = 0; q < RN; ++q) {
#pragma unroll
        for (int p2 = 0; p2 < 2; ++p2) {
          const int cs = 2 * p2 + (odd ? 1 : 0);  // the column group this lane stores
          const uint32_t ocn = s_cn[(wn * RN + q) * 16 + 4 * cs + 2 * half];
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            uint32_t w[2][2];  // [group 2 p2 + e][n bit 0]
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const int r = 4 * (2 * p2 + e);
              const __half2 h0 = __float22half2_rn(make_float2(acc[i][q][r] * f, acc[i][q][r + 1] * f));
              const __half2 h1 = __float22half2_rn(make_float2(acc[i][q][r + 2] * f, acc[i][q][r + 3] * f));
              w[e][0] = h2bits(h0);
              w[e][1] = h2bits(h1);
              const float2 b0 = __half22float2(h0), b1 = __half22float2(h1);
              mx = fmaxf(mx, fmaxf(fmaxf(fabsf(b0.x), fabsf(b0.y)), fmaxf(fabsf(b1.x), fabsf(b1.y))));
            }
            // send the group the partner stores, keep the own one
            const uint32_t s0 = odd ? w[0][0] : w[1][0];
            const uint32_t s1 = odd ? w[0][1] : w[1][1];
            const uint32_t r0 = (uint32_t)__builtin_amdgcn_mov_dpp((int)s0, 0xB1, 0xF, 0xF, false);  // lane ^ 1
            const uint32_t r1 = (uint32_t)__builtin_amdgcn_mov_dpp((int)s1, 0xB1, 0xF, 0xF, false);
            const u32x4 v = odd ? u32x4{r0, w[1][0], r1, w[1][1]} : u32x4{w[0][0], r0, w[0][1], r1};
            stg_u32x4(pc, om[i] - (odd ? 1u : 0u) + ocn, v);
          }
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < RN; ++q) {
#pragma unroll
        for (int rr = 0; rr < 8; ++rr) {
          const int r = 2 * rr;
          const int row = 8 * (rr >> 1) + 4 * half + 2 * (rr & 1);
          const int nl = (wn * RN + q) * 16 + (row >> 1);  // column within the tile
          const uint32_t ocn = s_cn[nl];
          uint64_t dst = pc;
          bool live = true;
          float fo = f;
          int g = 0;
          if (FAN) {
            g = nl >> d.nbits;
            const uint64_t cbs = s_cbase[g];  // uniform over the 32 lanes of a half-wave (one n)
            live = cbs != 0;
            dst = ws + cbs;
            fo = s_f[g];
          }
          float v = 0.f;
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            const __half2 h = __float22half2_rn(make_float2(acc[i][q][r] * fo, acc[i][q][r + 1] * fo));
            if (live) stg_u32(dst, om[i] + ocn, h2bits(h));
            const float2 back = __half22float2(h);
            v = fmaxf(v, fmaxf(fabsf(back.x), fabsf(back.y)));
          }
          if (FAN) {
#pragma unroll
            for (int o2 = 16; o2 > 0; o2 >>= 1) v = fmaxf(v, __shfl_xor(v, o2));
            if (l32 == 0 && live) atomicMax(&s_mx[g], __float_as_uint(v));
          } else {
            mx = fmaxf(mx, v);
          }
        }
      }
    }
    if (FAN) {
      __syncthreads();
      if (tid < slots) {
        const int jg = fj[tid];
        if (jg >= 0) {
          // the exponent is the same for every m tile of the slot: the first writes it
          if (t == 0) stg_scale_e(ws + d.c_scale_off, s * d.w + jg, s_e[tid]);
          if (s_mx[tid] > 0u) max_scale_mx(ws + d.c_scale_off, s * d.w + jg, s_mx[tid]);
        }
      }
    } else {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
      if (lane == 0) {
        // the exponent is the same for every tile of the instance: its first tile writes it
        if (t == 0 && wave == 0) stg_scale_e(ws + d.c_scale_off, inst, e_out);
        if (mx > 0.f) max_scale_mx(ws + d.c_scale_off, inst, __float_as_uint(mx));
      }
    }
    __syncthreads();  // the column and slot arrays are rewritten by the next tile
  }
}

__global__ __launch_bounds__(256) void k_slice_sum_h(OpDesc root, uint64_t ws, const int64_t* __restrict__ sig,
                                                     int nb, int64_t nrows, const int32_t* __restrict__ rows,
                                                     int open_bits, double2* __restrict__ amps) {
  const gptr<const int32_t> gmap = gmem<const int32_t>(ws + root.gmap_off);
  const uint64_t sc = ws + root.scale_off;
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
      const uint64_t base = ws + root.off + inst * root.inst_bytes;
      float2 v;
      if (root.half) {
        const uint32_t u = ldg_u32(base, o);
        __half2 h;
        __builtin_memcpy(&h, &u, 4);
        v = __half22float2(h);
      } else {
        v = ldg_f2(base, o);
      }
      const int e = ldg_scale(sc, inst).e;
      acc.x += ldexp((double)v.x, e);
      acc.y += ldexp((double)v.y, e);
    }
    amps[dst] = acc;
  }
}

// one block per (instance, segment of up to 8192 elements): max over the
// segment, one atomic per block
__global__ __launch_bounds__(256) void k_absmax(uint64_t base, int ebits, int64_t n_inst, uint64_t scales) {
  __shared__ float red[4];
  const int sbits = ebits < 13 ? ebits : 13;
  const int64_t seg_per_inst = (int64_t)1 << (ebits - sbits);
  const int64_t n_blk = n_inst * seg_per_inst;
  for (int64_t blk = blockIdx.x; blk < n_blk; blk += gridDim.x) {
    const int64_t inst = blk / seg_per_inst;
    const uint64_t e0 = ((uint64_t)inst << ebits) + ((uint64_t)(blk - inst * seg_per_inst) << sbits);
    float mx = 0.f;
    for (uint32_t e = threadIdx.x; e < (1u << sbits); e += 256) {
      const float2 v = ldg_f2(base, e0 + e);
      mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
      if (m > 0.f) max_scale_mx(scales, inst, __float_as_uint(m));
    }
    __syncthreads();  // red[] is rewritten by the next block
  }
}

__global__ __launch_bounds__(256) void k_zero(uint4* __restrict__ p, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------

constexpr int64_t kPersistentGridH = 2048;

struct MfmaCfgH {
  int tm_bits, tn_bits, tk_bits;
};

static const MfmaCfgH kMfmaCfgsH[] = {
    {7, 6, 4},  // 0: RM=2 RN=2 WM=2 WN=2, TK=16 -> TM=128, TN=64
    {7, 5, 4},  // 1: RM=2 RN=1 WM=2 WN=2, TK=16 -> TM=128, TN=32
    {6, 5, 4},  // 2: RM=1 RN=1 WM=2 WN=2, TK=16 -> TM=64,  TN=32
    {8, 5, 4},  // 3: RM=4 RN=1 WM=2 WN=2, TK=16 -> TM=256, TN=32
    {7, 5, 3},  // 4: RM=2 RN=1 WM=2 WN=2, TK=8  -> TM=128, TN=32
    {8, 6, 4},  // 5: RM=4 RN=2 WM=2 WN=2, TK=16 -> TM=256, TN=64
    {7, 6, 3},  // 6: RM=2 RN=2 WM=2 WN=2, TK=8  -> TM=128, TN=64
    // eight waves per workgroup: twice the flops per staged byte of the
    // four-wave tiles, for the MFMA-bound stem steps (large m, n and k)
    {8, 7, 4},  // 7: RM=2 RN=4 WM=4 WN=2, TK=16 -> TM=256, TN=128
    {8, 6, 4},  // 8: RM=2 RN=2 WM=4 WN=2, TK=16 -> TM=256, TN=64
};

int mfma_h_config_count() { return (int)(sizeof(kMfmaCfgsH) / sizeof(kMfmaCfgsH[0])); }

bool mfma_h_config_fits(int cfg, int mbits, int nbits, int kbits) {
  if (cfg < 0 || cfg >= mfma_h_config_count()) return false;
  const MfmaCfgH& c = kMfmaCfgsH[cfg];
  return mbits >= c.tm_bits && nbits >= c.tn_bits && kbits >= c.tk_bits;
}

int mfma_h_config_tn(int cfg) { return cfg < 0 || cfg >= mfma_h_config_count() ? 0 : 1 << kMfmaCfgsH[cfg].tn_bits; }

bool mfma_h_fan_config_fits(int cfg, int mbits, int nbits, int kbits, int fan_tn) {
  if (cfg < 0 || cfg >= mfma_h_config_count()) return false;
  const MfmaCfgH& c = kMfmaCfgsH[cfg];
  return (1 << c.tn_bits) == fan_tn && nbits < c.tn_bits && mbits >= c.tm_bits && kbits >= c.tk_bits;
}

template <bool FAN, bool HA, bool HB>
static hipError_t launch_mfma_h_cfg(const NodeDesc& d, int cfg, unsigned grid, uint64_t ws, const int64_t* sig,
                                    hipStream_t st) {
  switch (cfg) {
    case 0: hipLaunchKernelGGL((k_mfma_h<2, 2, 2, 2, 16, FAN, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 1: hipLaunchKernelGGL((k_mfma_h<2, 1, 2, 2, 16, FAN, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 2: hipLaunchKernelGGL((k_mfma_h<1, 1, 2, 2, 16, FAN, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 3: hipLaunchKernelGGL((k_mfma_h<4, 1, 2, 2, 16, FAN, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 4: hipLaunchKernelGGL((k_mfma_h<2, 1, 2, 2, 8, FAN, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 5: hipLaunchKernelGGL((k_mfma_h<4, 2, 2, 2, 16, FAN, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 6: hipLaunchKernelGGL((k_mfma_h<2, 2, 2, 2, 8, FAN, HA, HB>), dim3(grid), dim3(256), 0, st, d, ws, sig); break;
    case 7:
      if (FAN) return hipErrorInvalidValue;  // fan tables hold 32 or 64 columns
      hipLaunchKernelGGL((k_mfma_h<2, 4, 4, 2, 16, false, HA, HB>), dim3(grid), dim3(512), 0, st, d, ws, sig);
      break;
    case 8: hipLaunchKernelGGL((k_mfma_h<2, 2, 4, 2, 16, FAN, HA, HB>), dim3(grid), dim3(512), 0, st, d, ws, sig); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool FAN>
static hipError_t launch_mfma_h_t(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st) {
  if (d.n_inst == 0) return hipSuccess;
  const bool fits = FAN ? mfma_h_fan_config_fits(cfg, d.mbits, d.nbits, d.kbits, d.fan_tn)
                        : mfma_h_config_fits(cfg, d.mbits, d.nbits, d.kbits);
  if (!fits || (FAN && (d.w <= 0 || d.n_fan <= 0))) return hipErrorInvalidValue;
  const MfmaCfgH& c = kMfmaCfgsH[cfg];
  const int64_t units = FAN ? (d.n_inst / d.w) * d.n_fan : d.n_inst;
  const int64_t tiles = ((int64_t)1 << (d.mbits - c.tm_bits)) * (FAN ? 1 : ((int64_t)1 << (d.nbits - c.tn_bits)));
  // a persistent grid: 2048 workgroups (8 per CU) stride over the tiles, so
  // that each one's setup (tables, column data in LDS) is paid once per
  // several tiles; 3% faster than one workgroup per tile on the 6x6 stem
  // steps, with no dependence on the count between 1024 and 16384
  const unsigned grid = (unsigned)std::min<int64_t>(grid_for(units * tiles), kPersistentGridH);
  if (d.A.half) {
    if (d.B.half) return launch_mfma_h_cfg<FAN, true, true>(d, cfg, grid, ws, sig, st);
    return launch_mfma_h_cfg<FAN, true, false>(d, cfg, grid, ws, sig, st);
  }
  if (d.B.half) return launch_mfma_h_cfg<FAN, false, true>(d, cfg, grid, ws, sig, st);
  return launch_mfma_h_cfg<FAN, false, false>(d, cfg, grid, ws, sig, st);
}

hipError_t launch_mfma_h(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st) {
  if (!d.c_half) return hipErrorInvalidValue;  // FP16 outputs only
  return launch_mfma_h_t<false>(d, cfg, ws, sig, st);
}

hipError_t launch_mfma_h_fan(const NodeDesc& d, int cfg, uint64_t ws, const int64_t* sig, hipStream_t st) {
  if (!d.c_half) return hipErrorInvalidValue;
  return launch_mfma_h_t<true>(d, cfg, ws, sig, st);
}

hipError_t launch_slice_sum_h(const OpDesc& root, uint64_t ws, const int64_t* sig, int nb, int64_t nrows,
                              const int32_t* rows, int open_bits, double* amps, hipStream_t st) {
  const int64_t total = nrows << open_bits;
  if (total == 0 || nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_slice_sum_h, dim3(grid_for((total + 255) / 256)), dim3(256), 0, st, root, ws, sig, nb, nrows,
                     rows, open_bits, reinterpret_cast<double2*>(amps));
  return hipGetLastError();
}

hipError_t launch_absmax(const NodeDesc& d, uint64_t ws, hipStream_t st) {
  if (d.n_inst == 0) return hipSuccess;
  const int ebits = d.mbits + d.nbits;  // elements per output instance = 2^ebits (FP32 storage)
  const int sbits = ebits < 13 ? ebits : 13;
  const int64_t blocks = d.n_inst << (ebits - sbits);
  hipLaunchKernelGGL(k_absmax, dim3(grid_for(blocks)), dim3(256), 0, st, ws + d.c_off, ebits, d.n_inst,
                     ws + d.c_scale_off);
  return hipGetLastError();
}

hipError_t launch_zero(uint64_t ptr, uint64_t bytes, hipStream_t st) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(grid_for((n16 + 255) / 256)), dim3(256), 0, st, reinterpret_cast<uint4*>(ptr), n16);
  return hipGetLastError();
}

}  // namespace matnc
