// Device-visible descriptors of one contraction-tree node.
//
// Every index has dimension 2, so a tensor of rank r is 2^r elements and an
// element offset is a sum of independent bit contributions: the element at
// coordinates (m, n, k) of the pairwise step C[m, n] = sum_k A[m, k] B[k, n]
// sits at offset T_Am(m) + T_Ak(k) in A, T_Bk(k) + T_Bn(n) in B and
// T_Cm(m) + T_Cn(n) in C.  Each T_* is stored as four 256-entry tables of
// 8 coordinate bits each (uint32 element offsets; ranks <= 32), which is
// how the index permutation of every operand is fused into its loads and
// stores.
#pragma once
#include <stdint.h>

namespace matnc {

constexpr int kMaxLeafSliced = 16;
constexpr int kTabLevels = 4;
constexpr int kTabEntries = 256;
constexpr int kTabSize = kTabLevels * kTabEntries;  // uint32 per class table

// table classes inside a node's table block
enum TabClass { TAB_AM = 0, TAB_CM = 1, TAB_BN = 2, TAB_CN = 3, TAB_AK = 4, TAB_BK = 5, TAB_COUNT = 6 };

// How one node reads one operand instance.  For output instance (s, j)
// (slice s of the batch, reuse-tree key j of the node):
//   inst = gmap[j] * nsv + sub(sigma) + (dep ? s * w_child : 0)
// where sub(sigma) gathers the sigma bits sbit[0..nsb) into an nsv-index
// (leaves holding sliced indices), and dep marks an intermediate operand
// whose instances are stored per slice.
struct OpDesc {
  uint64_t off;         // byte offset of instance 0 in the workspace
  uint64_t inst_bytes;  // bytes per instance
  uint64_t gmap_off;    // byte offset of the int32 gather map (one entry per j)
  uint64_t scale_off;   // complex-half: byte offset of the {int32 e, uint32 max} pair of instance 0
  int32_t w_child;      // instances per slice of the operand
  int32_t dep;          // 1: operand instances repeat per slice
  int32_t nsv;          // leaf: 2^nsb slice variants per key; else 1
  int32_t nsb;          // number of sliced indices on the leaf
  int32_t half;         // complex-half plans: 1 = stored as FP16 with scales, 0 = FP32
  int32_t pad0;
  int8_t sbit[kMaxLeafSliced];  // sigma bit of each sliced index
};

struct NodeDesc {
  OpDesc A, B;
  uint64_t c_off;        // byte offset of output instance 0
  uint64_t c_inst_bytes; // bytes per output instance
  uint64_t tab_off;      // byte offset of the TAB_COUNT x kTabSize uint32 tables
  uint64_t c_scale_off;  // complex-half: byte offset of the output's {e, max} pairs
  int64_t n_inst;        // instances in this launch = w * (dep ? batch : 1)
  int32_t w;             // reuse-tree width w(v)
  int32_t dep;           // output instances repeat per slice
  int32_t mbits, nbits, kbits;
  int32_t c_half;        // complex-half plans: output stored as FP16 (1) or FP32 (0)
  // fan-out grouping (MFMA steps with few output columns whose A instance
  // is shared by several output instances): row g of the int32 table at
  // fan_off lists up to fan_tn >> nbits output instances j (-1 = empty
  // slot) that all read the same A instance; they are computed together as
  // one GEMM whose fan_tn columns are the slots' own B columns side by side
  // (fan_tn = the N width of the tile configuration)
  uint64_t fan_off;
  int64_t n_fan;         // rows of the fan table (per slice)
  int32_t fan_tn;
  // tile order: units (output instances, or fan-table rows) in blocks of
  // fan_rows with the units innermost (see unit_tile); 1 (plain) or 2 (fan
  // tables), or about the number of units that share one A instance when
  // that instance is too large for the caches
  int32_t fan_rows;
};

// Scaling of one stored instance in complex-half plans: true value = stored
// value * 2^e (e = 0 for FP32 storage); mx = largest |re| or |im| of the
// stored values (float bits, so that unsigned atomicMax orders it).
struct HalfScale {
  int32_t e;
  uint32_t mx;
};

__host__ __device__ inline int64_t sub_index(const OpDesc& o, int64_t sigma) {
  int64_t v = 0;
  for (int t = 0; t < o.nsb; ++t) v |= ((sigma >> o.sbit[t]) & 1) << t;
  return v;
}

}  // namespace matnc
