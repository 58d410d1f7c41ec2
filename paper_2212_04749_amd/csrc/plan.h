// Host-side plan of a sliced multi-amplitude contraction.
//
// A plan is static (main text: the reuse tree fixes contraction pattern,
// cost and memory before running; Supplementary Sec. III.C): for every node
// v of the given contraction tree it holds
//   idx(v)   free indices in storage order (bit 0 = lowest),
//   O(v)     closed output qubits below v,
//   keys(v)  the distinct projections of the batch onto O(v), sorted;
//            w(v) = |keys(v)| is the reuse-tree width at v (Eq. (1)),
//   ga, gb   gather maps from keys(v) into the children's keys,
//   dep(v)   whether a sliced index lies below v (slice-dependent),
// and the memory plan: every intermediate gets a fixed byte range of the
// caller's workspace for its lifetime in the schedule (invariant nodes once,
// dependent nodes once per slice batch), found by first-fit over lifetime
// overlaps.  Slice-invariant tensors consumed by dependent nodes stay for
// the whole run (the stem cache).
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <memory>
#include <cstdint>
#include <string>
#include <vector>

#include "desc.h"

namespace matnc {

struct Network {
  int n_tensors = 0;
  int n_qubits = 0;
  std::vector<std::vector<int>> idx;      // index ids per tensor (first = most significant)
  std::vector<std::vector<double>> data;  // interleaved complex128
  std::vector<int> out_index;             // output index id per qubit
};

struct PNode {
  int a = -1, b = -1;        // children (leaf: -1)
  int parent = -1;
  std::vector<int> idx;      // free indices, storage order
  uint64_t omask = 0;
  bool dep = false;
  std::vector<uint64_t> keys;
  std::vector<int32_t> ga, gb;  // per key: index into keys of child A / child B (roles below)
  // leaf data mapping
  std::vector<int> sl_bits;      // sigma bits of the sliced indices on this leaf (ascending)
  std::vector<int> sl_index;     // the sliced index ids, same order
  // step description (internal nodes)
  bool swap = false;             // true: operand A is child b
  bool half_store = false;       // complex-half plans: stored as FP16 (the costliest steps)
  bool rec_max = false;          // complex-half plans: FP32 tensor whose maximum an FP16 consumer needs
  int kernel = 0;                // 0 streaming, 1 MFMA
  int cfg = -1;
  bool fan = false;              // MFMA step run as fan-out tiles (rows of fanv)
  int fan_tn = 0;                // complex columns of its tiles (slots x 2^|N|): 32 or 64
  std::vector<int32_t> fanv[2];  // fan tables for 32- and 64-column tiles (unchunked plans)
  int64_t n_fan[2] = {0, 0};
  uint64_t fan_off[2] = {0, 0};
  int32_t fan_rows[2] = {2, 2};  // tile-order blocks of the two tables (NodeDesc::fan_rows)
  int32_t unit_rows = 1;         // ... of the output instances of a plain MFMA step
  std::vector<int> M, N, K;      // virtual orders of the three index classes
  // memory
  uint64_t inst_elems = 0;
  uint64_t buf_bytes = 0;        // whole buffer (all instances of a launch)
  uint64_t off = 0;              // byte offset in workspace
  uint64_t tab_off = 0, ga_off = 0, gb_off = 0;
  int time = 0;                  // schedule position
  uint64_t scale_off = 0;        // complex-half: byte offset of the HalfScale array
};

// One chunk of the reuse keys: the distinct root keys are split, in trie
// order, into chunks that run one after another.  A chunk first computes its
// own instances of the slice-invariant nodes wider than one key (its part of
// the cache), then runs every slice batch through the slice-dependent nodes,
// so that buffers only ever hold one chunk's instances.
struct ChunkNode {
  int32_t w = 0;                      // this chunk's instances of the node
  std::vector<int32_t> ga, gb;        // gather maps (local or full child indices)
  uint64_t ga_off = 0, gb_off = 0;
  std::vector<int32_t> fanv[2];       // fan tables over this chunk's instances (32, 64 columns)
  int64_t n_fan[2] = {0, 0};
  uint64_t fan_off[2] = {0, 0};
  int32_t fan_rows[2] = {2, 2};
  int32_t unit_rows = 1;
};

struct Chunk {
  std::vector<ChunkNode> nodes;       // indexed by position in Plan::chunked
  std::vector<int32_t> rows;          // input rows whose root key is in the chunk
  std::vector<int32_t> rootloc;       // local root instance of each of those rows
  uint64_t rows_off = 0, rootloc_off = 0;
};

// The plans of a queue bound to one workspace share one arena for their
// intermediates (they run one after another); `owner` names the plan whose
// tensors the arena holds now, so that the others know their stem cache is
// gone.
struct ArenaShare {
  uint64_t owner = 0;
};

struct Plan {
  Network net;
  int n_nodes = 0;               // n_tensors + steps
  std::vector<std::pair<int, int>> pairs;
  std::vector<int> sliced;
  std::vector<int> open_qubits;
  std::vector<uint64_t> words;   // closed bits only
  int precision = 0;
  int max_rank_cap = 0;
  int batch = 1;
  int elem_bytes = 8;
  uint64_t memory_budget = 0;    // 0 = no limit
  int half_nodes = 0;            // complex-half: budget of FP16-stored intermediates
  int n_half = 0;                // complex-half: FP16-stored intermediates
  int n_chunks = 1;
  std::vector<Chunk> chunks;
  std::vector<int> chunk_pos;    // node id -> position in chunked (-1 if not there)
  std::vector<PNode> nodes;
  uint64_t inv_scale_lo = 0, inv_scale_hi = 0;    // complex-half scale slots of prologue nodes
  uint64_t cpro_scale_lo = 0, cpro_scale_hi = 0;  // ... of per-chunk invariant nodes
  uint64_t dep_scale_lo = 0, dep_scale_hi = 0;    // ... and of per-batch nodes
  uint64_t sigma_off = 0;
  uint64_t static_bytes = 0;
  uint64_t workspace_bytes = 0;
  uint64_t cache_bytes = 0;
  // node ids in schedule order: computed once per cache fill (prologue),
  // once per chunk (cpro), per slice batch and chunk (loop); chunked =
  // cpro followed by loop
  std::vector<int> prologue, cpro, loop, chunked;
  // costs
  double cmac_single = 0, cmac_multi = 0, cmac_inv = 0, cmac_total = 0;
  double bytes_slice = 0, bytes_inv = 0;
  int max_rank = 0;
  int n_mfma = 0;
  int64_t n_unique = 0;
  // binding
  uint64_t arena_delta = 0;              // intermediates live at ws + off + arena_delta
  std::shared_ptr<ArenaShare> share;     // set when the arena is shared with other plans
  uint64_t share_id = 0;                 // this plan's name in share->owner
  bool bound = false;
  bool inv_valid = false;
  uint64_t ws = 0;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  std::vector<hipGraph_t> graphs;          // one full slice batch per chunk
  std::vector<hipGraphExec_t> graph_execs;
  double* graph_amps = nullptr;        // amplitude buffer the batch graphs add into
  uint64_t generation = 0;             // bumped whenever launch parameters change
  std::vector<unsigned char> staging;  // host image of the static region
  std::vector<NodeDesc> descs;         // per node (full-batch instance counts)
};

}  // namespace matnc
