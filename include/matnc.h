/*
 * matnc.h -- C ABI of libmatnc: sliced multi-amplitude tensor-network
 * contraction on one MI355X (gfx950).
 *
 * The problem (Supplementary Information Sec. II, main text "Multiple-
 * amplitude simulation"): a circuit becomes a tensor network whose n output
 * indices (one per qubit) are uncontracted.  Fixing every output index to a
 * bit of b gives a closed network whose value is the amplitude <b|psi>;
 * leaving some output indices open gives a block of correlated amplitudes.
 * k bitstrings give k networks that differ only in their bright tensors
 * (tensors holding an output index).  A contraction order (TNCO, a binary
 * tree) is given; every intermediate tensor computed before the subtree
 * meets an output index is shared by all bitstrings that agree on the
 * outputs below it (the reuse tree, Eq. (1)).  A sliced index set turns the
 * network into the sum of 2^|S| smaller networks (Supplementary Sec. IV.B).
 * Linear XEB is F = (2^n / K) sum |a|^2 - 1 over the K amplitudes (the mean
 * of x = 2^n p under Eq. (2) is 1 + F).
 *
 * Conventions shared by all calls:
 *  - every index has dimension 2; index ids are non-negative ints;
 *  - a tensor's data is complex128, interleaved (re, im), row-major over the
 *    tensor's index list with the FIRST index most significant;
 *  - bitstring words are uint64 with bit q = value of qubit q;
 *  - open-leg results: the amplitude block of group i has 2^n_open entries,
 *    entry j has the t-th open qubit (ascending qubit id) equal to bit t of j;
 *  - device amplitude buffers are complex128 interleaved, [k][2^n_open][2].
 *
 * Ownership: every host array passed in is copied before the call returns.
 * The library never allocates device memory: all device storage is the
 * caller's workspace (matnc_plan_bind) or the caller's output buffers, apart
 * from one 32 KiB device array per GPU owned by the library for
 * matnc_contract_noalloc.  The plan owns host metadata and, while bound, the
 * captured HIP graph.
 *
 * Errors: every call returns MATNC_OK (0) or one of the MATNC_E_* codes and
 * never throws or aborts across the ABI.  matnc_last_error() returns a
 * thread-local message for the last failing call of the calling thread.  On
 * error, output arguments are left unchanged.
 *
 * Threading: one plan per stream; a plan must not be used from two threads
 * at once.  Different plans are independent.
 */
#ifndef MATNC_H
#define MATNC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MATNC_OK = 0,
  MATNC_E_INVALID = 1, /* malformed input (ids, tree, bitstrings, sizes)       */
  MATNC_E_RANK = 2,    /* an intermediate exceeds max_rank after slicing      */
  MATNC_E_NOMEM = 3,   /* workspace smaller than matnc_plan_info's figure     */
  MATNC_E_HIP = 4,     /* a HIP runtime call failed; its text is in the message */
  MATNC_E_STATE = 5    /* call out of order (e.g. execute before bind)        */
};

enum {
  MATNC_C64 = 0,  /* complex64: FP32 storage, FP32 MFMA / FMA               */
  MATNC_CHALF = 1 /* complex-half: FP16 storage with a power-of-two exponent
                     per tensor instance, FP16 MFMA with FP32 accumulation   */
};

typedef struct matnc_network_s *matnc_network;
typedef struct matnc_plan_s *matnc_plan;
typedef struct matnc_queue_s *matnc_queue;

/* Version string of the library ("matnc <semver> gfx950"). */
const char *matnc_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char *matnc_last_error(void);

/*
 * matnc_network_create -- the tensor network of a circuit (Supplementary
 * Sec. II: |0>, one- and two-qubit gates as rank-1/2/4 tensors, possibly
 * fused).
 *   n_tensors              number of tensors, >= 1
 *   ranks[n_tensors]       rank of each tensor, 0..20
 *   index_ids[sum ranks]   index ids of tensor 0, then tensor 1, ...
 *   data_c128              2 * sum(2^rank) doubles, tensors concatenated
 *   n_qubits               1..64
 *   output_index_of_qubit[n_qubits]  the output index id of each qubit
 * Every output index must occur on exactly one tensor, every other index on
 * exactly two (no hyper-indices).  Errors: MATNC_E_INVALID.
 */
int matnc_network_create(int n_tensors, const int *ranks, const int *index_ids,
                         const double *data_c128, int n_qubits,
                         const int *output_index_of_qubit, matnc_network *out);
int matnc_network_destroy(matnc_network net);

/*
 * matnc_plan_create -- static multi-amplitude plan (main text: the reuse
 * tree makes contraction pattern, cost and memory known before running).
 *   pairs[2*(n_tensors-1)]  contraction tree in SSA form: step j contracts
 *                           ids pairs[2j], pairs[2j+1] into id n_tensors+j;
 *                           every id is consumed exactly once, the last
 *                           step is the root
 *   sliced_ids[n_sliced]    bond indices to slice (Supplementary Sec. IV.B);
 *                           slice id sigma assigns bit j of sigma to
 *                           sliced_ids[j]; 2^n_sliced slices (n_sliced <= 40)
 *   open_qubits[n_open]     qubits whose output index stays open (distinct)
 *   k, bitstrings[k]        batch; bits of open qubits are ignored, bits at
 *                           positions >= n_qubits must be zero; duplicates
 *                           are allowed (each gets its own result row)
 *   precision               MATNC_C64 or MATNC_CHALF
 *   max_rank                cap on every tensor's rank after slicing, <= 32
 *   slice_batch             slices contracted per launch sequence (>= 1);
 *                           the workspace grows with it
 *   memory_budget           largest workspace (bytes) the plan may need, 0 =
 *                           no limit.  If the breadth-first plan exceeds it,
 *                           the distinct bitstrings are split, in reuse-tree
 *                           (trie) order, into 2, 4, ... chunks that run one
 *                           after another through the per-batch steps, so
 *                           that only one chunk's instances are live
 *                           (MATNC_E_NOMEM if even single keys do not fit)
 * The library derives the reuse structure (distinct projections of the
 * batch onto the outputs below each tree node, gather maps between a node
 * and its children), the storage order of every intermediate, the kernel
 * choice per node and the static memory plan.
 * Errors: MATNC_E_INVALID, MATNC_E_RANK, MATNC_E_NOMEM.
 */
int matnc_plan_create(matnc_network net, const int *pairs, int n_sliced,
                      const int *sliced_ids, int n_open, const int *open_qubits,
                      int64_t k, const uint64_t *bitstrings, int precision,
                      int max_rank, int slice_batch, size_t memory_budget,
                      matnc_plan *out);

/*
 * matnc_plan_create_ex -- matnc_plan_create with its tuning choices in a
 * struct (zero-initialise it, then set the fields):
 *   slice_batch, memory_budget   as in matnc_plan_create
 *   half_nodes                   complex-half plans: how many intermediates
 *                                are stored in FP16 -- those whose steps
 *                                carry the most estimated FP32 time, which
 *                                then run on the FP16 MFMA kernels.  Each
 *                                adds one FP16 rounding (relative rms about
 *                                2^-11/sqrt(3)) to the amplitudes, so this is
 *                                the plan's precision budget; 0 keeps every
 *                                tensor in FP32; -1 = library default,
 *                                min(16, K / 282) for K = k * 2^n_open
 *                                amplitudes (the linear XEB of K amplitudes
 *                                moves by about 2 e / sqrt(K) for independent
 *                                relative errors of rms e; the cap of 16
 *                                keeps a margin for correlated ones).
 *                                Ignored for MATNC_C64.
 * Errors: as matnc_plan_create; MATNC_E_INVALID for a null opts or
 * half_nodes < -1.
 */
typedef struct {
  int slice_batch;
  size_t memory_budget;
  int half_nodes;
} matnc_plan_options_t;

int matnc_plan_create_ex(matnc_network net, const int *pairs, int n_sliced,
                         const int *sliced_ids, int n_open, const int *open_qubits,
                         int64_t k, const uint64_t *bitstrings, int precision,
                         int max_rank, const matnc_plan_options_t *opts,
                         matnc_plan *out);

typedef struct {
  double cmac_single;       /* S: complex MACs of one amplitude, one slice   */
  double cmac_multi;        /* S_k: complex MACs of the batch, one slice     */
  double cmac_invariant;    /* part of S_k in nodes that see no sliced index */
  double cmac_total;        /* all slices: invariant once + dependent x 2^|S| */
  double bytes_per_slice;   /* algorithmic HBM bytes of one slice (dependent) */
  double bytes_invariant;   /* algorithmic HBM bytes of the invariant nodes  */
  int64_t n_slices;         /* 2^n_sliced                                    */
  int64_t n_amplitudes;     /* k * 2^n_open                                  */
  int64_t n_unique;         /* distinct closed bitstrings                    */
  int max_rank;             /* largest tensor rank after slicing             */
  int n_nodes;              /* contraction steps                             */
  int n_mfma_nodes;         /* steps routed to the MFMA GEMM kernel          */
  int n_launches_per_batch; /* kernel launches per slice batch, all chunks   */
  size_t workspace_bytes;   /* device workspace needed by matnc_plan_bind    */
  size_t cache_bytes;       /* part of it holding slice-invariant tensors    */
  int n_chunks;             /* key chunks the bitstrings are processed in    */
  int n_fan_nodes;          /* MFMA steps run as fan-out tiles               */
  int n_half_nodes;         /* complex-half: intermediates stored in FP16    */
} matnc_plan_info_t;

int matnc_plan_info(matnc_plan plan, matnc_plan_info_t *info);

/*
 * matnc_plan_set_tensor -- replace the data of tensor t (same index list);
 * complex128 as in matnc_network_create, 2 * 2^rank(t) doubles.  The
 * network of a circuit (Supplementary Sec. II) depends on the gates only
 * through its numbers, so circuits with the same layout (another seed, the
 * permutation circuits used for exact checks) share one plan.  Bound plans
 * upload the new leaf variants at once (and wait for that copy); the
 * slice-invariant cache is invalidated and the change takes effect at the
 * next execute, through the same captured graphs.
 * Errors: MATNC_E_INVALID (null data, t out of range), MATNC_E_HIP.
 */
int matnc_plan_set_tensor(matnc_plan plan, int t, const double *data_c128);

/*
 * matnc_plan_bind -- attach the caller's device workspace (at least
 * workspace_bytes, 256-byte aligned) and HIP stream (hipStream_t, may be
 * NULL for the null stream), upload leaf variants, gather maps and offset
 * tables.  The workspace holds the static memory plan of the reuse tree
 * (Supplementary Sec. III.C: with the reuse tree fixed before running, the
 * place and lifetime of every intermediate is known in advance).  The per-batch launch sequence of each chunk is captured as a HIP
 * graph on the first execute over a full batch (non-null stream only) and
 * replayed for every later full batch into the same amplitude buffer.
 * The workspace must stay allocated until the plan is destroyed or re-bound.
 * Errors: MATNC_E_NOMEM, MATNC_E_HIP, MATNC_E_INVALID (misaligned).
 */
int matnc_plan_bind(matnc_plan plan, void *dev_workspace, size_t bytes, void *hip_stream);

/*
 * matnc_execute -- contract slices [slice_begin, slice_end) and ADD their
 * contributions into amps_dev (complex128, [k][2^n_open]) in FP64, one
 * slice after another in increasing slice id (so any split of a slice range
 * into calls gives bit-identical results).  Each slice is the multi-
 * amplitude contraction of the main text (every intermediate computed once
 * per distinct projection of the batch, Eq. (1)); the amplitude is the sum
 * over slices (Supplementary Sec. IV.B).  Slice-invariant intermediates
 * are computed on the first call after bind/set_tensor and kept (stem
 * cache).  With several key chunks, the chunks run one after another: each
 * first computes its own instances of the invariant nodes wider than one
 * key (on every call), then runs the slice range.  Asynchronous on the
 * bound stream.
 * Errors: MATNC_E_STATE (not bound), MATNC_E_INVALID (range), MATNC_E_HIP.
 */
int matnc_execute(matnc_plan plan, int64_t slice_begin, int64_t slice_end, double *amps_dev);

/* matnc_execute_timed: the same work as matnc_execute over the same range
 * (same launches, same results, bit for bit), launched one by one rather
 * than replayed from captured graphs, with a pair of HIP events on the
 * bound stream around every launch of contraction step `step` (0 ..
 * n_tensors - 2, the order of the plan's pairs).  It blocks until the
 * stream is idle, then stores in *ms_total the summed event time of those
 * launches (milliseconds) and in *launches their number (once per slice
 * batch and key chunk for a slice-dependent step, once for an invariant
 * one computed by this call, 0 for an invariant one already cached).  For
 * timing one kernel inside a throughput measurement; the events are the
 * library's own and freed before it returns.
 * Errors: as matnc_execute, MATNC_E_INVALID (step, null outputs).
 */
int matnc_execute_timed(matnc_plan plan, int64_t slice_begin, int64_t slice_end, double *amps_dev, int step,
                        double *ms_total, int64_t *launches);

/*
 * matnc_xeb -- linear XEB of the amplitudes in amps_dev over all
 * k * 2^n_open entries: F = (2^n_qubits / K) sum |a|^2 - 1, a deterministic
 * FP64 reduction written to xeb_dev[0].  Asynchronous on the bound stream.
 */
int matnc_xeb(matnc_plan plan, const double *amps_dev, double *xeb_dev);

int matnc_plan_destroy(matnc_plan plan);

/*
 * matnc_plan_autotune -- choose the tile configuration of every step that
 * runs on the MFMA kernel by timing each configuration that fits the step's
 * shape (the fastest of reps separately timed launches, HIP events on the
 * bound stream) and keeping the fastest configuration; for fan-out steps the configuration's N width (32 or 64 complex
 * columns) also picks the fan table.  The launch graphs are re-captured at
 * the next execute.  Choices are keyed by shape class (precision, storage,
 * fan-out, m/n/k bits, instance count rounded to a power of two) and, if
 * cache_path is not NULL, read from and written back to that JSON file
 * (classes already in the file are not re-timed).  Overwrites intermediate
 * tensors (the stem cache is recomputed at the next execute).  Waits for the
 * stream.  Errors: MATNC_E_STATE (not bound), MATNC_E_HIP, MATNC_E_INVALID.
 */
int matnc_plan_autotune(matnc_plan plan, int reps, const char *cache_path);

/*
 * matnc_plan_reset_cache -- drop the slice-invariant tensors (stem cache)
 * so that the next matnc_execute recomputes them; used to time a complete
 * pass.  No device work is queued.  Errors: MATNC_E_INVALID (null plan).
 */
int matnc_plan_reset_cache(matnc_plan plan);

/*
 * matnc_plan_profile -- diagnostic pass: recompute the slice-invariant
 * nodes, then contract one slice batch of nb slices (1 <= nb <= slice_batch)
 * starting at slice_begin, with a HIP event pair around every node's launch
 * on the bound stream; waits for the stream.  For step j (0 <= j <
 * n_tensors - 1) it writes
 *   time_ms[j]  elapsed time of that launch (-1 if the node has no work),
 *   kernel[j]   0 = streaming kernel, 100 + c = FP32 MFMA tile
 *               configuration c, 200 + c = FP32 MFMA configuration c as
 *               fan-out tiles (the output instances that share an A
 *               instance computed as one GEMM); 300 + c and 400 + c the
 *               same for the FP16 MFMA kernels of complex-half steps whose
 *               result is stored in FP16,
 *   cmac[j]     algorithmic complex MACs of the launch (w * instances * 2^(m+n+k)),
 *   bytes[j]    algorithmic HBM bytes of the launch (each output instance
 *               written once, each distinct operand instance read once).
 * Arrays are caller-owned host memory of n_tensors - 1 entries.  The
 * amplitude buffers are not touched.  Errors: MATNC_E_STATE, MATNC_E_INVALID,
 * MATNC_E_HIP.
 */
int matnc_plan_profile(matnc_plan plan, int64_t slice_begin, int nb, float *time_ms, int *kernel,
                       double *cmac, double *bytes);

/*
 * Uneven batches: several bound plans (each with its own workspace and
 * circuit, or all on one workspace through matnc_queue_bind) executed over
 * all of their slices as one queue, with one FP64 amplitude buffer and one
 * XEB slot per plan -- contractions of very different sizes batched into
 * one launch sequence, as the tensor-size-dependent parallelisation of
 * Supplementary Sec. V batches many small contractions.
 *   matnc_queue_execute(q, amps_dev[n], xeb_dev[n]) contracts every slice
 *   of every plan (adding into amps_dev[i]) and writes XEB of plan i to
 *   xeb_dev[i].  All plans must be bound to the same (non-null) stream.  The
 *   whole queue -- every plan's stem, slice batches, slice-sums and XEB --
 *   is captured once as a single HIP graph (re-captured when the buffers or
 *   a plan's binding change) and launched as one graph per call.
 */
int matnc_queue_create(int n_plans, const matnc_plan *plans, matnc_queue *out);
int matnc_queue_execute(matnc_queue q, double *const *amps_dev, double *xeb_dev);
int matnc_queue_destroy(matnc_queue q);

/*
 * matnc_queue_workspace_bytes -- device workspace matnc_queue_bind needs:
 * the static regions of all plans (leaf data, gather maps, offset tables,
 * scale slots) side by side, then ONE arena for the intermediates, as large
 * as the largest plan's -- the plans of a queue run one after another, so
 * their intermediates (stem caches included) never need to coexist.
 *
 * matnc_queue_bind -- bind every plan of the queue to one caller workspace
 * (256-byte aligned, at least matnc_queue_workspace_bytes) and one stream,
 * replacing each plan's own binding (so a queue of circuits of uneven size
 * fits wherever its largest member fits).  The next matnc_queue_execute
 * captures the whole queue as one graph.  A plan may still be executed on
 * its own afterwards: it recomputes its slice-invariant tensors whenever
 * another plan of the queue has used the arena since.  The workspace must
 * stay allocated while the plans are bound to it.
 * Errors: MATNC_E_NOMEM (workspace too small), MATNC_E_INVALID (misaligned,
 * a plan listed twice), MATNC_E_HIP.
 */
int matnc_queue_workspace_bytes(matnc_queue q, size_t *out);
int matnc_queue_bind(matnc_queue q, void *dev_workspace, size_t bytes, void *hip_stream);

/*
 * matnc_contract -- one pairwise contraction with bit-permuted layouts
 * (the kernel behind every tree node; exposed for testing and tuning).
 * All indices have dimension 2.  For tensor X in {A, B, C}, pos_X[i] is the
 * storage bit position of the i-th index of that class:
 *   C[m, n] = sum_k A[m, k] * B[k, n]
 *   m bits: posA_m[nm], posC_m[nm];  n bits: posB_n[nn], posC_n[nn];
 *   k bits: posA_k[nk], posB_k[nk].
 * rank(A) = nm + nk, rank(B) = nn + nk, rank(C) = nm + nn (each <= 32) and
 * each tensor's positions form a permutation of 0..rank-1.
 * A, B, C are device pointers to complex64 (float2) data; batch instances
 * are contiguous: C[i] = A[i] x B[i] for i < batch (stride 2^rank).
 * kernel: -1 = library choice, 0 = streaming (VALU), 1 = MFMA GEMM with
 * the first tile configuration that fits, 100 + c = MFMA tile configuration
 * c (0 <= c < matnc_mfma_config_count()).
 * dev_scratch: caller's device buffer of at least
 * matnc_contract_scratch_bytes() bytes, 256-byte aligned, holding the
 * offset tables of the call (the library allocates nothing).  The call
 * uploads them and waits for that copy; the contraction itself is
 * asynchronous on hip_stream.  Errors: MATNC_E_INVALID, MATNC_E_NOMEM
 * (scratch too small), MATNC_E_HIP.
 */
size_t matnc_contract_scratch_bytes(void);
int matnc_mfma_config_count(void);
int matnc_contract(const void *A, const void *B, void *C, int64_t batch,
                   int nm, int nn, int nk,
                   const int *posA_m, const int *posA_k,
                   const int *posB_k, const int *posB_n,
                   const int *posC_m, const int *posC_n,
                   int kernel, void *dev_scratch, size_t scratch_bytes,
                   void *hip_stream);

/*
 * matnc_contract_noalloc -- matnc_contract for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops): the same
 * arguments without dev_scratch, the same kernels and results (bit for bit).
 * The offset tables live in a library-owned device array of 32 KiB per GPU
 * (one call needs matnc_contract_scratch_bytes() = 24832 bytes of it), held
 * from the first call on a GPU until the process ends; they are written by a
 * kernel on hip_stream, so the call neither copies from the host nor waits.
 * The current device must be the device of hip_stream and of A, B, C.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different threads) race on it and must be
 * serialised by the caller.  Nothing is allocated by the call.
 * Errors: MATNC_E_INVALID (as matnc_contract), MATNC_E_HIP.
 */
int matnc_contract_noalloc(const void *A, const void *B, void *C, int64_t batch,
                           int nm, int nn, int nk,
                           const int *posA_m, const int *posA_k,
                           const int *posB_k, const int *posB_n,
                           const int *posC_m, const int *posC_n,
                           int kernel, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MATNC_H */
