/*
 * tn.h -- C ABI of the sliced tensor-network contraction library (gfx950).
 *
 * The library computes the contraction of a tensor network of complex
 * tensors along a given pairwise contraction path (Sec. 2.3, Eq. sequence),
 * with a given set of sliced indices (Sec. 2.4, Eq. sliced_sum): the result
 * is the sum over all slices of the sliced networks' contractions.  Work that
 * does not depend on a slice is done once and reused by every slice
 * (Sec. 3.2, Fig. 5, Eq. task_based_amplitude_flops).
 *
 * Conventions shared by every call
 *   - Tensors are complex64 (interleaved re, im float32), row-major over the
 *     tensor's index list: the last listed index varies fastest.
 *   - Every index dimension is a power of two, 2 .. 65536.  An index that is
 *     not open appears in exactly two tensors and is summed when they meet
 *     (or kept and summed at the very end if it is sliced).  An open index
 *     may appear in any number of tensors (e.g. a batch of outcome strings
 *     shared by all output tensors); it is never summed and indexes the
 *     output.
 *   - Slice ids are mixed radix over the sliced indices in the order given at
 *     plan creation, the first one most significant.
 *   - Output buffers are complex128 (interleaved re, im float64), row-major
 *     over the open indices in the order given at plan creation.
 *   - Device pointers are HIP device pointers on the current device; the
 *     stream argument is a hipStream_t (NULL = default stream).  All device
 *     work is asynchronous on that stream.
 *   - Ownership: the plan copies every host array it is given.  The caller
 *     owns every device buffer (leaves, outputs, gradients, workspace); the
 *     library never allocates or frees device memory on its own and never
 *     keeps a device pointer past the call that received it.
 *   - Errors: every call returns a tn_status; no call aborts and no C++
 *     exception crosses this boundary.  tn_last_error() returns a message for
 *     the last failing call on the calling thread.
 *   - Concurrency: a plan is immutable after creation; it may be used by
 *     concurrent calls on different streams with distinct workspaces.
 */
#ifndef TN_H_
#define TN_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_plan_s* tn_plan_t;

typedef enum {
  TN_OK = 0,
  TN_E_INVALID = 1,      /* malformed network, path, slice list or argument   */
  TN_E_UNSUPPORTED = 2,  /* valid input outside what the library supports    */
  TN_E_WORKSPACE = 3,    /* workspace smaller than tn_plan_info.workspace_bytes */
  TN_E_OOM = 4,          /* host allocation failed                            */
  TN_E_HIP = 5           /* a HIP runtime call or kernel launch failed        */
} tn_status;

typedef enum { TN_C64 = 0, TN_SPLIT_BF16 = 1 } tn_precision;

typedef enum { TN_OUT_SUM = 0, TN_OUT_PER_SLICE = 1 } tn_out_mode;

/* plan flags */
#define TN_FLAG_NO_REUSE 1u   /* every slice recomputes every step (Eq. sliced_flops) */
#define TN_FLAG_SIMPLE_KERNELS 2u /* force the plain per-element kernels (debug)     */
#define TN_FLAG_NO_PERSISTENT 4u  /* no persistent segments (the default; kept so
                                     existing callers stay valid)                    */
#define TN_FLAG_CHAIN_VALU 32u    /* chains compute every step on the vector units
                                     (bitwise equal to per-step launches) instead of
                                     the matrix cores for 2^nk >= 4, 2^nn >= 8       */
#define TN_FLAG_CHAIN_STEPWISE 64u /* plan chains (and their layouts) but launch each
                                     of their steps separately; with
                                     TN_FLAG_CHAIN_VALU results are bitwise equal to
                                     the fused launches                              */
#define TN_FLAG_PERSISTENT 16u    /* experimental: run runs of small steps as one
                                     persistent launch each (workgroups claim work
                                     items and wait on completion counters)          */
#define TN_FLAG_NO_CHAIN 8u       /* run every step of a chain (consecutive stream
                                     steps on one running tensor) as its own launch
                                     instead of one fused launch per chain           */
#define TN_FLAG_CHAIN_NO_SINGLE 128u /* a chainable step with no chainable
                                     neighbour runs on its own kernel instead of as
                                     a one-step chain                                */
#define TN_FLAG_FIT_BACKWARD 256u  /* the resident / outer split also keeps
                                     info.workspace_backward_bytes within
                                     workspace_limit (plans used for gradients)      */
#define TN_FLAG_NO_TINY 512u      /* run tiny steps (at most 2^13 multiply-adds and
                                     2^11 outputs) one launch each instead of in
                                     batches of up to 20 consecutive ones per launch
                                     of one workgroup (forward batches are formed
                                     only without TN_FLAG_PERSISTENT); the same for
                                     the tiny products of tn_contract_backward      */
#define TN_FLAG_GEMM_EMBED 1024u  /* complex64 tiled GEMM steps (configurations 0, 1,
                                     3-6) use the real embedding of the complex
                                     product (8 real flops per complex multiply-add)
                                     instead of three real products (6 flops:
                                     Re A Re B, Im A Im B, (Re A + Im A)(Re B + Im B))
                                     */
#define TN_N_GEMM_CONFIGS 10      /* tile configurations per precision.  8 streams
                                     32-row bands past the whole B block of a column
                                     tile held in LDS: steps with one batch, at least
                                     2^10 rows and 2^4 columns, no split k and a
                                     column tile whose B block (all k) fits 64 KiB
                                     (complex64: 2^min(nn,7) columns and at most
                                     2^13 entries; split-BF16: 2^min(nn,6) columns
                                     and at most 2^12 entries).  9 is 8 with three
                                     real products per complex product (complex64,
                                     5 <= nk <= 7, column tiles of
                                     2^min(nn, 6, 12 - nk) >= 32 columns).  A step
                                     given 9 that it does not take runs as 8, and
                                     one given 8 that 8 does not take runs with the
                                     built-in rule's configuration                  */

typedef struct {
  int32_t precision;          /* tn_precision                                       */
  int32_t max_resident_bits;  /* cap on log2(slices computed together); -1 = auto   */
  int64_t workspace_limit;    /* bytes the arena may use; 0 = no limit              */
  uint32_t flags;             /* TN_FLAG_*                                          */
  int32_t gemm_config;        /* -1: per step from the tune table, else the built-in
                                 rule (steps with >= 2^18 rows: 9 in complex64, 8
                                 in split-BF16; others by column count);
                                 >= 0: this tile configuration for every GEMM step  */
  const int32_t* tune;        /* n_tune entries of 5 int32 {precision, nm, nn, nk,
                                 config}: measured best tile configuration for GEMM
                                 steps of that shape (log2 rows, cols, summed); a
                                 step uses the entry of its precision and nn with
                                 the nearest (nm, nk); copied at plan creation     */
  int32_t n_tune;
  int32_t checkpoint_policy;  /* tn_contract_backward: TN_CKPT_AUTO (every forward
                                 value stored if the backward workspace fits
                                 workspace_limit, else TN_CKPT_RECOMPUTE),
                                 TN_CKPT_ALL, or TN_CKPT_RECOMPUTE (values used
                                 inside one block of the schedule are recomputed
                                 before that block's adjoint; the blocks are
                                 chosen for the least recomputation within
                                 workspace_limit)                                  */
  int32_t n_variable;         /* variable_leaves[n_variable]: leaves whose values may
                                 change between calls (e.g. the output leaves of an
                                 amplitude batch).  The steps that depend on none
                                 of them and on no outer sliced index are the
                                 invariant steps; their results consumed by other
                                 steps stay in the workspace after tn_contract_ex,
                                 so a later call with TN_CALL_REUSE_INVARIANT skips
                                 them (Sec. 3.2 shared work, kept across calls)  */
  const int32_t* variable_leaves;
  int32_t batch;              /* amplitude batch: 0 or 1 = none; > 1 (a power of
                                 two) adds one index of dimension batch, id
                                 n_index, as the leading axis of every leaf in
                                 batched_leaves (their device buffers hold batch
                                 variants of the leaf, batch-major) and as the
                                 leading open index (the output is batch-major):
                                 entry b is the contraction with every batched
                                 leaf at its variant b, e.g. the amplitudes of a
                                 batch of outcomes, which share every step that
                                 no batched leaf reaches (Sec. 3.2).  Step,
                                 chain and leaf numbering are unchanged; the
                                 added index counts in the plan's index ids.
                                 TN_E_UNSUPPORTED if batch is not a power of two,
                                 TN_E_INVALID for a leaf id out of range or
                                 listed twice, or no leaf listed              */
  int32_t n_batched;
  const int32_t* batched_leaves;
} tn_plan_options;

typedef enum { TN_CKPT_AUTO = 0, TN_CKPT_ALL = 1, TN_CKPT_RECOMPUTE = 2 } tn_checkpoint_policy;

typedef struct {
  int32_t n_tensors, n_steps, n_index, n_sliced;
  int32_t n_open_bits;            /* log2 of the output elements per slice         */
  int32_t n_resident_bits;        /* log2 of slices contracted together in HBM     */
  int32_t n_outer_bits;           /* log2 of outer iterations                       */
  int32_t max_log2_per_slice;     /* largest per-slice intermediate, log2 elements  */
  int32_t max_log2_resident;      /* largest intermediate as held in HBM, log2      */
  int32_t n_launches;             /* kernel launches of one tn_contract (all slices) */
  int64_t n_slices;
  int64_t out_elems;              /* complex128 elements per output row             */
  int64_t workspace_bytes;        /* bytes tn_contract needs                        */
  int64_t workspace_backward_bytes; /* bytes tn_contract_backward needs             */
  int64_t arena_bytes;            /* peak intermediate bytes (with deletion)        */
  int64_t bytes_no_deletion;      /* intermediate bytes if nothing were freed       */
  /* complex multiply-adds (one CMAC = 8 real flops) */
  double cmac_reuse;              /* shared work done once, all slices resident     */
  double cmac_noreuse;            /* N_sl x per-slice cost (Eq. sliced_flops)       */
  double cmac_exec;               /* what tn_contract executes with this plan       */
  double cmac_per_slice;          /* FLOP_sl of Eq. sliced_flops                    */
  double f_sl;                    /* shared fraction of Eq. task_based_amplitude_flops */
  double bytes_min_exec;          /* algorithmic HBM bytes of one tn_contract       */
  /* where each slice's result lives in the root tensor (log2 strides):
   * output bit j (lsb first, row-major over the open indices) at 2^root_open_log2[j];
   * resident slice bit j at 2^root_res_log2[j], which is bit res_slicebit[j] of
   * the slice id; outer iteration bit j is bit outer_slicebit[j] of the slice id. */
  int8_t root_open_log2[48];
  int8_t root_res_log2[48];
  int8_t res_slicebit[48];
  int8_t outer_slicebit[48];
  int32_t n_chains;               /* fused chains of stream steps (one launch each) */
  int32_t n_segments;             /* persistent launches of small steps             */
  int64_t segment_table_bytes;    /* control tables of the persistent segments      */
  int64_t segment_table_offset;   /* their byte offset inside the workspace         */
  int32_t n_phase0;               /* schedule positions 0 .. n_phase0-1 run once
                                     (they depend on no outer sliced index)         */
  int32_t backward_policy;        /* TN_CKPT_ALL or TN_CKPT_RECOMPUTE (in effect)   */
  int32_t backward_blocks;        /* blocks of the backward schedule                */
  int32_t n_invariant;            /* schedule positions 0 .. n_invariant-1: the
                                     invariant steps (0 without variable leaves)    */
  double cmac_backward_recompute; /* multiply-adds the backward recomputes          */
  double cmac_invariant;          /* multiply-adds of the invariant steps           */
  int32_t n_launches_reuse;       /* launches of a call that reuses them            */
  int32_t reserved_info;
} tn_plan_info;

/* One step as scheduled (tests, benchmarks, autotuning). */
typedef struct {
  int32_t a, b, c;            /* SSA ids: leaves 0..n-1, step k creates n+k       */
  int32_t phase;              /* 0: once, 1: once per outer iteration             */
  int32_t kind;               /* kernel family chosen for the step                */
  int32_t nb, nm, nn, nk;     /* bits of batch / row / column / summed indices    */
  int32_t inst_bits;          /* log2 instances (slices) computed by this step    */
  int32_t tile;               /* GEMM tile configuration (kind == GEMM)           */
  double cmac;                /* multiply-adds per execution                      */
  /* log2 strides (elements) of each bit, least significant index bit first;
   * A holds batch,m,k; B holds batch,k,n; C holds batch,m,n. */
  int8_t sA_b[48], sB_b[48], sC_b[48];
  int8_t sA_m[48], sC_m[48];
  int8_t sB_n[48], sC_n[48];
  int8_t sA_k[48], sB_k[48];
  int64_t c_offset;           /* arena byte offset of the result (-1: the result
                                 stays inside a fused chain and is never stored)  */
  int64_t c_bytes;
  int32_t chain;              /* fused chain holding the step, or -1              */
  int32_t chunks;             /* split-k kernels and GEMM steps split over k: chunks
                                 of the summed bits, added up in a fixed order (1:
                                 no split)                                          */
  int32_t tile_run;           /* the GEMM tile configuration that runs: tile, or
                                 where a stream configuration (8, 9) does not take
                                 the step's shape the one it falls back to (see
                                 TN_N_GEMM_CONFIGS); -1 for other kinds           */
  int32_t tiny_batch;         /* batch of tiny steps running the step (one launch
                                 of one workgroup), or -1                         */
  int32_t tiny_level;         /* its level inside the batch: the steps of one
                                 level run at once, levels one after another     */
} tn_step_info;

/* One fused chain as planned (tests).  A chain runs steps first..last (path
 * order) in one launch over tiles of the running tensor: the tile bits of the
 * chain input are loaded into LDS slots, every step maps the tile through its
 * small operand, and the tile bits of the chain output are stored.  Bit j of a
 * tile-local index sits in LDS slot in_slot[j] / out_slot[j] and at log2
 * stride in_log2[j] / out_log2[j] in HBM; bit q of the tile number has HBM
 * strides pas_in[q] / pas_out[q]. */
typedef struct {
  int32_t step;               /* step index                                      */
  int32_t nrow, nk, nn, nbb;  /* row / summed / new bits, batch bits of B         */
  int8_t kslot[8], nslot[8];  /* LDS slots of summed and new bits                 */
  int8_t kB[8], nB[8];        /* B strides of summed and new bits                 */
  int8_t rslot[12];           /* LDS slots of the row bits                        */
  int8_t bB[12], bpas[12];    /* batch bits: B stride and tile-number bit         */
} tn_chain_step_info;

typedef struct {
  int32_t first, last, phase, tile_bits;
  int32_t n_in, n_out, n_passive, n_steps;
  int8_t in_slot[12], in_log2[12], out_slot[12], out_log2[12];
  int8_t pas_in[40], pas_out[40];
  tn_chain_step_info st[8];
} tn_chain_info;

/*
 * Build a plan.  Arguments:
 *   n_tensors, ranks[n_tensors]     leaf tensors and their ranks
 *   index_ids[sum ranks]            index ids of every leaf, concatenated, each
 *                                   in 0..n_index-1, in the leaf's axis order
 *   index_dims[n_index]             dimension of every index (power of two)
 *   open_ids[n_open]                open (output) indices
 *   path[2*n_steps]                 SSA pairs, n_steps = n_tensors - 1 (Sec. 2.3)
 *   sliced_ids[n_sliced]            sliced indices (Sec. 2.4), not open
 *   opts                            may be NULL (defaults: complex64, auto)
 * Returns TN_E_INVALID for a malformed network or path, TN_E_UNSUPPORTED for a
 * dimension that is not a power of two or a tensor above 2^40 elements.
 * Needs no GPU.
 */
tn_status tn_plan_create(int32_t n_tensors, const int32_t* ranks, const int32_t* index_ids,
                         int32_t n_index, const int32_t* index_dims, int32_t n_open,
                         const int32_t* open_ids, int32_t n_steps, const int32_t* path,
                         int32_t n_sliced, const int32_t* sliced_ids,
                         const tn_plan_options* opts, tn_plan_t* out);

/* Plan statistics (Eqs. sliced_flops and task_based_amplitude_flops, memory
 * with and without deletion of intermediates, Sec. 4 Fig. 8).  Needs no GPU. */
tn_status tn_plan_query(tn_plan_t plan, tn_plan_info* out);

/* Schedule of step ``step`` (0 .. n_steps-1, path order).  Needs no GPU. */
tn_status tn_plan_step(tn_plan_t plan, int32_t step, tn_step_info* out);

/*
 * Contract.  leaves[n_tensors]: device complex64 tensors (read only).
 * slice_ids[n_slice_ids]: slices to include (NULL, 0 = all, in id order).
 * out_mode TN_OUT_SUM: out = sum of the selected slices, out_elems complex128.
 * out_mode TN_OUT_PER_SLICE: out[i] = slice slice_ids[i] (or slice i),
 *   n_slice_ids (or n_slices) rows of out_elems complex128.
 * ws / ws_bytes: device workspace of at least info.workspace_bytes bytes.
 * The sum over slices is accumulated in float64 in a fixed order, so results
 * are reproducible run to run.  Fused chains of stream steps run as one
 * launch each.  With TN_FLAG_PERSISTENT, runs of small steps execute as
 * persistent launches whose schedule tables are copied from host memory into
 * the workspace once at entry (the host copy is staged before the call
 * returns).
 */
tn_status tn_contract(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                      int64_t n_slice_ids, int32_t out_mode, void* out, void* ws,
                      size_t ws_bytes, void* stream);

/*
 * tn_contract for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * workspace is the library's own file-scope device array of
 * TN_NOALLOC_WORKSPACE_BYTES bytes (one per GPU, held until the process
 * ends), so the caller passes only leaves and out.  Arguments and results as
 * in tn_contract; the call itself allocates nothing.
 * Returns TN_E_WORKSPACE when info.workspace_bytes exceeds
 * TN_NOALLOC_WORKSPACE_BYTES.  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and give wrong results; serialise them.  Nothing in the array needs to
 * start at zero (every buffer is written before it is read).
 */
#define TN_NOALLOC_WORKSPACE_BYTES (64ull << 20)
tn_status tn_contract_noalloc(tn_plan_t plan, const void* const* leaves,
                              const int64_t* slice_ids, int64_t n_slice_ids, int32_t out_mode,
                              void* out, void* stream);

/*
 * A contraction as a HIP graph (the launch sequence of one tn_contract,
 * captured once and replayed).  tn_graph_create records the kernels that
 * tn_contract would launch with these arguments -- leaves, slice_ids,
 * out_mode, out and ws are fixed in the graph: the caller keeps those device
 * buffers alive and unmoved for the graph's lifetime and may change the
 * leaves' contents between launches -- and instantiates the graph.  Capture
 * runs on an internal stream (default priority), so nothing is launched by
 * tn_graph_create itself; stream is unused and may be NULL.  tn_graph_launch
 * runs one contraction on `stream`; launches on one workspace must not
 * overlap.  Same errors as tn_contract, and TN_E_UNSUPPORTED for a plan with
 * persistent segments (their tables are uploaded from the host on every
 * call).  For callers that repeat a contraction of fixed shape on new leaf
 * values (batches of amplitudes, training loops), where per-launch host
 * overhead dominates small plans.
 */
typedef struct tn_graph_s* tn_graph_t;
tn_status tn_graph_create(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                          int64_t n_slice_ids, int32_t out_mode, void* out, void* ws,
                          size_t ws_bytes, void* stream, tn_graph_t* graph);
tn_status tn_graph_launch(tn_graph_t graph, void* stream);
/* Frees the graph; call it after its last launch has completed. */
void tn_graph_destroy(tn_graph_t graph);
/*
 * The adjoint as a HIP graph: records the kernels tn_contract_backward would
 * launch with these arguments (leaves, grad_out, grad_leaves, slice_ids and
 * ws fixed in the graph, as for tn_graph_create; the caller may change the
 * contents of the leaves and of grad_out between launches) and instantiates
 * it; tn_graph_launch then runs one backward pass, which ADDS the leaf
 * gradients into grad_leaves like tn_contract_backward (clear them between
 * launches for a fresh gradient).  Nothing is launched at creation; stream
 * is unused and may be NULL.  Same errors as tn_contract_backward.  For
 * training loops of fixed shape, where the adjoint's many small launches
 * make host overhead the bound.
 */
tn_status tn_graph_create_backward(tn_plan_t plan, const void* const* leaves,
                                   const void* grad_out, void* const* grad_leaves,
                                   const int64_t* slice_ids, int64_t n_slice_ids, void* ws,
                                   size_t ws_bytes, void* stream, tn_graph_t* graph);

/*
 * Adjoint of tn_contract with out_mode TN_OUT_SUM over the slices
 * slice_ids[n_slice_ids] (NULL, 0 = all; a slice listed twice counts twice):
 * the sum over slices (Eq. sliced_sum) and every pairwise step are linear in
 * each leaf, so the gradient is the reverse sweep of the steps, dA = dC.B^H
 * and dB = A^H.dC, with the gradients of results shared by many slices
 * summed over them, and with outer iterations accumulated.
 * grad_out: device complex128[out_elems], the gradient of a real loss with
 * respect to the output in PyTorch's convention (dL/d conj(out)).
 * grad_leaves[n_tensors]: device complex64 buffers shaped like the leaves;
 * the gradient of each leaf is ADDED to it (NULL entries are skipped).
 * ws / ws_bytes: at least info.workspace_backward_bytes (the plan's
 * checkpoint policy decides which forward values are stored and which are
 * recomputed).  Returns TN_E_WORKSPACE for a smaller workspace and
 * TN_E_INVALID for a slice id out of range.
 */
tn_status tn_contract_backward(tn_plan_t plan, const void* const* leaves, const void* grad_out,
                               void* const* grad_leaves, const int64_t* slice_ids,
                               int64_t n_slice_ids, void* ws, size_t ws_bytes, void* stream);

/*
 * tn_contract with call flags.  TN_CALL_REUSE_INVARIANT: the workspace holds
 * the invariant results of an earlier tn_contract / tn_contract_ex on this
 * plan and this workspace (same ws pointer) whose invariant leaves (all but
 * the plan's variable leaves) had the same values; the invariant steps are
 * not run again and their kept results are read instead.  The caller keys the
 * reuse by the invariant leaves' contents; the library cannot check it.
 * TN_E_INVALID if the flag is given for a plan without variable leaves.
 */
#define TN_CALL_REUSE_INVARIANT 1u
tn_status tn_contract_ex(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                         int64_t n_slice_ids, int32_t out_mode, void* out, void* ws,
                         size_t ws_bytes, void* stream, uint32_t call_flags);

/*
 * tn_contract with timing of one step: ev_start / ev_stop (hipEvent_t created
 * by the caller with timing enabled) are recorded on ``stream`` right before
 * the first launch and right after the last launch of step ``probe_step``
 * (its first execution when it runs once per outer iteration).  Otherwise
 * identical to tn_contract.
 */
tn_status tn_contract_probe(tn_plan_t plan, const void* const* leaves, const int64_t* slice_ids,
                            int64_t n_slice_ids, int32_t out_mode, void* out, void* ws,
                            size_t ws_bytes, void* stream, int32_t probe_step, void* ev_start,
                            void* ev_stop);

/*
 * Execution order of the steps: order[i] is the step run at position i
 * (n >= n_steps entries).  Positions 0 .. info.n_phase0-1 run once per call,
 * the rest once per outer iteration.  Needs no GPU.
 */
tn_status tn_plan_schedule(tn_plan_t plan, int32_t* order, int32_t n);

/*
 * Control tables of the persistent segments (TN_FLAG_PERSISTENT) exactly as
 * tn_contract copies them to ws + info.segment_table_offset for these leaf
 * and workspace pointers (which are only stored, never dereferenced: needs no
 * GPU).  blob receives info.segment_table_bytes bytes:
 *   bytes 0..255          header; int32 word 0 is the error word that every
 *                         segment launch sets to 1 when a wait timed out;
 *   per (segment, execution) lay[i] gives the byte offsets (from the start
 *   of blob) of
 *     off_desc   n_steps descriptors of 272 bytes: A, B, C device pointers,
 *                int32 nb, nm, nn, nk, n_items, item0, dep0, dep1 (segment
 *                positions of producer steps inside the segment, -1 = none),
 *                then 24-entry int8 log2-stride arrays sA_b, sB_b, sC_b,
 *                sA_m, sC_m, sB_n, sC_n, sA_k, sB_k;
 *     off_items  n_items int32: the segment position of each work item
 *                (work items are claimed in this order);
 *     off_ctr    zeroed int32 counters: word 0 the ticket, word 32*(1+s)
 *                the completed items of segment position s.
 * lay[max_lay] receives one entry per (segment, execution), *n_lay their
 * number; TN_E_INVALID if blob_bytes or max_lay is too small.
 */
typedef struct {
  int32_t segment, execution;  /* segment index, outer iteration (0 for phase 0) */
  int32_t n_steps, n_items;
  int32_t first_pos;           /* schedule position of the segment's first step  */
  int32_t reserved;
  int64_t off_desc, off_items, off_ctr;
} tn_segment_layout;
tn_status tn_plan_segment_tables(tn_plan_t plan, const void* const* leaves, void* ws,
                                 void* blob, int64_t blob_bytes, tn_segment_layout* lay,
                                 int32_t max_lay, int32_t* n_lay);

/*
 * Backward schedule of the plan (tests and diagnostics; needs no GPU).  Per
 * node (leaves 0..n_tensors-1, then one per step; 2*n_tensors-1 entries):
 * keep (0: value recomputed inside its block, 1: stored from the forward
 * pass, 2: not needed), frontier (1: a phase-0 result consumed by a phase-1
 * step, whose gradient accumulates over outer iterations), and workspace byte
 * offsets of the value in the forward pass, of the recomputed value and of
 * the gradient (-1: none).  block_of[n_steps]: block of each schedule
 * position (tn_plan_schedule order).  fuse_chain[info.n_chains] (may be
 * NULL): 1 if the chain runs as one fused launch in the backward's forward
 * pass.
 */
tn_status tn_plan_backward_tables(tn_plan_t plan, int8_t* keep, int8_t* frontier,
                                  int64_t* value_off, int64_t* recompute_off, int64_t* grad_off,
                                  int32_t* block_of, int8_t* fuse_chain);

/* Chain ``i`` (0 <= i < info.n_chains) of the plan. */
tn_status tn_plan_chain(tn_plan_t plan, int32_t i, tn_chain_info* out);

void tn_plan_destroy(tn_plan_t plan);

const char* tn_last_error(void);

/*
 * Bit permutation of one tensor (the transpose of the TTGT decomposition,
 * Sec. 3.1).  in / out: device complex64, 2^nbits elements each.  Element
 * with index bits (i_0 .. i_{nbits-1}) is read at sum_j i_j 2^in_log2[j] and
 * written at sum_j i_j 2^out_log2[j]; both stride lists must be permutations
 * of 0..nbits-1.  nbits <= 40.
 */
tn_status tn_permute(const void* in, void* out, int32_t nbits, const int8_t* in_log2,
                     const int8_t* out_log2, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TN_H_ */
