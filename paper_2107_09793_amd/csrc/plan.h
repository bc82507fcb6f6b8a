// Contraction plan: everything the device schedule needs, computed on the
// host once per (network, path, slices).  No HIP dependency.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace tn {

constexpr int kMaxBits = 48;       // bits of one class in one step
constexpr int kMaxTensorBits = 40; // elements of any executed tensor <= 2^40

enum Kind : int32_t {
  KIND_SIMPLE = 0,   // one thread per output element, full k loop
  KIND_SPLITK = 1,   // few outputs, long k: chunked partial sums + fixed-order reduce
  KIND_STREAM = 2,   // one large operand streamed past a small one held on chip
  KIND_GEMM = 3,     // MFMA tiles with bit-gather operand loads
};

enum Precision : int32_t { PREC_C64 = 0, PREC_SPLIT_BF16 = 1 };

struct StepDesc {
  int32_t a, b, c;        // SSA ids
  int32_t phase;          // 0 once, 1 per outer iteration
  int32_t kind;
  int32_t inst_bits;      // log2 instances of this step, all slices resident
  std::vector<int8_t> bA, bB, bC, mA, mC, nB, nC, kA, kB;   // log2 strides
  double cmac;            // multiply-adds per execution
  int64_t c_off;          // arena byte offset of the result
  int64_t c_bytes;
  int64_t scratch_bytes;  // split-k partials
  int32_t splitk_chunks;
  int32_t tile;           // GEMM tile configuration
  bool small = false;     // runs inside a persistent segment
  bool tiny = false;      // runs inside a batch of tiny steps (one workgroup)
  int32_t chain = -1;     // chain group this step belongs to
  // 0: invariant (depends on no variable leaf and no outer index; its result
  // may be kept from an earlier call), 1: rest of phase 0, 2: phase 1.
  // Scheduled in that order; chains and segments never mix groups.
  int32_t group = 1;
};

// A run of consecutive small steps in the schedule executed by one launch.
struct Segment {
  int32_t begin, end;     // positions in Plan::sched
  int32_t n_items;        // work items (chunks of 256 outputs)
  int32_t phase;
};

constexpr int kSmallClassBits = 24;     // per class, to fit the device descriptor
constexpr int kTinyMaxSteps = 20;       // steps per batch of tiny steps
constexpr int kTinyClassBits = 14;      // per class, to fit the kernel arguments
// a tiny step: at most 2^kTinyCmacBits complex multiply-adds and
// 2^kTinyOutBits outputs, so that the one workgroup running a batch gives
// each thread a few outputs (the loads of one output wait on each other)
constexpr int kTinyCmacBits = 13;
constexpr int kTinyOutBits = 11;
constexpr int64_t kSmallStepBytes = 272; // sizeof the device descriptor
constexpr int64_t kCtrStride = 32;       // int32 slots between completion counters

// A chain: consecutive stream steps (path order) where each step's large
// operand is the previous step's result and its small operand is read whole
// per tile.  One launch runs the chain over tiles of the running tensor: a
// workgroup loads the tile bits of the chain input (the bits the chain
// contracts, plus low-stride bits for coalescing) into LDS, applies every step
// there, and writes the tile bits of the chain output.  Intermediate results
// of the chain never reach HBM.
constexpr int kChainMaxSteps = 8;
constexpr int kChainTileBits = 12;   // LDS tile: 2^12 complex64 per buffer
constexpr int kChainPassive = 40;    // bits enumerating tiles
constexpr int kChainBFloats = 4096;  // staged small operands in LDS, all steps (floats)
constexpr int kChainVElems = 512;    // of which complex entries of vector-unit steps

// Which chain steps run on the matrix cores: 4 <= 2^nk <= 64 summed and
// 8 <= 2^nn <= 32 new values with 2^(nk+nn) <= 512, at least 16 rows, and
// matrix cores not switched off (TN_FLAG_CHAIN_VALU).  Such a step stages
// the real embedding of its small operand (4 floats per complex entry); a
// vector-unit step stages the complex entries (2 floats each).  (Wider small
// operands, 2^(nk+nn) = 1024, were measured slower inside chains than as
// stand-alone GEMM launches: the larger staging area and register budget
// halve the chain kernel's occupancy.)
inline bool chain_mfma_shape(int nk, int nn) {
  return nk >= 2 && nk <= 6 && nn >= 3 && nn <= 5 && nk + nn <= 9;
}
inline bool chain_step_mfma(int nk, int nn, int nrow, uint32_t flags) {
  return !(flags & 32u) && chain_mfma_shape(nk, nn) && nrow >= 4;
}
// Split-BF16 matrix-core chain steps with 2^nk >= 32 need the register-heavy
// build of the chain kernel (the others run in the build that prefetches).
inline bool chain_needs_heavy(int nk, bool mfma, bool split) { return mfma && split && nk >= 5; }
// Floats a chain step stages: the complex entries (vector units), or B' in
// the lanes' order, padded to 8 complex k (split-BF16 k steps cover 16 reals).
inline int chain_staged_floats(int nk, int nn, bool mfma) {
  return mfma ? 4 * (nk < 3 ? 8 : 1 << nk) << nn : 2 << (nk + nn);
}


struct ChainStepDesc {
  int32_t step;                      // step index
  int32_t nrow;                      // live tile bits that are not summed
  std::vector<int8_t> kslot, nslot, rslot;   // LDS slots of summed / new / row bits
  std::vector<int8_t> kB, nB;        // small-operand strides of summed / new bits
  std::vector<int8_t> bB, bpas;      // batch bits: small-operand stride, passive-bit index
};

struct ChainGroup {
  int32_t first = 0, last = 0;       // step indices (path order), inclusive
  int32_t phase = 0;
  int32_t tile_bits = 0;             // slots used (LDS buffer = 2^tile_bits)
  std::vector<int8_t> in_slot, in_log2;    // input tile bits, input-stride order
  std::vector<int8_t> out_slot, out_log2;  // output tile bits, output-stride order
  std::vector<int8_t> pas_in, pas_out;     // passive bits: input / output strides
  std::vector<ChainStepDesc> st;
};

// Backward (adjoint) schedule.  The forward values a step's adjoint needs
// are either stored from the forward pass or recomputed: the schedule is cut
// into blocks; a value consumed in the block that produced it is freed in the
// forward pass and recomputed (and then kept) just before that block's
// adjoint runs, while a value crossing a block boundary (or the phase
// boundary) is stored from the forward pass until its consumer's adjoint.
// Every position its own block stores everything (no recomputation).
enum CheckpointPolicy : int32_t { CKPT_AUTO = 0, CKPT_ALL = 1, CKPT_RECOMPUTE = 2 };

struct BwdPlan {
  int32_t policy = CKPT_ALL;         // the policy in effect (ALL or RECOMPUTE)
  std::vector<int32_t> block_of;     // block id of each schedule position
  std::vector<int32_t> block_begin;  // first position of each block (ascending)
  std::vector<uint8_t> keep;         // per node: 0 recomputed, 1 stored, 2 not needed (root)
  std::vector<uint8_t> frontier;     // per node: phase-0 result consumed by a phase-1 step
  std::vector<uint8_t> fuse_chain;   // per chain: fused launch in the backward's forward pass
  std::vector<int64_t> fwd_off;      // per node: value offset in the forward pass (-1 none)
  std::vector<int64_t> rec_off;      // per node: value offset when recomputed (-1 none)
  std::vector<int64_t> grad_off;     // per node: gradient offset (-1 none)
  int64_t arena_bytes = 0;
  int64_t scratch_bytes = 0;         // split-k partials of forward and adjoint products
  double cmac_recompute = 0;         // multiply-adds recomputed (all outer iterations)
};

struct LeafDesc {
  std::vector<int32_t> bits;      // global bit ids (all), layout order lsb first
  std::vector<int8_t> log2s;      // stride of each bit
  std::vector<int32_t> outer_bits; // subset of bits fixed per outer iteration
  std::vector<int8_t> outer_log2s;
};

struct Plan {
  // input (copied)
  int32_t n_tensors = 0, n_index = 0;
  std::vector<std::vector<int32_t>> leaf_index;
  std::vector<int32_t> index_dims, index_w, index_bit0;
  std::vector<int32_t> open_ids, sliced_ids;
  std::vector<int32_t> path;       // 2 * n_steps
  int32_t precision = PREC_C64;
  uint32_t flags = 0;
  int32_t gemm_config = -1;
  std::vector<int32_t> tune;       // 5 ints per entry

  // derived
  int32_t n_bits = 0;                        // global bits
  std::vector<uint8_t> bit_kept;             // sliced or open
  std::vector<uint8_t> bit_sliced, bit_outer;
  std::vector<std::vector<int32_t>> node_bits;  // all-resident bit set (sorted)
  std::vector<std::vector<int32_t>> node_ebits; // executed bit set (outer removed)
  std::vector<std::vector<int8_t>> node_log2s;  // stride per executed bit (same order)
  std::vector<std::vector<int32_t>> node_layout; // executed bits in layout order (lsb first)
  std::vector<int32_t> node_phase;
  std::vector<int32_t> node_sv;              // |S_v| in bits (sliced bits below)
  std::vector<LeafDesc> leaves;
  std::vector<StepDesc> steps;               // path order
  std::vector<int32_t> sched;                // step indices, execution order
  int32_t n_phase0 = 0;                      // sched[0 .. n_phase0) run once
  int32_t n_invariant = 0;                   // sched[0 .. n_invariant): invariant steps
  std::vector<uint8_t> leaf_variable;        // leaves that may change between calls
  std::vector<Segment> segments;             // persistent launches
  std::vector<Segment> tiny_runs;            // batches of tiny steps (schedule positions)
  std::vector<int8_t> tiny_level;            // per schedule position: level inside its batch
  std::vector<ChainGroup> chains;            // fused chains of stream steps
  std::map<int32_t, std::vector<int32_t>> chain_in_low;  // chain input node -> bits to put lowest
  std::vector<std::vector<int32_t>> chain_sum_bits;      // summed bits of each step
  int64_t persist_bytes = 0;                 // control region for one tn_contract

  // outer / resident split (whole sliced indices)
  std::vector<int32_t> outer_idx, resident_idx;   // sliced index ids
  int32_t outer_bits = 0, resident_bits = 0, sliced_bits = 0, open_bits = 0;

  // root / output
  std::vector<int8_t> root_open_log2;     // stride in root of each output bit (lsb first)
  std::vector<int8_t> root_res_log2;      // stride in root of each resident slice bit
  std::vector<int32_t> res_slicebit;      // slice-id bit position of each resident bit
  std::vector<int32_t> outer_slicebit;    // slice-id bit position of each outer bit
  std::vector<int32_t> outer_bit_ids;     // global bit id of each outer bit (same order)

  // memory
  int64_t arena_bytes = 0, bytes_no_deletion = 0, scratch_bytes = 0;
  int64_t ctrl_bytes = 0, workspace_bytes = 0, workspace_bwd_bytes = 0;
  int32_t ckpt_policy = CKPT_AUTO;    // requested
  BwdPlan bwd;

  // statistics
  double cmac_reuse = 0, cmac_noreuse = 0, cmac_exec = 0, cmac_sl = 0, f_sl = 0;
  double bytes_min_exec = 0;
  int32_t max_log2_sl = 0, max_log2_res = 0;
  int64_t n_slices = 1;
  int32_t n_launches = 0;
};

// Kernel family for a step shape; split-k chunk count and scratch bytes.
int32_t choose_kind(int nb, int nm, int nn, int nk, uint32_t flags, int32_t* chunks,
                    int64_t* scratch);

// GEMM tile configuration for a step shape: forced, tune table, or rule.
// Configuration kGemmStream streams 32-row bands past a B block resident in
// LDS (few columns and summed values against many rows); a shape it does not
// take (stream_gemm_shape) runs with the rule's tile configuration instead.
constexpr int kNumGemmConfigs = 10;
constexpr int kGemmStream = 8;
// Configuration kGemmStreamGauss: the stream kernel with three real products
// per complex product (complex64, column tiles of 32 or 64); a shape it does
// not take runs as kGemmStream.
constexpr int kGemmStreamGauss = 9;
int32_t choose_tile(const Plan& p, int nm, int nn, int nk);
int32_t rule_tile(int nn);
bool stream_gemm_shape(int nb, int nm, int nn, int nk, int32_t chunks, int32_t precision);
bool stream_gauss_shape(int nb, int nm, int nn, int nk, int32_t chunks, int32_t precision);
// The configuration that runs a GEMM step given configuration `tile`: the
// stream configurations fall back (9 -> 8 -> the rule's) on shapes they do
// not take.
int32_t tile_run(int32_t tile, int nb, int nm, int nn, int nk, int32_t chunks, int32_t precision);
// Column tile (log2 columns) and k tile (log2 complex k) of the stream kernel.
void stream_gemm_tile(int nn, int nk, int32_t precision, int* ln, int* lkt);

// Builds the plan; returns empty string on success, else an error message.
// *unsupported is set when the input is valid but outside what is supported.
std::string build_plan(Plan& p, int32_t n_tensors, const int32_t* ranks,
                       const int32_t* index_ids, int32_t n_index, const int32_t* index_dims,
                       int32_t n_open, const int32_t* open_ids, int32_t n_steps,
                       const int32_t* path, int32_t n_sliced, const int32_t* sliced_ids,
                       int32_t precision, int32_t max_resident_bits, int64_t ws_limit,
                       uint32_t flags, int32_t gemm_config, const int32_t* tune, int32_t n_tune,
                       int32_t ckpt_policy, const int32_t* variable_leaves, int32_t n_variable,
                       bool* unsupported);

}  // namespace tn
