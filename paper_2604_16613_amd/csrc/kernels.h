// Device stages of the compiler (gfx950). Launch wrappers take device pointers
// and enqueue on the given stream; none of them synchronises.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lower.h"

namespace gp {

// Device-side status block shared by the kernels of one compile.
struct DevHeader {
  uint32_t n_seg;      // classes found after sorting
  uint32_t empty_seg;  // class index of an empty signature, or 0xFFFFFFFF (none after compaction)
  uint32_t n_edges;    // hyperedges
  uint32_t flags;      // FLAG_* bits
  uint64_t n_bits;     // total signature bits over all hyperedges
  uint64_t n_words;    // stage-1 signature words written (= words the hash reads)
  uint32_t n_live;     // faults with a non-empty signature (the sorted ones)
  uint32_t n_big;      // classes with more faults than one thread merges
  uint64_t n_nz_words; // non-zero signature words stored by stage 1
  uint32_t flags_seen; // FLAG_* bits raised by any compile since the host last cleared this word
  uint32_t lookback_passes;  // bit p: a tile of radix pass p gave up its look-back (with FLAG_LOOKBACK)
};

enum : uint32_t {
  FLAG_GAUGE = 1u,      // a detector/observable is sensitive right after a reset/measurement
  FLAG_COLLISION = 2u,  // equal class keys with different check hashes
  FLAG_OVERFLOW = 4u,   // output signature bits exceed the reserved capacity
  FLAG_LOOKBACK = 8u,   // a sort tile gave up waiting for its predecessor: the pass's placement is
                        // wrong, so every later grouping kernel returns at once and the host redoes
                        // the compile (an error if it happens again)
  FLAG_BUCKET = 16u,    // a bucket of the bucket grouping exceeded its LDS capacity (redo with the full sort)
};

// Stage-2 grouping: 0 = buckets where they pay (up to kBucketMaxFaults: one
// stable pass on the top key digit, then every bucket sorted and merged in
// LDS; from kBucket16MinFaults to kBucket16MaxFaults: two stable passes on the
// top two digits, then every 16-bit bucket in LDS), else the full radix sort;
// 1 = always the full radix sort; 2 = the 16-bit buckets wherever the key has
// the digits.
enum : uint32_t { SORT_AUTO = 0, SORT_FULL = 1, SORT_BUCKET16 = 2 };
constexpr uint32_t kBuckets = 256;         // buckets = values of the top 8-bit digit
constexpr uint32_t kBucketCap = 8192;      // faults one bucket sorts in LDS
// bucket grouping is used up to this many faults (mean bucket <= 6144)
constexpr uint64_t kBucketMaxFaults = uint64_t(kBuckets) * 6144;
constexpr uint32_t kBuckets16 = 65536;     // buckets = values of the top two digits
constexpr uint32_t kBucket16Cap = 2048;    // faults one 16-bit bucket sorts in LDS
// 16-bit buckets are used from kBucket16MinFaults (mean bucket >= 183;
// below it a work-group's fixed cost per bucket makes the full sort faster)
// up to kBucket16MaxFaults (mean bucket <= 1024)
constexpr uint64_t kBucket16MinFaults = 12000000;
constexpr uint64_t kBucket16MaxFaults = uint64_t(kBuckets16) * 1024;

constexpr uint32_t kNone = 0xFFFFFFFFu;
// look-back rounds (each ends in a short sleep) before a sort tile gives up
constexpr uint32_t kSpinLimit = 1u << 22;
constexpr int kTile = 4096;       // items per tile in the sort, scan and compaction kernels
constexpr int kMaxPasses = 8;     // 8-bit digits of a 64-bit key

// Per fault position: what the merge gathers for each class member, in one
// 16-byte record (one random sector per member instead of two).
struct __align__(16) FaultRec {
  double p;      // fault probability
  uint64_t chk;  // check hash of the signature
};

// Per fault position, written by the hash for the edge writer: which covered
// columns hold non-zero words, the signature weight and the boundary row (in
// the batch's boundary tables), read in one access per representative.
struct __align__(16) EdgeRec {
  uint64_t nzm;
  uint32_t popc;
  uint32_t bnd;
};

// Per fault position that represents its class (the class's lowest
// position), written by the merge for the output pass: the merged
// probability and the class's members as a range of the sorted positions.
struct __align__(16) RepRec {
  double q;
  uint32_t first;  // first index of the members in the sorted positions (ord)
  uint32_t cnt;    // member count
};

// Hyperedges are numbered by their representative's position: hyperedge e
// is the class of the e-th representative in position order, so the
// hyperedges of a batch come out circuit by circuit (a circuit's positions are
// contiguous) and each circuit's in the order it has when compiled alone.
// Output tiles of kTile positions; a tile's count is packed as
// (representatives << kRepShift) | signature bits.
constexpr int kRepShift = 34;

// Everything one compile reads or writes on the device.
struct DevState {
  // lowered tables (inputs, uploaded per circuit)
  const uint32_t* layer_off;
  const uint32_t* chan_qa;
  const uint32_t* chan_qb;
  const uint8_t* chan_kind;
  const double* chan_rate;
  const uint32_t* chan_src;    // per channel (lowered order): its program-order number
  const uint32_t* chan_foff;
  const uint32_t* bnd_chan_off;
  const uint32_t* bnd_fault_off;
  const int32_t* col_top;
  const int32_t* col_lo;
  const uint64_t* col_base;
  const uint32_t* item_col;
  const uint32_t* item_blo;
  const uint32_t* item_bhi;
  const uint64_t* fnv_pow;
  const uint32_t* ops32;       // compact op words for the sweep
  const uint32_t* inj_off;     // per column: injection entries
  const uint32_t* inj_layer;
  const uint32_t* inj_qubit;
  const uint64_t* inj_word;
  const uint32_t* inj_next;
  const uint32_t* hchunk_pos;  // hash chunks: first position, boundary
  const uint32_t* hchunk_bnd;
  const uint32_t* bnd_bm_off;  // per boundary: first word of its bitmap within a column's bitmaps
  const uint64_t* col_bm_base; // per column: first word of its bitmaps
  const BranchDesc* branch;    // per circuit of the batch
  const uint32_t* item_branch; // per sweep item / hash chunk: its circuit
  const uint32_t* hchunk_branch;
  const uint32_t* layer_win;   // per layer: its op window
  const uint32_t* win_lo;      // per op window: lowest layer, first op, op count
  const uint32_t* win_obase;
  const uint32_t* win_cnt;

  // sizes
  // most qubits / layers / op windows of any circuit; word columns in all and
  // in the widest circuit; circuits in the batch
  uint32_t n_qubits, n_layers, n_det, wd, w;
  uint32_t w_max, n_branch;
  uint32_t n_chan, n_items;
  uint32_t n_faults;
  uint32_t n_hchunks;
  uint32_t n_win;
  uint32_t level;       // correlation level (Table 1) the faults were kept at
  uint32_t max_win_ops;  // most ops in one op window
  // class key: 0 = FNV-1a of the signature (kept to its low key_bits bits);
  // 1 = FNV-1a mixed with the check hash (used after a key collision)
  uint32_t key_mode;
  uint32_t key_bits;
  uint32_t n_pass;      // radix passes (8-bit digits) over the class key
  uint32_t sort_mode;   // SORT_*
  uint32_t sweep_shape; // stage-1 work-group shape: 0 automatic, 1 = 1024 threads, 2 = 256 threads
  uint32_t item_xcd;    // 1: sweep work-group b runs the item of its XCD's contiguous share (all items resident)
  uint32_t spin_limit;  // look-back rounds a sort tile waits for a predecessor before giving up
  uint32_t max_tiles;   // tiles the sort/compaction scratch is sized for

  // work buffers
  uint64_t* slab;        // stage-1 signature words, column slabs (only non-zero words are stored)
  uint64_t* bm;          // per (column, boundary): one bit per fault position, set where the word is non-zero
  int32_t* cover_lo;     // per column: lowest boundary written
  uint32_t* cov;         // per boundary row: covered columns, ascending (rows of w_max)
  uint32_t* ncov;        // per boundary: number of covered columns
  FaultRec* frp;         // per fault position: probability and check hash
  FaultRec* crp;         // bucket grouping: the records of the partitioned pairs, in pair order
  uint32_t* frec;        // per fault position: qubit a | qubit b << 14 | Pauli code << 28 (b = a for one-qubit faults)
  uint64_t* key[2];      // class keys: per position (key[1]) then compacted, ping-pong in the sort
  uint32_t* val[2];      // fault positions riding with the keys
  uint32_t* popc;        // per fault position: signature weight
  EdgeRec* erec;         // per fault position: non-zero-word mask, weight, boundary row
  uint32_t* tile_cnt;    // per compaction tile: live faults, then their exclusive prefix
  uint64_t* tile_nzw;    // per compaction tile: non-zero signature words | (fault, covered column) pairs read << 32
  uint32_t* digit_tot;   // per pass: total count of each digit value (summed by the compaction tiles)
  uint32_t* lookback;    // per pass, tile and digit: published count with status bits
  uint32_t* tile_ctr;    // per pass: tile ticket counter
  uint32_t* tile_sum;    // scan tile sums
  uint32_t* segstart;    // full sort: first sorted index of each class
  uint32_t* big;         // classes too large for one thread
  uint32_t* b16_lo;      // 16-bit buckets: first and end sorted index (cleared per compile)
  uint32_t* b16_hi;
  uint32_t use_b16;      // this compile groups with 16-bit buckets (k_prepare clears their ranges)
  // the class structure a compile leaves for rate refreshes and the adjoint:
  uint32_t* ord;         // fault positions, classes contiguous, members in position order (set by enqueue_compile)
  uint32_t* e_first;     // per hyperedge: first index into ord, member count
  uint32_t* e_cnt;
  double* gfault;        // per fault position: dL/dp (adjoint)
  double* gq;            // per hyperedge: dL/dq (adjoint input)
  double* gr;            // per channel (lowered order): dL/d(rate) (adjoint output)
  // output in representative-position order
  uint64_t* rep_bm;      // per 64 fault positions: bit set where the position represents its class (cleared per compile)
  RepRec* rrec;          // per representative position: merged probability, members
  uint64_t* out_lb;      // output look-back words: hyperedges of tile t at [t], bits at [max_tiles + t]
  uint32_t* out_ctr;     // output tile ticket
  uint32_t* rep_pos;     // per hyperedge: its representative's position
  uint32_t* circ_eoff;   // per circuit: its first hyperedge (n_branch + 1 entries)
  uint32_t* edge_off32;  // per hyperedge: first bit (n_edges + 1)
  uint32_t* edge_bits;   // output signature bits (external numbering)
  double* edge_q;        // output probabilities
  uint64_t bits_cap;
  DevHeader* hdr;
  uint64_t* item_clock;  // per sweep item: device wall clock at start and end (profiling)
};

// Names of the kernels (for timing tables).
enum KernelId : int {
  K_PREPARE = 0, K_SWEEP, K_HASH, K_SCAN_SINGLE, K_COMPACT, K_ONESWEEP, K_HEADS_COUNT, K_HEADS_APPLY, K_REDUCE,
  K_REDUCE_BIG, K_EDGE_WRITE, K_BUCKET, K_BUCKET_BOUNDS, K_REP_LIST, K_COUNT
};
const char* kernel_name(int id);

// A hook the driver uses to time launches: called before and after each one.
struct LaunchHook {
  void (*before)(void* ctx, int kernel_id) = nullptr;
  void (*after)(void* ctx, int kernel_id) = nullptr;
  void* ctx = nullptr;
};

// Radix passes needed for `n` keys: enough key bits that two distinct classes
// share them with probability below about 2^-12 (collisions are still caught).
uint32_t sort_passes(uint64_t n);
// key bits a first (FNV-1a keyed) compile of n faults keeps: those its sort
// passes cover, at most cap
uint32_t class_key_bits(uint64_t n, uint32_t cap);

// Enqueue both stages for the lowered circuit described by `st`; st.ord is
// set to the buffer that then holds the class members.
hipError_t enqueue_compile(DevState& st, hipStream_t stream, const LaunchHook& hook);

// After a compile (and its fetch): per-fault probabilities from the channel
// rates now in the tables, then every hyperedge re-merged over the cached
// members with the compile's merge shape; n_edges hyperedges.
hipError_t enqueue_refresh(const DevState& st, uint32_t n_edges, hipStream_t stream);

// Adjoint of stage 2: with dL/dq per hyperedge in st.gq, dL/d(rate) per
// channel (lowered order) into st.gr.
hipError_t enqueue_rates_gradient(const DevState& st, uint32_t n_edges, hipStream_t stream);

// Stage 2 over the cached structure with every operand on the device (the
// rate refresh and its adjoint without host transfers). rates: per channel in
// program order; q, gq: per hyperedge (the output order); grates: per
// channel in program order. The forward writes q; the backward recomputes
// the per-fault probabilities at `rates` and writes grates.
hipError_t enqueue_aggregate(const DevState& st, uint32_t n_edges, const double* rates, double* q,
                             hipStream_t stream);
// gfault: the per-fault dL/dp buffer (null: the driver's st.gfault).
hipError_t enqueue_aggregate_backward(const DevState& st, uint32_t n_edges, const double* rates,
                                      const double* gq, double* grates, double* gfault, hipStream_t stream);

// A per-fault dL/dp buffer of kScratchFaults doubles (16 MiB) in a static
// device array, for the adjoint entry point that allocates nothing. Each GPU
// holds its own copy until the process ends. scratch_init(device), with
// `device` current, looks up this device's address once (later calls return
// at once); scratch_for(device) returns it, or null before scratch_init.
constexpr uint64_t kScratchFaults = uint64_t(1) << 21;
hipError_t scratch_init(int device);
double* scratch_for(int device);

// Dynamic LDS the sweep needs for n qubits, and the largest it may use.
size_t sweep_lds_bytes(uint32_t n_qubits);
// the 256-thread stage-1 work-group holds this compile's tables
bool sweep_small_fits(const DevState& st);
// Dynamic LDS the hash needs for w signature words.
size_t hash_lds_bytes(uint32_t w);
// Whether the bucket grouping's LDS fits this device (set by configure_kernels).
bool bucket_grouping_available();
// Largest word-column count the hash kernel stages in LDS.
constexpr uint32_t kMaxHashWords = 1024;
size_t sweep_lds_limit();
hipError_t configure_kernels();

}  // namespace gp
