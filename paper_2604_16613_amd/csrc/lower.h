// Host lowering: realised circuit text -> the tables the device stages consume.
//
// The circuit is lowered to the space-time error propagation graph of paper
// Sec. 2.3.1 in an implicit form: operations are scheduled as soon as possible
// into layers in which every qubit is touched at most once, and a boundary b
// (0 <= b <= L) sits before layer b. Each (boundary, qubit) owns an X and a Z
// vertex (symplectic doubling, Sec. 2.3.4). Instead of storing two successor
// indices per vertex, a layer is stored as its list of operations; the device
// applies each operation's successor rule to the X/Z vertices of its qubits
// (identity for idle qubits), which is the same straight-line program (Eq. 1)
// with the identity edges left implicit.
//
// Measurement leaves (Eq. 2): every measurement m owns the set of signature
// bits (detectors, then observables) whose definitions list m an odd number of
// times. Signature bits are packed into 64-bit words; detector bits occupy
// words [0, WD) and observable bits words [WD, WD + WO), so the long-lived
// observable columns are separate from the short-lived detector columns.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

struct gp_circuit_ir;

namespace gp {

enum OpKind : uint8_t {
  OP_H = 1, OP_S, OP_SQRTX, OP_CX, OP_CZ, OP_SWAP,
  OP_R, OP_RX, OP_M, OP_MX, OP_MR, OP_MRX
};

enum ChanKind : uint8_t { CH_X = 1, CH_Y, CH_Z, CH_DEP1, CH_DEP2 };

// op word: kind in bits 56..63, a in bits 28..55, b in bits 0..27.
// a = qubit (control for CX); b = second qubit, or the measurement index.
constexpr uint64_t kField = (1ull << 28) - 1;
inline uint64_t pack_op(uint32_t kind, uint32_t a, uint32_t b) {
  return (uint64_t(kind) << 56) | (uint64_t(a & kField) << 28) | uint64_t(b & kField);
}

// Compact op word for the device sweep: kind in bits 28..31, a in bits 14..27,
// b (second qubit, unused for one-qubit operations) in bits 0..13. Leaves
// reach the sweep through the per-column injection lists instead.
constexpr uint32_t kQubitBits = 14;
constexpr uint32_t kMaxSweepQubits = 1u << kQubitBits;
constexpr uint32_t kQField = kMaxSweepQubits - 1;
// Correlation level of a fault's Pauli (code: x on a | z on a << 1 | x on b <<
// 2 | z on b << 3), Table 1: 0 for products of X's or of Z's (IX, IZ, XI, XX,
// ZI, ZZ; one-qubit X, Z), 1 for a Y next to the identity or a mixed X/Z pair
// (IY, YI, XZ, ZX; one-qubit Y), 2 for a Y next to X, Y or Z. Level L keeps
// the faults of level <= L (L0 in L1 in L2 = every Pauli).
constexpr uint32_t pauli_level(uint32_t code) {
  const uint32_t a = code & 3u, b = (code >> 2) & 3u;  // per qubit: 0 I, 1 X, 2 Z, 3 Y
  if (a != 3u && b != 3u) return (a == 0u || b == 0u || a == b) ? 0u : 1u;
  return (a == 0u || b == 0u) ? 1u : 2u;
}

// The Pauli codes of a channel, in fault order: a DEPOLARIZE1 gives X, Y, Z; a
// DEPOLARIZE2 the fifteen non-identity codes in ascending order.
constexpr uint32_t channel_code(uint32_t kind, uint32_t k) {
  return kind == 5u ? k + 1u : kind == 4u ? (k == 0u ? 1u : k == 1u ? 3u : 2u) : kind == 1u ? 1u : kind == 2u ? 3u : 2u;
}
constexpr uint32_t channel_codes(uint32_t kind) { return kind == 5u ? 15u : kind == 4u ? 3u : 1u; }

// Faults a channel keeps at a correlation level, and the code of its k-th kept fault.
constexpr uint32_t kept_faults(uint32_t kind, uint32_t level) {
  uint32_t n = 0;
  for (uint32_t k = 0; k < channel_codes(kind); k++) n += pauli_level(channel_code(kind, k)) <= level;
  return n;
}
constexpr uint32_t kept_code(uint32_t kind, uint32_t level, uint32_t j) {
  for (uint32_t k = 0; k < channel_codes(kind); k++)
    if (pauli_level(channel_code(kind, k)) <= level && j-- == 0u) return channel_code(kind, k);
  return 0u;
}

// Both, tabulated once per (channel kind, level): n[kind][level] kept faults
// with Pauli codes code[kind][level][0 ..).
struct KeptCodes {
  uint8_t n[6][3];
  uint8_t code[6][3][15];
};
constexpr KeptCodes make_kept_codes() {
  KeptCodes t{};
  for (uint32_t kind = 1; kind <= 5; kind++)
    for (uint32_t level = 0; level <= 2; level++) {
      t.n[kind][level] = uint8_t(kept_faults(kind, level));
      for (uint32_t j = 0; j < t.n[kind][level]; j++) t.code[kind][level][j] = uint8_t(kept_code(kind, level, j));
    }
  return t;
}
inline constexpr KeptCodes kKeptCodes = make_kept_codes();

// Compact ops one LDS op window of the sweep holds.
constexpr uint32_t kSweepWinOps = 4096;
// Circuits of at most this many qubits (so at most this many ops in a layer)
// get windows of this many ops: small enough for the sweep's small shape.
constexpr uint32_t kSmallWinOps = 1024;
// Sweep items that run at once: one per CU of the target GPU (256 on gfx950).
constexpr uint32_t kSweepSlots = 256;
// An observable column is not cut into ranges of fewer faults than this.
constexpr uint64_t kMinObsChunkFaults = 8192;
inline uint32_t pack_op32(uint32_t kind, uint32_t a, uint32_t b) {
  return (kind << 28) | ((a & kQField) << kQubitBits) | (b & kQField);
}

// One circuit of a batch, as the device sees it (a single compile is a batch
// of one). Qubits, layers, boundaries and windows are the circuit's own; the
// bases say where its entries start in the concatenated tables.
struct BranchDesc {
  uint32_t n_qubits, n_layers;
  uint32_t lob;        // layer offsets and layer windows: entries [lob, lob + n_layers + 1)
  uint32_t bb;         // boundary tables (channel, fault, bitmap offsets; cover rows): [bb, bb + n_layers + 2)
  uint32_t wb, nw;     // word columns [wb, wb + nw)
  uint32_t wd;         // of which detector columns
  uint32_t n_det;      // detectors (observable k is output as bit n_det + k)
  uint32_t n_obs;      // observables
  uint32_t wib, n_win; // op windows [wib, wib + n_win)
  uint32_t fb, fe;     // fault positions [fb, fe)
};

struct Lowered {
  uint32_t n_qubits = 0, n_layers = 0, n_meas = 0, n_det = 0, n_obs = 0;
  uint32_t wd = 0, wo = 0, w = 0;     // word columns: detector, observable, total
  uint64_t n_faults = 0;

  std::vector<uint64_t> ops;          // sorted by layer
  std::vector<uint32_t> layer_off;    // L + 1
  std::vector<uint32_t> leaf_off;     // n_meas + 1
  std::vector<uint32_t> leaf_bits;    // internal bit index, sorted per measurement
  std::vector<uint32_t> meas_layer;   // n_meas

  // channels, sorted by (boundary, program order)
  std::vector<uint32_t> chan_qa, chan_qb;   // qb = UINT32_MAX for one-qubit channels
  std::vector<uint8_t> chan_kind;
  std::vector<double> chan_rate;            // rate in sorted order
  std::vector<uint32_t> chan_src;           // program-order channel index
  std::vector<uint32_t> chan_foff;          // C + 1: first fault position of each channel
  std::vector<uint32_t> bnd_chan_off;       // L + 2: channels at boundary b
  std::vector<uint32_t> bnd_fault_off;      // L + 2: fault positions at boundary b

  // word columns and sweep work items
  std::vector<int32_t> col_top;             // highest layer holding a leaf bit of the column (-1: none)
  std::vector<int32_t> col_lo;              // lowest such layer
  std::vector<uint64_t> col_base;           // slab offset: word of (column w, position p) at base[w] + p
  uint64_t slab_words = 0;
  uint32_t level = 2;                       // correlation level the faults were kept at
  std::vector<uint32_t> item_col, item_blo, item_bhi;  // emission boundaries [blo, bhi]

  std::vector<uint64_t> fnv_pow;            // w + 1 entries: FNV prime^(8k) mod 2^64

  // device sweep inputs
  std::vector<uint32_t> ops32;              // compact op words, same order as ops
  // per column: the leaf words it receives (Eq. 2), one entry per (column,
  // measurement), ordered by layer from the top down: the measurement's layer,
  // its qubit, and the 64-bit word of leaf bits that fall in this column
  std::vector<uint32_t> inj_off;            // w + 1
  std::vector<uint32_t> inj_layer, inj_qubit;
  std::vector<uint64_t> inj_word;
  std::vector<uint32_t> inj_next;           // per entry: first entry (column-relative) of a lower layer

  // hash work chunks: at most 256 consecutive fault positions of one boundary
  std::vector<uint32_t> hchunk_pos, hchunk_bnd;

  // op windows of the sweep: layers cut from the top down into ranges of at
  // most kSweepWinOps ops; window k (k grows downward) holds layers
  // [win_lo[k], win_lo[k-1]) and its ops start at win_obase[k]
  std::vector<uint32_t> layer_win;          // per layer: its window
  std::vector<uint32_t> win_lo, win_obase, win_cnt;

  // non-zero-word bitmaps: per boundary b, ceil(faults at b / 64) words
  // starting at bnd_bm_off[b] (L + 2 entries); column w's bitmaps start at
  // col_bm_base[w] (boundaries 0 .. its top leaf layer)
  std::vector<uint32_t> bnd_bm_off;
  std::vector<uint64_t> col_bm_base;
  uint64_t bm_words = 0;

  // batch view: one descriptor per circuit, the circuit of every sweep item
  // and hash chunk, and the most word columns of any circuit
  std::vector<BranchDesc> branches;
  std::vector<uint32_t> item_branch, hchunk_branch;
  uint32_t w_max = 0;

  // Empty tables, keeping the vectors' storage: a driver lowers circuit after
  // circuit into one Lowered without touching fresh pages each time.
  void reset();
};

// Concatenate independently lowered circuits into one batch: tables are
// appended and rebased (operations, channels, fault positions, columns, slab
// and bitmap words, injections, windows are global; qubits, layers and
// boundaries stay per circuit, reached through the descriptors). Sweep items
// are ordered by the number of layers they sweep, longest first.
void merge_branches(const std::vector<Lowered>& in, Lowered& out);
void merge_branches(const std::vector<const Lowered*>& in, Lowered& out);

struct LowerError {
  int code;
  std::string msg;
};

// Lower `text`; `rates` (if non-null) overrides the channel rates in program
// order. `sweep_slots` is the number of sweep items that run at once (one per
// CU); observable columns are cut into ranges that fill the slots the
// detector columns leave. Returns 0 or a negative GP_E_* status with err set.
// Observable columns are cut into boundary ranges of equal estimated sweep
// time: a layer costs 1, emitting a boundary costs 1 + fault_cost per fault
// there (the default was measured at d = 25; gp_autotune measures others).
constexpr double kDefaultFaultCost = 6.2e-4;

int lower_circuit(const char* text, size_t len, const double* rates, size_t n_rates,
                  uint32_t sweep_slots, Lowered& out, LowerError& err, uint32_t level = 2,
                  double fault_cost = kDefaultFaultCost);

// The same for the binary form of a circuit (gp_circuit_ir in gp.h): the
// same tables as lowering the equivalent text. Errors name the operation.
int lower_ir(const ::gp_circuit_ir& ir, const double* rates, size_t n_rates, uint32_t sweep_slots, Lowered& out,
             LowerError& err, uint32_t level = 2, double fault_cost = kDefaultFaultCost);

// Re-apply a rate array to an already lowered circuit (same structure).
int apply_rates(Lowered& lw, const double* rates, size_t n_rates, LowerError& err);

constexpr uint64_t kFnvOffset = 14695981039346656037ull;
constexpr uint64_t kFnvPrime = 1099511628211ull;

}  // namespace gp
