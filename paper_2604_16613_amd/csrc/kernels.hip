// Device stages for gfx950 (wave64, 160 KB LDS per CU).
//
// Stage 1 (paper Sec. 3.1, Alg. 1, Eq. 1-2): one work item sweeps the layers
// of the circuit backwards for one 64-bit word column of the class bit
// vectors. The column's X/Z vertex words of all qubits live in LDS; a layer
// is applied in place, one thread per operation (the operations of a layer
// touch disjoint qubits, so their updates are independent), while the next
// layer's operations are already being fetched. After each layer the faults
// placed at that boundary read their qubits' words and write their signature
// word (composite Paulis are XORs of the X and Z words, Sec. 2.3.4) into the
// column's slab. A column's sweep starts at the highest layer that holds one of
// its leaves and stops once its frame is all zero below its last leaf: every
// lower boundary is then zero in that column and is not written.
//
// Stage 2 (Sec. 3.2, Eq. 3): per fault, the 64-bit FNV-1a hash of its
// signature's 8W octets (zero words only multiply by prime^8) as class key, an
// independent check hash, the signature weight and a mask of its non-zero
// words. Faults with an empty signature are dropped by a stable compaction
// (their class is never output). The rest are sorted by key with a stable LSD
// radix sort: one histogram for all passes, then one kernel per 8-bit pass
// that ranks a tile in LDS, finds its global offsets by looking back at the
// tiles before it, and writes runs of equal digits contiguously. Class heads,
// merged probabilities q <- q + p(1 - 2q) in sorted (fault) order, and the
// hyperedges' bit lists follow. If two faults share a key but not a check
// hash, the host re-runs the compile keyed on both hashes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "kernels.h"
#include "lower.h"

namespace gp {

namespace {

constexpr int kSweepBlock = 1024;
constexpr uint32_t kXcds = 8;          // accelerator dies of the MI355X, each with its own L2
constexpr int kWinOps = int(kSweepWinOps);  // compact ops per LDS window buffer (two buffers)
constexpr int kEmitPre = 8;            // fault records per thread fetched during the op phase
constexpr int kLofsMax = 2048;         // layer offsets staged in LDS when the circuit has fewer layers
constexpr int kInjLds = 512;           // a column's injections staged in LDS when it has at most this many
constexpr int kWinTableLds = 512;      // op windows whose table is staged in LDS
constexpr int kBranchLds = 1024;
// LDS table sizes of the two sweep shapes (work-group size kBlk)
template <int kBlk> struct SweepShape;
template <> struct SweepShape<1024> {
  static constexpr int kLofs = kLofsMax, kInj = kInjLds, kWinTab = kWinTableLds, kWin = kWinOps;
};
template <> struct SweepShape<256> {
  static constexpr int kLofs = 512, kInj = 256, kWinTab = 128, kWin = int(kSmallWinOps);
};       // circuits of a batch whose first fault the edge writer stages in LDS
constexpr int kBlock = 256;
constexpr int kPerThread = kTile / kBlock;
constexpr int kScanSingleBlock = 1024;
constexpr uint32_t kBigSegment = 64;   // classes with more faults reduce in a whole block
constexpr uint32_t kLbAgg = 1u << 30;  // look-back status: tile aggregate published
constexpr uint32_t kLbPre = 2u << 30;  // look-back status: inclusive prefix published
constexpr uint32_t kLbMask = (1u << 30) - 1;
constexpr int kLookWin = 8;             // look-back: predecessor tiles read per round
constexpr uint32_t kHashBmw = 5;        // bitmap words 256 consecutive positions span at most

// Barrier that orders LDS only: global loads issued before it (prefetches)
// stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exclusive scan over a block with one barrier: every thread sums the wave
// totals itself. s_wave needs BLOCK/64 entries; callers barrier before the
// next use of s_wave.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_scan_1sync(uint32_t v, uint32_t* s_wave, uint32_t& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) s_wave[wv] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < BLOCK / 64; ++k) {
    const uint32_t x = s_wave[k];
    off += k < wv ? x : 0u;
    tot += x;
  }
  total = tot;
  return off + inc - v;
}

// Exclusive scan over a block; s_wave needs BLOCK/64 + 1 entries and holds the
// block total in s_wave[BLOCK/64] on return. Callers barrier before reuse.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wave) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t inc = wave_inclusive_scan(v);
  if (lane == 63) s_wave[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = 0; k < BLOCK / 64; ++k) {
      uint32_t t = s_wave[k];
      s_wave[k] = run;
      run += t;
    }
    s_wave[BLOCK / 64] = run;
  }
  __syncthreads();
  return s_wave[wv] + inc - v;
}

// MurmurHash3's 64-bit finaliser (public domain): a bijective avalanche mix.
__device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ uint64_t check_term(uint32_t w, uint64_t v) {
  return fmix64(v + 0x9E3779B97F4A7C15ull * (uint64_t(w) + 1));
}

// Per-fault probability of one Pauli of a channel (see gp.h): the p with
// (1-2p)^k = 1 - x, i.e. p = -expm1(log1p(-x)/k)/2.
__device__ __forceinline__ double fault_probability(uint32_t kind, double r) {
  if (kind == CH_DEP1) return -0.5 * expm1(0.5 * log1p(-4.0 * r / 3.0));
  if (kind == CH_DEP2) return -0.5 * expm1(0.125 * log1p(-16.0 * r / 15.0));
  return r;
}

__device__ __forceinline__ uint32_t digit_of(uint64_t k, uint32_t pass) { return uint32_t(k >> (8 * pass)) & 255u; }

// Sets a status flag of this compile and records it in the union of the
// flags raised since the host last cleared that union.
__device__ __forceinline__ void raise_flag(DevHeader* hdr, uint32_t f) {
  atomicOr(&hdr->flags, f);
  atomicOr(&hdr->flags_seen, f);
}

// A partition pass gave up its look-back: the pairs after it are misplaced
// (positions may be stale), so the grouping kernels that follow do nothing.
// The merged class whose lowest fault position is `rep`: its record at that
// position and its bit in the representative bitmap (the output pass numbers
// the hyperedges by these bits in position order).
__device__ __forceinline__ void put_rep(const DevState& st, uint32_t rep, double q, uint32_t first, uint32_t cnt) {
  RepRec r;
  r.q = q;
  r.first = first;
  r.cnt = cnt;
  st.rrec[rep] = r;
  atomicOr(reinterpret_cast<unsigned long long*>(st.rep_bm) + (rep >> 6), 1ull << (rep & 63));
}

__device__ __forceinline__ bool grouping_aborted(const DevHeader* hdr) {
  return (__hip_atomic_load(&hdr->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & FLAG_LOOKBACK) != 0u;
}

// ------------------------------------------------------------------ prepare

// the Pauli codes each channel kind keeps at each correlation level
__constant__ KeptCodes c_kept = make_kept_codes();

// A block takes kPrepChan consecutive channels: one thread per channel computes
// the per-fault probability and the qubits and marks its faults in an LDS map
// (fault -> channel), then the block writes the faults of those channels
// (consecutive positions) one thread per fault, coalesced.
constexpr uint32_t kMaxChanFaults = sizeof(KeptCodes::code[0][0]);  // faults of one channel at most

// output tiles of a compile of n faults (at least one)
__device__ __forceinline__ uint32_t ntiles_out(uint32_t n) { return n ? (n + kTile - 1) / kTile : 1u; }

// Channels per block: small blocks spread a compile's channels over several
// work-groups per CU (one 256-channel block per CU wrote the records of about
// 3,800 faults with 4 waves).
constexpr uint32_t kPrepChan = 64;

__global__ __launch_bounds__(kBlock) void k_prepare(DevState st) {
  __shared__ double s_p[kPrepChan];
  __shared__ uint32_t s_q[kPrepChan];          // qubit a | qubit b << 14 | kind << 28
  __shared__ uint32_t s_off[kPrepChan + 1];    // first fault of each channel, from the block's first
  __shared__ uint8_t s_ch[kPrepChan * kMaxChanFaults];  // channel (in the block) of each fault
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t stride = gridDim.x * blockDim.x;
  const uint32_t n_blk = (st.n_chan + kPrepChan - 1) / kPrepChan;
  for (uint32_t cb = blockIdx.x; cb < n_blk; cb += gridDim.x) {
    const uint32_t c0 = cb * kPrepChan, nc = min(kPrepChan, st.n_chan - c0);
    const uint32_t f_lo = st.chan_foff[c0];
    if (threadIdx.x < nc) {
      const uint32_t c = c0 + threadIdx.x;
      const uint32_t kind = st.chan_kind[c];
      const uint32_t qa = st.chan_qa[c] & kQField;
      // a one-qubit channel names its qubit twice, so that "both qubits'
      // frame words are zero" is the test for an empty word (see k_sweep)
      const uint32_t qb = kind == CH_DEP2 ? (st.chan_qb[c] & kQField) : qa;
      s_p[threadIdx.x] = fault_probability(kind, st.chan_rate[c]);
      s_q[threadIdx.x] = qa | (qb << kQubitBits) | (kind << 28);
      const uint32_t o = st.chan_foff[c] - f_lo, o1 = st.chan_foff[c + 1] - f_lo;
      s_off[threadIdx.x] = o;
      for (uint32_t i = o; i < o1; ++i) s_ch[i] = uint8_t(threadIdx.x);
    }
    if (threadIdx.x == 0) s_off[nc] = st.chan_foff[c0 + nc] - f_lo;
    __syncthreads();
    const uint32_t nf = s_off[nc];
    for (uint32_t i = threadIdx.x; i < nf; i += kBlock) {
      const uint32_t lo = s_ch[i];
      const uint32_t q = s_q[lo], kind = q >> 28;
      st.frp[f_lo + i].p = s_p[lo];
      // Pauli code: x on a | z on a << 1 | x on b << 2 | z on b << 3
      const uint32_t code = c_kept.code[kind][st.level][i - s_off[lo]];
      st.frec[f_lo + i] = (q & ((1u << 28) - 1u)) | (code << 28);
    }
    __syncthreads();
  }
  for (uint32_t w = gid; w < st.w; w += stride) st.cover_lo[w] = 0;
  for (uint32_t i = gid; i < (st.n_faults + 63) / 64; i += stride) st.rep_bm[i] = 0;
  for (uint32_t t = gid; t < ntiles_out(st.n_faults); t += stride) {
    st.out_lb[t] = 0;
    st.out_lb[st.max_tiles + t] = 0;
  }
  if (gid == 0) *st.out_ctr = 0;
  const uint32_t ntiles = (st.n_faults + kTile - 1) / kTile;
  for (uint32_t t = gid; t < ntiles + 1; t += stride) {
    st.tile_cnt[t] = 0;
    st.tile_nzw[t] = 0;
  }
  // look-back words of every pass (each pass owns max_tiles * 256 of them)
  const uint32_t per_pass = ntiles * 256;
  for (uint32_t i = gid; i < st.n_pass * per_pass; i += stride)
    st.lookback[size_t(i / per_pass) * st.max_tiles * 256 + i % per_pass] = 0;
  if (gid < kMaxPasses) st.tile_ctr[gid] = 0;
  for (uint32_t i = gid; i < st.n_pass * 256; i += stride) st.digit_tot[i] = 0;
  if (st.use_b16)
    for (uint32_t i = gid; i < kBuckets16; i += stride) {
      st.b16_lo[i] = 0;
      st.b16_hi[i] = 0;
    }
  if (gid == 0) {
    st.hdr->lookback_passes = 0;
    st.hdr->n_seg = 0;
    st.hdr->empty_seg = kNone;
    st.hdr->n_edges = 0;
    st.hdr->flags = 0;
    st.hdr->n_bits = 0;
    st.hdr->n_words = 0;
    st.hdr->n_live = 0;
    st.hdr->n_big = 0;
    st.hdr->n_nz_words = 0;
  }
}

// ------------------------------------------------------------------ stage 1

__device__ __forceinline__ int nzd(uint64_t nv, uint64_t ov) { return int(nv != 0) - int(ov != 0); }

// Apply one compact operation backwards to the frame (the (X_q, Z_q) pair of
// qubit q at frame[q]). Both qubits' pairs are read up front (a one-qubit op
// reads qubit 0's and ignores it). A measurement takes its leaf word for this
// column from pend[q] (scattered there from the column's injection list) and
// clears it.
__device__ __forceinline__ void apply_op(uint32_t op, ulonglong2* frame, uint64_t* pend, int& dnz, int& gauge) {
  const uint32_t kind = op >> 28;
  const uint32_t a = (op >> kQubitBits) & kQField;
  const uint32_t b = op & kQField;
  const ulonglong2 pa = frame[a], pb = frame[b];
  const uint64_t xa = pa.x, za = pa.y, xb = pb.x, zb = pb.y;
  switch (kind) {
    case OP_H:
      frame[a] = make_ulonglong2(za, xa);
      break;
    case OP_S: {  // X -> XZ
      const uint64_t n = xa ^ za;
      frame[a].x = n;
      dnz += nzd(n, xa);
      break;
    }
    case OP_SQRTX: {  // Z -> XZ
      const uint64_t n = xa ^ za;
      frame[a].y = n;
      dnz += nzd(n, za);
      break;
    }
    case OP_CX: {  // X_c -> X_c X_t, Z_t -> Z_t Z_c
      const uint64_t nxa = xa ^ xb, nzb = zb ^ za;
      frame[a].x = nxa;
      frame[b].y = nzb;
      dnz += nzd(nxa, xa) + nzd(nzb, zb);
      break;
    }
    case OP_CZ: {  // X_a -> X_a Z_b, X_b -> X_b Z_a
      const uint64_t nxa = xa ^ zb, nxb = xb ^ za;
      frame[a].x = nxa;
      frame[b].x = nxb;
      dnz += nzd(nxa, xa) + nzd(nxb, xb);
      break;
    }
    case OP_SWAP:
      frame[a] = pb;
      frame[b] = pa;
      break;
    case OP_R:  // a Z error right after a Z reset must be invisible
      gauge |= za != 0;
      frame[a] = make_ulonglong2(0, 0);
      dnz -= int(xa != 0) + int(za != 0);
      break;
    case OP_RX:
      gauge |= xa != 0;
      frame[a] = make_ulonglong2(0, 0);
      dnz -= int(xa != 0) + int(za != 0);
      break;
    case OP_M: {  // X before the measurement flips it (leaf) and persists
      gauge |= za != 0;
      const uint64_t n = xa ^ pend[a];
      pend[a] = 0;
      frame[a].x = n;
      dnz += nzd(n, xa);
      break;
    }
    case OP_MX: {
      gauge |= xa != 0;
      const uint64_t n = za ^ pend[a];
      pend[a] = 0;
      frame[a].y = n;
      dnz += nzd(n, za);
      break;
    }
    case OP_MR: {  // the reset erases what the measurement did not see
      gauge |= za != 0;
      const uint64_t n = pend[a];
      pend[a] = 0;
      frame[a] = make_ulonglong2(n, 0);
      dnz += nzd(n, xa) - int(za != 0);
      break;
    }
    case OP_MRX: {
      gauge |= xa != 0;
      const uint64_t n = pend[a];
      pend[a] = 0;
      frame[a] = make_ulonglong2(0, n);
      dnz += nzd(n, za) - int(xa != 0);
      break;
    }
    default:
      break;
  }
}

// Sum over the wave of per-lane values with |v| < 2^(BITS-1), by BITS ballots:
// scalar popcounts instead of a chain of cross-lane LDS permutes. Every lane
// of the wave must be active.
template <int BITS>
__device__ __forceinline__ int wave_total(int v) {
  const uint32_t u = uint32_t(v + (1 << (BITS - 1)));
  int s = 0;
#pragma unroll
  for (int bit = 0; bit < BITS; ++bit) s += int(__popcll(__ballot((u >> bit) & 1u))) << bit;
  return s - 64 * (1 << (BITS - 1));
}

// One work item = one word column (or one boundary range of an observable
// column). LDS holds the column's frame, two parity buffers of pending leaf
// words, two op windows (the circuit's layers cut from the top into ranges of
// at most kWinOps ops; the next window is fetched into registers while the
// current one is applied), the layer, fault and bitmap offsets and the
// column's injection list.
// Layers above the item's emission range only transform the frame: one
// barrier each, and no global memory access besides the window prefetch.
// Layers in the range apply the ops (one thread per op) while the next
// boundary's fault records are in flight, then emit the non-zero signature
// words of the boundary's faults (one thread per fault, coalesced) with a
// ballot bitmap of which words are non-zero.
// The count of non-zero frame words (for the early exit) is taken once at the
// top of the emission range, then kept per wave as a running sum of the
// changes and published in per-wave LDS slots (two sets, alternating).

template <bool kStaged, int kBlk>
__global__ __launch_bounds__(kBlk) void k_sweep(DevState st) {
  // kBlk = 1024: one item per CU (large circuits); 256: a smaller LDS
  // footprint so that several items share a CU (many items of small circuits)
  constexpr int kLofs = SweepShape<kBlk>::kLofs;
  constexpr int kInj = SweepShape<kBlk>::kInj;
  constexpr int kWinN = SweepShape<kBlk>::kWin;  // ops per window buffer
  constexpr int kPreN = kWinN / kBlk;
  extern __shared__ __align__(16) uint64_t lds[];
  __shared__ int s_wnz[2][kBlk / 64];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  // Work-groups are dispatched to the XCDs round robin (b mod kXcds). When
  // every item is resident at once, XCD x takes a contiguous share of the
  // items (columns in time order), so the fault records of a layer are
  // fetched into one XCD's L2 instead of all eight.
  uint32_t item = blockIdx.x;
  if (st.item_xcd) {
    const uint32_t x = item % kXcds, q = gridDim.x / kXcds, r = gridDim.x % kXcds;
    item = x * q + min(x, r) + item / kXcds;
  }
  const BranchDesc br = st.branch[st.item_branch[item]];
  const uint32_t n = br.n_qubits;
  // this circuit's layer, boundary and window tables
  const uint32_t* layer_off = st.layer_off + br.lob;
  const uint32_t* layer_win = st.layer_win + br.lob;
  const uint32_t* bnd_fault_off = st.bnd_fault_off + br.bb;
  const uint32_t* bnd_bm_off = st.bnd_bm_off + br.bb;
  const uint32_t* win_lo = st.win_lo + br.wib;
  const uint32_t* win_obase = st.win_obase + br.wib;
  const uint32_t* win_cnt = st.win_cnt + br.wib;
  uint64_t* frame = lds;
  uint64_t* pend = frame + 2 * size_t(n);  // two buffers, by layer parity
  uint64_t* sinj_w = pend + 2 * size_t(n);
  uint32_t* opbuf = reinterpret_cast<uint32_t*>(sinj_w + kInj);
  uint32_t* slofs = opbuf + 2 * kWinN;
  uint32_t* sbfo = slofs + kLofs;
  uint32_t* sbmo = sbfo + kLofs + 1;
  uint32_t* sinj_l = sbmo + kLofs + 1;
  uint32_t* sinj_q = sinj_l + kInj;
  uint32_t* sinj_n = sinj_q + kInj;
  uint32_t* swin = sinj_n + kInj;  // per op window: lowest layer, first op, op count

  if (tid == 0) st.item_clock[2 * item] = wall_clock64();
  const uint32_t w = st.item_col[item];
  const int top = st.col_top[w];
  const int clo = st.col_lo[w];
  const int blo = int(st.item_blo[item]);
  const int bhi = int(st.item_bhi[item]);
  uint64_t* out = st.slab + st.col_base[w];
  uint64_t* obm = st.bm + st.col_bm_base[w];
  // kStaged: the layer offsets (and the column's injections, where they fit)
  // sit in LDS, so the layer loop reads no global memory besides the window
  // prefetch and the emission's fault records
  constexpr bool lofs_lds = kStaged;
  const uint32_t i0 = st.inj_off[w];
  const uint32_t ni = st.inj_off[w + 1] - i0;
  // a column with more injections than the LDS list holds reads them from
  // global memory (the same for every thread of the item)
  const bool inj_lds = kStaged && ni <= uint32_t(kInj);

  for (uint32_t i = tid; i < 4 * n; i += kBlk) frame[i] = 0;  // frame and both pend buffers
  if (lofs_lds)
    for (uint32_t k = tid; k <= br.n_layers + 1; k += kBlk) {
      if (k <= br.n_layers) slofs[k] = layer_off[k];
      sbfo[k] = bnd_fault_off[k];
      sbmo[k] = bnd_bm_off[k];
    }
  if (inj_lds)
    for (uint32_t k = tid; k < ni; k += kBlk) {
      sinj_w[k] = st.inj_word[i0 + k];
      sinj_l[k] = st.inj_layer[i0 + k];
      sinj_q[k] = st.inj_qubit[i0 + k];
      sinj_n[k] = st.inj_next[i0 + k];
    }
  // the window table sits in LDS (kStaged): reading it from global memory with
  // scalar loads would make the next LDS wait also wait for them
  if (lofs_lds)
    for (uint32_t k = tid; k < br.n_win; k += kBlk) {
      swin[3 * k] = win_lo[k];
      swin[3 * k + 1] = win_obase[k];
      swin[3 * k + 2] = win_cnt[k];
    }
  auto WLO = [&](int k) -> uint32_t { return lofs_lds ? swin[3 * k] : win_lo[k]; };
  auto WOB = [&](int k) -> uint32_t { return lofs_lds ? swin[3 * k + 1] : win_obase[k]; };
  auto WCN = [&](int k) -> uint32_t { return lofs_lds ? swin[3 * k + 2] : win_cnt[k]; };
  // the op window holding the top layer, loaded directly
  int wid = int(layer_win[top]);
  uint32_t o_base = win_obase[wid];
  int wlo = int(win_lo[wid]);
  {
    const uint32_t cnt = win_cnt[wid];
    for (uint32_t i = tid; i < cnt; i += kBlk) opbuf[i] = st.ops32[o_base + i];
  }
  __syncthreads();
  auto LO = [&](int t) -> uint32_t { return lofs_lds ? slofs[t] : layer_off[t]; };
  auto BFO = [&](int t) -> uint32_t { return lofs_lds ? sbfo[t] : bnd_fault_off[t]; };
  auto BMO = [&](int t) -> uint32_t { return lofs_lds ? sbmo[t] : bnd_bm_off[t]; };
  auto INJ_L = [&](uint32_t k) -> int { return int(inj_lds ? sinj_l[k] : st.inj_layer[i0 + k]); };
  auto INJ_Q = [&](uint32_t k) -> uint32_t { return inj_lds ? sinj_q[k] : st.inj_qubit[i0 + k]; };
  auto INJ_W = [&](uint32_t k) -> uint64_t { return inj_lds ? sinj_w[k] : st.inj_word[i0 + k]; };
  auto INJ_N = [&](uint32_t k) -> uint32_t { return inj_lds ? sinj_n[k] : st.inj_next[i0 + k]; };
  // scatter the leaf words of layer t into its pend buffer; the layer of the
  // next injection group is kept in a register
  uint32_t ip = 0;
  int inj_t = ni ? INJ_L(0) : -1;
  uint32_t inj_e = ni ? INJ_N(0) : 0;
  auto scatter = [&](int t) {
    if (inj_t == t) {
      uint64_t* pb = pend + size_t(t & 1) * n;
      for (uint32_t k = ip + tid; k < inj_e; k += kBlk) pb[INJ_Q(k)] = INJ_W(k);
      ip = inj_e;
      inj_t = ip < ni ? INJ_L(ip) : -1;
      inj_e = ip < ni ? INJ_N(ip) : 0;
    }
  };
  scatter(top);
  // the next window (layers below wlo) into registers, if the item needs it;
  // its op count, first op and lowest layer stay in registers too, so that
  // the swap reads no table entry before it stores the window
  uint32_t pre[kPreN];
  uint32_t nbase = 0, ncnt = 0;
  int nwlo = 0;
  auto prefetch = [&]() {
    const bool need = wlo - 1 >= blo;
    ncnt = need ? WCN(wid + 1) : 0u;
    nbase = need ? WOB(wid + 1) : 0u;
    nwlo = need ? int(WLO(wid + 1)) : 0;
#pragma unroll
    for (int k = 0; k < kPreN; ++k) {
      const uint32_t i = tid + k * kBlk;
      pre[k] = i < ncnt ? st.ops32[nbase + i] : 0u;
    }
  };
  prefetch();
  __syncthreads();
  int cur = 0;
  int gauge = 0;
  int wave_nz = 0;   // this wave's running share of the non-zero word count
  uint32_t ck = 0;   // count publications so far (slot set ck & 1)
  uint32_t lo_hi = LO(top + 1);

  // the ops of layer t; dnz accumulates the change in non-zero frame words
  auto apply_layer = [&](int t, uint32_t lo_t, int& dnz) {
    const uint32_t* buf = opbuf + cur * kWinN;
    uint64_t* pb = pend + size_t(t & 1) * n;
    // a layer never exceeds a window
    for (uint32_t i = lo_t - o_base + tid; i < lo_hi - o_base; i += kBlk)
      apply_op(buf[i], reinterpret_cast<ulonglong2*>(frame), pb, dnz, gauge);
  };
  // publish this wave's running count in slot set ck & 1 (read after a barrier)
  auto publish = [&](int dnz) {
    wave_nz += wave_total<10>(dnz);
    if (lane == 0) s_wnz[ck & 1][wave] = wave_nz;
  };
  auto count_published = [&]() -> int {
    int nz = 0;
#pragma unroll
    for (int k = 0; k < kBlk / 64; ++k) nz += s_wnz[ck & 1][k];
    return nz;
  };
  // the next layer's leaf words, and the window swap when layer t ends it
  auto advance = [&](int t) {
    if (t - 1 >= blo) scatter(t - 1);
    if (t == wlo && t - 1 >= blo) {
      // the prefetched window becomes current (the other buffer is no longer
      // read), and the window after it is fetched into registers
      uint32_t* nb = opbuf + (cur ^ 1) * kWinN;
#pragma unroll
      for (int k = 0; k < kPreN; ++k) {
        const uint32_t i = tid + k * kBlk;
        if (i < ncnt) nb[i] = pre[k];
      }
      cur ^= 1;
      wid++;
      o_base = nbase;
      wlo = nwlo;
      prefetch();
    }
  };

  bool dead = false;
  int t = top;
  // the next layer's offsets are read before each barrier
  uint32_t lo_t = LO(top);
  // layers above the emission range: transform only, without counting the
  // frame's non-zero words (nothing is emitted there)
  for (; t > bhi; --t) {
    int unused = 0;
    apply_layer(t, lo_t, unused);
    advance(t);
    const uint32_t lo_n = LO(t > 0 ? t - 1 : 0);
    lds_barrier();
    lo_hi = lo_t;
    lo_t = lo_n;
  }
  if (bhi < top) {
    // count the non-zero words of the frame at boundary bhi + 1 once; the
    // emission layers keep the count by differences from here
    int cnt = 0;
    for (uint32_t i = tid; i < 2 * n; i += kBlk) cnt += int(frame[i] != 0);
    wave_nz = wave_total<10>(cnt);
    if (lane == 0) s_wnz[ck & 1][wave] = wave_nz;
    lds_barrier();
    const bool zero = bhi + 1 <= clo && count_published() == 0;
    ck++;
    // the frame is zero and no leaf lies below: this column is zero on every
    // boundary of this item's range (the item that holds the boundary where
    // it died records it)
    if (zero) dead = true;
  }
  if (!dead) {
    uint32_t f_hi = BFO(t + 1), f0 = BFO(t);
    // The Pauli records of boundary t's faults are loaded one layer ahead:
    // while layer t is applied and emitted, boundary t-1's records are in
    // flight (two register sets, the loop unrolled by two so that neither is
    // copied while its loads are outstanding).
    // Every load is issued whatever the boundary's fault count (indices past
    // it are clamped into the array and their values never used), so that
    // the number of loads in flight is known where the records are used and
    // the wait there covers only the loads that are needed.
    uint32_t recA[kEmitPre], recB[kEmitPre];
    const uint32_t f_last = st.n_faults ? st.n_faults - 1 : 0u;
    auto load_recs = [&](uint32_t (&r)[kEmitPre], uint32_t fa) {
#pragma unroll
      for (int k = 0; k < kEmitPre; ++k) r[k] = st.frec[min(fa + tid + k * kBlk, f_last)];
    };
    load_recs(recA, f0);
    // one boundary: returns true when the item is done (range end or the
    // frame died)
    auto step = [&](uint32_t (&rec)[kEmitPre], uint32_t (&nxt)[kEmitPre]) -> bool {
      // A: fetch the next boundary's records, then transform the frame from
      // boundary t+1 to boundary t, in place
      const uint32_t nf = f_hi - f0;
      const uint32_t f_n = BFO(t > 0 ? t - 1 : 0);
      load_recs(nxt, f_n);
      int dnz = 0;
      apply_layer(t, lo_t, dnz);
      advance(t);
      publish(dnz);
      const uint32_t lo_n = LO(t > 0 ? t - 1 : 0);
      lds_barrier();
      lo_hi = lo_t;
      const bool zero = t <= clo && count_published() == 0;
      ck++;
      // B: faults at boundary t, one per thread: signature word = XOR of the
      // X/Z words their Pauli selects (composite Paulis, Sec. 2.3.4);
      // consecutive threads store consecutive positions
      auto word_of = [&](uint32_t r) -> uint64_t {
        const uint32_t qa = r & kQField, qb = (r >> kQubitBits) & kQField, code = r >> 28;
        const ulonglong2 p0 = reinterpret_cast<const ulonglong2*>(frame)[qa];
        const ulonglong2 p1 = reinterpret_cast<const ulonglong2*>(frame)[qb];
        // most faults sit on qubits whose frame words are all zero (a
        // one-qubit fault names its qubit twice): skip the selection then
        if (((p0.x | p0.y) | (p1.x | p1.y)) == 0ull) return 0ull;
        return (p0.x & (0ull - (code & 1u))) ^ (p0.y & (0ull - ((code >> 1) & 1u))) ^
               (p1.x & (0ull - ((code >> 2) & 1u))) ^ (p1.y & (0ull - ((code >> 3) & 1u)));
      };
      // only non-zero words are stored; a ballot per wave records which
      // (bit i of bitmap word i / 64 of this boundary)
      uint64_t* bmp = obm + BMO(t);
#pragma unroll
      for (int k = 0; k < kEmitPre; ++k) {
        const uint32_t i = tid + k * kBlk;
        const uint64_t v = i < nf ? word_of(rec[k]) : 0ull;
        if (v) out[f0 + i] = v;
        const uint64_t msk = __ballot(v != 0);
        if (lane == 0 && i < nf) bmp[i >> 6] = msk;
      }
      for (uint32_t k = kEmitPre; k * kBlk < nf; ++k) {
        const uint32_t i = tid + k * kBlk;
        const uint64_t v = i < nf ? word_of(st.frec[f0 + i]) : 0ull;
        if (v) out[f0 + i] = v;
        const uint64_t msk = __ballot(v != 0);
        if (lane == 0 && i < nf) bmp[i >> 6] = msk;
      }
      if (zero) {
        // no leaf of this column lies below t and the frame is zero: every
        // lower boundary is zero in this column
        if (tid == 0) st.cover_lo[w] = t;
        dead = true;
        return true;
      }
      lo_t = lo_n;
      f_hi = f0;
      f0 = f_n;
      lds_barrier();
      --t;
      return t < blo;
    };
    while (!step(recA, recB) && !step(recB, recA)) {
    }
  }
  if (!dead && blo == 0) {
    // every qubit starts in |0>: a Z error at the very start must be invisible
    for (uint32_t q = tid; q < n; q += kBlk) gauge |= frame[2 * q + 1] != 0;
  }
  if (gauge) raise_flag(st.hdr, FLAG_GAUGE);
  if (tid == 0) st.item_clock[2 * item + 1] = wall_clock64();
}

// ------------------------------------------------------------------ stage 2

// FNV-1a over the 8W octets of each fault's signature (h <- (h ^ octet) *
// prime), a run of k zero words multiplying by prime^(8k); the check hash, the
// weight and the non-zero-word mask; live-fault and non-zero-word counts per
// compaction tile. One block = at most 256 positions of one boundary: it
// lists the columns that cover the boundary (top leaf layer >= b >= the
// column's lowest written boundary) in LDS with their slab bases and the
// bitmap words its positions span; the boundary's first chunk also stores
// the list for the edge writer and counts the boundary's words. Each thread
// then loads only its fault's non-zero words, up to eight at once.
__global__ __launch_bounds__(kBlock) void k_hash(DevState st) {
  extern __shared__ __align__(16) uint64_t hlds[];
  const uint32_t bi = st.hchunk_branch[blockIdx.x];
  const BranchDesc br = st.branch[bi];
  const uint32_t W = br.nw;  // this circuit's word columns (the LDS holds the widest circuit's)
  uint64_t* s_pow = hlds;                  // W + 1
  uint64_t* s_base = s_pow + W + 1;        // W: slab base of each covered column
  uint64_t* s_bmb = s_base + W;            // W: bitmap base of each covered column at this boundary
  uint64_t* s_bm = s_bmb + W;              // W * kHashBmw: the bitmap words this chunk spans
  uint32_t* s_w = reinterpret_cast<uint32_t*>(s_bm + size_t(W) * kHashBmw);  // W: covered columns
  __shared__ uint32_t s_wave[kBlock / 64 + 1];
  const uint32_t b = st.hchunk_bnd[blockIdx.x];  // the circuit's boundary
  const uint32_t gb = br.bb + b;                  // its row in the batch's boundary tables
  const uint32_t p0 = st.hchunk_pos[blockIdx.x];
  const uint32_t fb = st.bnd_fault_off[gb];
  const uint32_t p1 = min(p0 + uint32_t(kBlock), st.bnd_fault_off[gb + 1]);
  const uint32_t bmo = st.bnd_bm_off[gb];
  const uint32_t nwb = st.bnd_bm_off[gb + 1] - bmo;  // bitmap words of this boundary
  const uint32_t wb0 = (p0 - fb) >> 6;              // first of them this chunk touches
  const bool first_chunk = p0 == fb;
  for (uint32_t k = threadIdx.x; k <= W; k += kBlock) s_pow[k] = st.fnv_pow[k];
  uint32_t n = 0;
  for (uint32_t w0 = 0; w0 < W; w0 += kBlock) {
    const uint32_t wl = w0 + threadIdx.x, w = br.wb + wl;  // the circuit's column, the batch's
    uint32_t f = 0;
    if (wl < W) {
      const int top = st.col_top[w];
      f = (top >= 0 && int(b) <= top && int(b) >= st.cover_lo[w]) ? 1u : 0u;
    }
    const uint32_t at = block_exclusive_scan<kBlock>(f, s_wave);
    if (f) {
      s_w[n + at] = wl;
      s_base[n + at] = st.col_base[w];
      s_bmb[n + at] = st.col_bm_base[w] + bmo;
      if (first_chunk) st.cov[size_t(gb) * st.w_max + n + at] = w;
    }
    n += s_wave[kBlock / 64];
    __syncthreads();
  }
  if (first_chunk && threadIdx.x == 0) st.ncov[gb] = n;
  for (uint32_t i = threadIdx.x; i < n * kHashBmw; i += kBlock) {
    const uint32_t k = i / kHashBmw, j = i % kHashBmw;
    s_bm[i] = wb0 + j < nwb ? st.bm[s_bmb[k] + wb0 + j] : 0ull;
  }
  __syncthreads();
  const uint32_t pos = p0 + threadIdx.x;
  const bool valid = pos < p1;
  const uint32_t ib = (valid ? pos : p0) - fb;  // bit ib & 63 of bitmap word ib / 64 of the boundary
  const uint32_t wj = (ib >> 6) - wb0, bit = ib & 63;
  uint64_t h1 = kFnvOffset, h2 = 0, mask = 0;
  uint32_t wn = 0, weight = 0, nzw = 0;
  for (uint32_t seg = 0; seg < n; seg += 64) {
    // this fault's non-zero words among covered columns seg .. seg + 63
    const uint32_t cnt = min(64u, n - seg);
    uint64_t msk = 0;
    for (uint32_t q = 0; q < cnt; ++q) msk |= ((s_bm[(seg + q) * kHashBmw + wj] >> bit) & 1ull) << q;
    if (!valid) msk = 0;
    if (seg == 0) mask = msk;
    while (msk) {
      uint32_t kk[8];
      bool on[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        on[j] = msk != 0;
        kk[j] = on[j] ? seg + uint32_t(__builtin_ctzll(msk)) : 0u;
        msk &= msk - 1;
      }
      uint64_t vv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) vv[j] = on[j] ? st.slab[s_base[kk[j]] + pos] : 0ull;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (!on[j]) continue;
        const uint64_t v = vv[j];
        const uint32_t w = s_w[kk[j]];
        h1 *= s_pow[w - wn];
#pragma unroll
        for (int o = 0; o < 8; ++o) h1 = (h1 ^ ((v >> (8 * o)) & 0xffu)) * kFnvPrime;
        wn = w + 1;
        nzw++;
        h2 += check_term(w, v);
        weight += __popcll(v);
      }
    }
  }
  h1 *= s_pow[W - wn];
  if (bi) {
    // circuits of a batch share column numbers: a per-circuit salt keeps
    // equal signatures of different circuits in different classes
    h1 ^= fmix64(0x9e3779b97f4a7c15ull * bi);
    h2 += fmix64(0xc2b2ae3d27d4eb4full * bi);
  }
  uint64_t key = h1;
  if (st.key_mode == 1) key = h1 ^ fmix64(h2 ^ 0x5851f42d4c957f2dull);
  if (st.key_bits < 64) key &= (1ull << st.key_bits) - 1;
  if (valid) {
    st.key[1][pos] = key;
    st.frp[pos].chk = h2;
    st.popc[pos] = weight;
    st.erec[pos] = EdgeRec{mask, weight, gb};
  }
  // live faults and non-zero words per compaction tile: the chunk's
  // positions span at most two tiles; reduce over the block, then at most
  // four global atomics
  __shared__ uint32_t s_cnt[4];
  if (threadIdx.x < 4) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t ta = p0 / kTile;
  const bool live = valid && weight != 0;
  const bool in_a = pos / kTile == ta;
  const uint32_t c_a = wave_sum((live && in_a) ? 1u : 0u);
  const uint32_t c_b = wave_sum((live && !in_a) ? 1u : 0u);
  const uint32_t z_a = wave_sum(valid && in_a ? nzw : 0u);
  const uint32_t z_b = wave_sum(valid && !in_a ? nzw : 0u);
  if ((threadIdx.x & 63) == 0) {
    if (c_a) atomicAdd(&s_cnt[0], c_a);
    if (c_b) atomicAdd(&s_cnt[1], c_b);
    if (z_a) atomicAdd(&s_cnt[2], z_a);
    if (z_b) atomicAdd(&s_cnt[3], z_b);
  }
  __syncthreads();
  if (threadIdx.x == 0 && s_cnt[0]) atomicAdd(&st.tile_cnt[ta], s_cnt[0]);
  if (threadIdx.x == 1 && s_cnt[1]) atomicAdd(&st.tile_cnt[ta + 1], s_cnt[1]);
  // per tile: non-zero words (low half) and the (fault, covered column)
  // pairs this chunk read (high half), in one 64-bit add; the compaction sums
  // the tiles (one atomic per tile rather than one per boundary on a single
  // counter)
  const uint32_t in_tile_a = min(p1, (ta + 1) * uint32_t(kTile)) - p0;
  const uint64_t w_a = uint64_t(n) * in_tile_a, w_b = uint64_t(n) * (p1 - p0 - in_tile_a);
  if (threadIdx.x == 2 && (s_cnt[2] || w_a)) atomicAdd(&st.tile_nzw[ta], (w_a << 32) | s_cnt[2]);
  if (threadIdx.x == 3 && (s_cnt[3] || w_b)) atomicAdd(&st.tile_nzw[ta + 1], (w_b << 32) | s_cnt[3]);
}

// In-place exclusive scan of n (host value, or *n_dev when given) words by one
// block; each thread scans a contiguous chunk. The total goes to *total.
template <typename TotalT>
__global__ __launch_bounds__(kScanSingleBlock) void k_scan_single(uint32_t* data, uint32_t n_host,
                                                                  const uint32_t* n_dev, TotalT* total) {
  __shared__ uint32_t s_wave[kScanSingleBlock / 64 + 1];
  const uint32_t n = n_dev ? *n_dev : n_host;
  const uint32_t chunk = (n + kScanSingleBlock - 1) / kScanSingleBlock;
  const uint32_t b0 = min(n, threadIdx.x * chunk), b1 = min(n, b0 + chunk);
  uint32_t s = 0;
  for (uint32_t i = b0; i < b1; ++i) s += data[i];
  uint32_t run = block_exclusive_scan<kScanSingleBlock>(s, s_wave);
  for (uint32_t i = b0; i < b1; ++i) {
    const uint32_t v = data[i];
    data[i] = run;
    run += v;
  }
  if (threadIdx.x == 0 && total) *total = TotalT(s_wave[kScanSingleBlock / 64]);
}

// Lanes of the wave below this one whose bit is set in m.
__device__ __forceinline__ uint32_t lane_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
}

// Stable compaction of the live faults (non-empty signatures) into (key,
// position) pairs, adding this tile's digit counts of radix passes
// [p0, n_pass) to the totals. Round k of the tile covers positions [k*1024, k*1024+1024):
// consecutive lanes read consecutive positions and write consecutive
// compacted slots.
constexpr int kCompactBlock = 1024;
constexpr int kCompactRounds = kTile / kCompactBlock;
static_assert(kCompactRounds * (kCompactBlock / 64) == 64, "compaction offsets are scanned by one wave");

__global__ __launch_bounds__(kCompactBlock) void k_compact(DevState st, uint32_t p0) {
  constexpr int kWaves = kCompactBlock / 64;
  __shared__ uint32_t s_off[kCompactRounds * kWaves];  // per (round, wave): first slot in the tile
  __shared__ uint32_t s_hist[kMaxPasses][256];
  __shared__ uint32_t s_red[kWaves];
  const uint32_t tile = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (uint32_t i = threadIdx.x; i < kMaxPasses * 256; i += kCompactBlock) (&s_hist[0][0])[i] = 0;
  const uint32_t base = tile * kTile + threadIdx.x;
  uint32_t flags = 0;
#pragma unroll
  for (int k = 0; k < kCompactRounds; ++k) {
    const uint32_t i = base + k * kCompactBlock;
    const bool live = i < st.n_faults && st.popc[i] != 0;
    flags |= uint32_t(live) << k;
    const uint64_t m = __ballot(live);
    if (lane == 0) s_off[k * kWaves + wv] = uint32_t(__popcll(m));
  }
  __syncthreads();
  if (threadIdx.x < kCompactRounds * kWaves) {
    const uint32_t v = s_off[threadIdx.x];
    s_off[threadIdx.x] = wave_inclusive_scan(v) - v;
  }
  __syncthreads();
  // live faults before this tile (the hash counted them per tile); the last
  // tile also records the total
  uint32_t tb = 0;
  {
    uint32_t part = 0;
    for (uint32_t t2 = threadIdx.x; t2 < tile; t2 += kCompactBlock) part += st.tile_cnt[t2];
    part = wave_sum(part);
    if (lane == 0) s_red[wv] = part;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kWaves; ++k) tb += s_red[k];
    if (threadIdx.x == 0 && tile + 1 == gridDim.x) st.hdr->n_live = tb + st.tile_cnt[tile];
  }
  const uint32_t P = st.n_pass;
  if (threadIdx.x == 0 || threadIdx.x == 1) {
    const uint64_t nzw = st.tile_nzw[tile];
    const uint64_t v = threadIdx.x == 0 ? (nzw & 0xFFFFFFFFull) : (nzw >> 32);
    if (v) atomicAdd(reinterpret_cast<unsigned long long*>(threadIdx.x == 0 ? &st.hdr->n_nz_words : &st.hdr->n_words),
                     (unsigned long long)v);
  }
#pragma unroll
  for (int k = 0; k < kCompactRounds; ++k) {
    const bool live = (flags >> k) & 1u;
    const uint64_t m = __ballot(live);
    if (live) {
      const uint32_t i = base + k * kCompactBlock;
      const uint32_t slot = tb + s_off[k * kWaves + wv] + lane_rank(m);
      const uint64_t key = st.key[1][i];
      st.key[0][slot] = key;
      st.val[0][slot] = i;
      for (uint32_t p = p0; p < P; ++p) atomicAdd(&s_hist[p][digit_of(key, p)], 1u);
    }
  }
  __syncthreads();
  // digit totals over all tiles
  for (uint32_t i = threadIdx.x; i < (P - p0) * 256; i += kCompactBlock) {
    const uint32_t p = p0 + i / 256, dg = i % 256;
    if (s_hist[p][dg]) atomicAdd(&st.digit_tot[p * 256 + dg], s_hist[p][dg]);
  }
}

// Lanes of the wave (among the valid ones) whose 8-bit digit equals this
// lane's: eight ballots, one per digit bit.
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool on = (d >> bit) & 1u;
    const uint64_t m = __ballot(on);
    peers &= on ? m : ~m;
  }
  return peers;
}

// One stable pass of 8-bit digits over the live keys (n = hdr->n_live). Tiles
// are taken in ticket order, so every tile a block waits for is already
// running. Wave v ranks tile items [v*256, (v+1)*256) in order, 64 at a time;
// each round's digit-peer masks serve both the wave's histogram and the
// placement. The tile publishes its digit counts first, ranks its items into
// LDS, and only then looks back for the counts of the tiles before it.
constexpr int kSortBlock = 1024;
constexpr int kSortWaves = kSortBlock / 64;
constexpr int kSortRounds = kTile / kSortBlock;

// With pout set, each pair's FaultRec (gathered from pin by its position)
// moves along with it, so that a later kernel reads it in pair order.
__global__ __launch_bounds__(kSortBlock) void k_onesweep(DevState st, uint32_t pass, const uint64_t* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
                                                         uint32_t* __restrict__ vout, const FaultRec* __restrict__ pin,
                                                         FaultRec* __restrict__ pout) {
  __shared__ uint64_t s_key[kTile];
  __shared__ uint32_t s_val[kTile];
  __shared__ uint32_t s_cnt[kSortWaves][256];
  __shared__ uint32_t s_start[256];
  __shared__ uint32_t s_gbase[256];
  __shared__ uint32_t s_wave[kSortWaves + 1];
  __shared__ uint32_t s_tile;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // an earlier pass gave up its look-back: its output is not a permutation
  // of valid pairs (a pass's own give-ups are not checked here, so that no
  // tile of this pass stops publishing)
  if (st.hdr->lookback_passes & ((1u << pass) - 1u)) return;
  const uint32_t n = st.hdr->n_live;
  const uint32_t ntiles = (n + kTile - 1) / kTile;
  if (tid == 0) s_tile = atomicAdd(&st.tile_ctr[pass], 1u);
  for (int k = tid; k < kSortWaves * 256; k += kSortBlock) (&s_cnt[0][0])[k] = 0;
  __syncthreads();
  const uint32_t tile = s_tile;
  if (tile >= ntiles) return;
  const uint32_t base = tile * kTile + wv * (kTile / kSortWaves);
  uint64_t k[kSortRounds];
  uint32_t v[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const uint32_t i = base + r * 64 + lane;
    k[r] = i < n ? kin[i] : 0;
    v[r] = i < n ? vin[i] : 0;
  }
  // global start of every digit value: exclusive prefix of the digit totals
  const uint32_t digit_base =
      block_exclusive_scan<kSortBlock>(tid < 256 ? st.digit_tot[pass * 256 + tid] : 0u, s_wave);
  const uint64_t lt = (1ull << lane) - 1;
  uint64_t peers[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool valid = base + r * 64 + lane < n;
    const uint32_t d = valid ? digit_of(k[r], pass) : 0u;
    peers[r] = digit_peers(d, valid);
    if (valid && (peers[r] & lt) == 0) s_cnt[wv][d] += uint32_t(__popcll(peers[r]));
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  uint32_t* lb = st.lookback + size_t(pass) * st.max_tiles * 256;
  uint32_t tot = 0;
  if (tid < 256) {
    // thread d: tile count of digit d; publish it
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) tot += s_cnt[w][tid];
    __hip_atomic_store(&lb[size_t(tile) * 256 + tid], (tile == 0 ? kLbPre : kLbAgg) | tot, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  {
    // local start of digit d, then of each wave's share of it
    const uint32_t start = block_exclusive_scan<kSortBlock>(tot, s_wave);
    if (tid < 256) {
      s_start[tid] = start;
      uint32_t run = start;
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) {
        const uint32_t c = s_cnt[w][tid];
        s_cnt[w][tid] = run;
        run += c;
      }
    }
  }
  __syncthreads();
  // rank in order and place into LDS sorted by digit
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const bool valid = base + r * 64 + lane < n;
    const uint32_t d = valid ? digit_of(k[r], pass) : 0u;
    const uint32_t rank = uint32_t(__popcll(peers[r] & lt));
    uint32_t li = 0;
    if (valid) li = s_cnt[wv][d] + rank;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) s_cnt[wv][d] += uint32_t(__popcll(peers[r]));
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      s_key[li] = k[r];
      s_val[li] = v[r];
    }
  }
  if (tid < 256) {
    // thread d: counts of digit d in the tiles before this one, kLookWin at a
    // time, until a tile that already published its inclusive prefix. Every
    // tile runs at once, so the inclusive prefixes spread from tile 0 while
    // all tiles walk back. Each round's loads are issued together and waited
    // for together: a window of 8 balances their cost against the number of
    // (cross-XCD latency) rounds.
    const uint32_t d = tid;
    uint32_t excl = 0;
    if (tile > 0) {
      int j = int(tile) - 1;
      uint32_t spins = 0;
      bool done = false;
      while (!done) {
        if (spins >= st.spin_limit) {
          // gave up: the prefix is partial, so this pass misplaces pairs
          // (every placement stays below the true one, so in bounds); later
          // passes and grouping kernels then do nothing and the fetch fails
          raise_flag(st.hdr, FLAG_LOOKBACK);
          atomicOr(&st.hdr->lookback_passes, 1u << pass);
          break;
        }
        uint32_t x[kLookWin];
#pragma unroll
        for (int q = 0; q < kLookWin; ++q)
          x[q] = (j - q >= 0) ? __hip_atomic_load(&lb[size_t(j - q) * 256 + d], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)
                              : kLbPre;
        bool stalled = false;
#pragma unroll
        for (int q = 0; q < kLookWin; ++q) {
          if (done || stalled) continue;
          if ((x[q] & ~kLbMask) == 0) {
            stalled = true;
            continue;
          }
          if (j >= 0) excl += x[q] & kLbMask;
          if (x[q] & kLbPre) done = true;
          else --j;
        }
        if (stalled && !done) {
          ++spins;
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __hip_atomic_store(&lb[size_t(tile) * 256 + d], kLbPre | (excl + tot), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    s_gbase[d] = digit_base + excl;
  }
  __syncthreads();
  // write runs of equal digits to consecutive global positions
  const uint32_t cnt = min(uint32_t(kTile), n - tile * kTile);
  if (pout) {
    // the records are read first (independent loads), then written
    double pp[kSortRounds];
    uint64_t pc[kSortRounds];
    uint32_t pd[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
      const uint32_t li = tid + r * kSortBlock;
      const bool ok = li < cnt;
      const uint64_t key = ok ? s_key[li] : 0ull;
      const uint32_t d = digit_of(key, pass);
      const uint32_t dst = ok ? s_gbase[d] + (li - s_start[d]) : 0u;
      const uint32_t v = ok ? s_val[li] : 0u;
      if (ok) {
        kout[dst] = key;
        vout[dst] = v;
      }
      pp[r] = ok ? pin[v].p : 0.0;
      pc[r] = ok ? pin[v].chk : 0ull;
      pd[r] = dst;
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r)
      if (tid + r * kSortBlock < cnt) {
        pout[pd[r]].p = pp[r];
        pout[pd[r]].chk = pc[r];
      }
    return;
  }
  for (uint32_t li = tid; li < cnt; li += kSortBlock) {
    const uint64_t key = s_key[li];
    const uint32_t d = digit_of(key, pass);
    const uint32_t dst = s_gbase[d] + (li - s_start[d]);
    kout[dst] = key;
    vout[dst] = s_val[li];
  }
}

// Class heads in the sorted key array (n = hdr->n_live): counts per tile.
__global__ __launch_bounds__(kBlock) void k_heads_count(const uint64_t* __restrict__ keys, const DevHeader* hdr,
                                                        uint32_t* __restrict__ tile_sum) {
  __shared__ uint32_t s_wave[kBlock / 64 + 1];
  const uint32_t n = hdr->n_live;
  const uint32_t base = blockIdx.x * kTile;
  uint32_t s = 0;
  for (int r = 0; r < kPerThread; ++r) {
    const uint32_t i = base + r * kBlock + threadIdx.x;
    if (i < n) s += (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
  }
  block_exclusive_scan<kBlock>(s, s_wave);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = s_wave[kBlock / 64];
}

// segstart[class] = first sorted index of the class.
__global__ __launch_bounds__(kBlock) void k_heads_apply(const uint64_t* __restrict__ keys, const DevHeader* hdr,
                                                        const uint32_t* __restrict__ tile_off,
                                                        uint32_t* __restrict__ segstart) {
  __shared__ uint32_t s_wave[kBlock / 64 + 1];
  const uint32_t n = hdr->n_live;
  const uint32_t i0 = blockIdx.x * kTile + threadIdx.x * kPerThread;
  uint32_t flags = 0, s = 0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const uint32_t i = i0 + k;
    const bool h = i < n && (i == 0 || keys[i] != keys[i - 1]);
    flags |= uint32_t(h) << k;
    s += h;
  }
  uint32_t run = block_exclusive_scan<kBlock>(s, s_wave) + tile_off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kPerThread; ++k)
    if ((flags >> k) & 1u) segstart[run++] = i0 + k;
}

// One thread per class of at most kBigSegment faults: merge probabilities in
// sorted (fault position) order and check that the check hashes agree.
__global__ __launch_bounds__(kBlock) void k_reduce(DevState st, const uint32_t* __restrict__ vals) {
  if (grouping_aborted(st.hdr)) return;
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t S = st.hdr->n_seg;
  if (s >= S) return;
  const uint32_t n = st.hdr->n_live;
  const uint32_t i0 = st.segstart[s];
  const uint32_t i1 = (s + 1 < S) ? st.segstart[s + 1] : n;
  if (i1 - i0 > kBigSegment) {  // merged by a whole block in k_reduce_big
    st.big[atomicAdd(&st.hdr->n_big, 1u)] = s;
    return;
  }
  const uint32_t rep = vals[i0];
  const FaultRec r0 = st.frp[rep];
  bool bad = false;
  double q = r0.p;
  for (uint32_t i = i0 + 1; i < i1; ++i) {
    const FaultRec r = st.frp[vals[i]];
    bad |= r.chk != r0.chk;
    q = fma(r.p, 1.0 - 2.0 * q, q);  // Eq. 3: q(1-p) + p(1-q)
  }
  if (bad) raise_flag(st.hdr, FLAG_COLLISION);
  put_rep(st, rep, q, i0, i1 - i0);
}

// One block per class of more than kBigSegment faults (the list k_reduce
// built; its order does not matter): strided partial merges per thread, then
// a fixed-shape tree, so the result is the same on every run.
__global__ __launch_bounds__(kBlock) void k_reduce_big(DevState st, const uint32_t* __restrict__ vals) {
  __shared__ double s_q[kBlock];
  __shared__ int s_bad;
  if (grouping_aborted(st.hdr)) return;
  const uint32_t S = st.hdr->n_seg;
  const uint32_t n = st.hdr->n_live;
  const uint32_t nb = st.hdr->n_big;
  for (uint32_t g = blockIdx.x; g < nb; g += gridDim.x) {
    const uint32_t s = st.big[g];
    const uint32_t i0 = st.segstart[s];
    const uint32_t i1 = (s + 1 < S) ? st.segstart[s + 1] : n;
    if (threadIdx.x == 0) s_bad = 0;
    const uint32_t rep = vals[i0];
    const uint64_t c0 = st.frp[rep].chk;
    bool bad = false;
    double q = 0.0;
    for (uint32_t i = i0 + threadIdx.x; i < i1; i += kBlock) {
      const FaultRec r = st.frp[vals[i]];
      bad |= r.chk != c0;
      q = fma(r.p, 1.0 - 2.0 * q, q);
    }
    s_q[threadIdx.x] = q;
    __syncthreads();
    if (bad) s_bad = 1;
    for (int h = kBlock / 2; h > 0; h >>= 1) {
      if (threadIdx.x < h) {
        const double a = s_q[threadIdx.x], c = s_q[threadIdx.x + h];
        s_q[threadIdx.x] = fma(c, 1.0 - 2.0 * a, a);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (s_bad) raise_flag(st.hdr, FLAG_COLLISION);
      put_rep(st, rep, s_q[0], i0, i1 - i0);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ buckets

constexpr int kBucketBlock = 1024;
constexpr uint32_t kBucketSortBits = 24;  // key bits a bucket sorts in LDS; longer runs of equal bits are rare

// Grouping inside one bucket: the live faults whose key has top digit d
// (k16: top two digits), which the stable partition passes left in position
// order at [bkt_start, bkt_start + m). Values (key bits below the top digit << 16 |
// index in the bucket) are sorted in LDS by stable 8-bit LSD passes over the
// key bits, so each class is a run of equal key bits whose members are in
// position order. Per class: Eq. 3 merge in that order (one thread, or the
// whole block for classes of more than kBigSegment faults), the check-hash
// comparison, the representative (first member), its bit count and the
// class's bit offset within the bucket. Class c of the bucket is stored at
// slot bkt_start + c; its members (positions) go to mem in class order. The
// bucket's class and bit counts go to b_cls[d] and b_bits[d]. One work-group
// of kBlk threads per bucket of at most kCap faults.
template <int kBlk, int kCap, bool k16>
__global__ __launch_bounds__(kBlk) void k_bucket(DevState st, const uint64_t* __restrict__ keys,
                                                 const uint32_t* __restrict__ vals, uint32_t* __restrict__ mem) {
  constexpr int kWaves = kBlk / 64;
  constexpr int kPer = kCap / kBlk;  // sorted values per thread
  static_assert(kBlk % 256 == 0 && kCap % kBlk == 0 && kPer <= 32, "bucket shape");
  extern __shared__ __align__(16) uint64_t s_buf[];  // two buffers of kCap values
  __shared__ uint32_t s_cnt[kWaves][256];
  __shared__ uint32_t s_wave[kWaves + 1];
  __shared__ uint32_t s_big[2 * (kCap / (kBigSegment + 1) + 1)];  // (representative, first sorted index)
  __shared__ uint64_t s_hb[kCap / 64];                            // class heads, one bit per value
  __shared__ uint64_t s_rb[kCap / 64];                            // starts of runs of equal sorted bits
  __shared__ uint64_t s_mb[kCap / 64];                            // run members whose key differs
  __shared__ int s_bad_bucket;
  __shared__ uint32_t s_nbig;
  __shared__ uint32_t s_big_end;
  __shared__ uint32_t s_start;
  __shared__ double s_q[kBlk];
  __shared__ int s_bad;
  if (grouping_aborted(st.hdr)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const uint32_t d = blockIdx.x;
  const uint32_t msd = st.n_pass - 1;
  const uint32_t* tot = st.digit_tot + msd * 256;
  {
    if (k16) {
      if (tid == 0) s_start = st.b16_lo[d];
    } else {
      const uint32_t v = tid < int(kBuckets) ? tot[tid] : 0u;
      const uint32_t ex = block_exclusive_scan<kBlk>(v, s_wave);
      if (uint32_t(tid) == d) s_start = ex;
    }
    if (tid == 0) {
      s_nbig = 0;
      s_bad = 0;
      s_bad_bucket = 0;
    }
    for (uint32_t k = tid; k < kCap / 64; k += kBlk) s_hb[k] = 0;
  }
  __syncthreads();
  const uint32_t start = s_start;
  const uint32_t m = k16 ? st.b16_hi[d] - start : tot[d];
  if (m == 0 || m > kCap) {
    if (tid == 0 && m) raise_flag(st.hdr, FLAG_BUCKET);
    return;
  }
  const uint32_t top = k16 ? 2u : 1u;  // digits that chose the bucket
  const uint32_t lbits = 8 * (msd + 1 - top);  // key bits below them (at most 48)
  const uint64_t lmask = (1ull << lbits) - 1;
  uint64_t* a = s_buf;
  uint64_t* b = s_buf + kCap;
  for (uint32_t i = tid; i < m; i += kBlk) a[i] = ((keys[start + i] & lmask) << 16) | i;
  // wave wv owns the contiguous values [wv*chunk, (wv+1)*chunk), 64 per round
  const uint32_t rounds = (m + kBlk - 1) / kBlk;
  const uint32_t chunk = rounds * 64;
  const uint64_t lt = (1ull << lane) - 1;
  // stable LSD passes over the lowest kBucketSortBits key bits (fewer when
  // the key has fewer); equal keys then sit in runs of equal sorted bits
  const uint32_t npass = min(msd + 1 - top, kBucketSortBits / 8);
  for (uint32_t pass = 0; pass < npass; ++pass) {
    const uint32_t sh = 16 + 8 * pass;
    for (int k = tid; k < kWaves * 256; k += kBlk) (&s_cnt[0][0])[k] = 0;
    __syncthreads();
    uint64_t val[kPer], pe[kPer];
#pragma unroll
    for (int r = 0; r < int(kPer); ++r) {
      if (uint32_t(r) < rounds) {
        const uint32_t i = wv * chunk + r * 64 + lane;
        const bool valid = i < m;
        val[r] = valid ? a[i] : 0ull;
        const uint32_t dg = uint32_t(val[r] >> sh) & 255u;
        pe[r] = digit_peers(dg, valid);
        if (valid && (pe[r] & lt) == 0) atomicAdd(&s_cnt[wv][dg], uint32_t(__popcll(pe[r])));
      }
    }
    __syncthreads();
    {
      // exclusive scan in (digit, wave) order: thread t owns digit t/T and
      // waves 4(t%T)..4(t%T)+3, with T = kBlk/256 threads per digit
      constexpr int kTpd = kBlk / 256;
      const uint32_t dg = tid / kTpd, w0 = (tid % kTpd) * 4;
      uint32_t c[4], sum = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        c[j] = s_cnt[w0 + j][dg];
        sum += c[j];
      }
      uint32_t total;
      uint32_t run = block_scan_1sync<kBlk>(sum, s_wave, total);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        s_cnt[w0 + j][dg] = run;
        run += c[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < int(kPer); ++r) {
      if (uint32_t(r) < rounds) {
        const uint32_t i = wv * chunk + r * 64 + lane;
        const bool valid = i < m;
        const uint32_t dg = uint32_t(val[r] >> sh) & 255u;
        const uint32_t rank = uint32_t(__popcll(pe[r] & lt));
        const uint32_t base = valid ? s_cnt[wv][dg] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) s_cnt[wv][dg] = base + uint32_t(__popcll(pe[r]));
        __builtin_amdgcn_wave_barrier();
        if (valid) b[base + rank] = val[r];
      }
    }
    __syncthreads();
    uint64_t* t = a;
    a = b;
    b = t;
  }
  if (8 * npass < lbits) {
    // Runs of equal sorted bits that hold more than one key (rare: the keys
    // are hashes) are sorted by the whole value (key bits, then index) by
    // one thread; a longer such run hands the bucket to the full sort.
    // run starts and mixed elements (key bits differ from the previous
    // value's inside a run) as bitmasks, read-only while runs are sorted
    const uint64_t smask = (1ull << (16 + 8 * npass)) - 1;
    for (uint32_t k = tid; k < kCap / 64; k += kBlk) {
      s_rb[k] = 0;
      s_mb[k] = 0;
    }
    __syncthreads();
    const uint32_t j0 = tid * rounds;
    uint32_t mixed = 0;
    for (uint32_t k = 0; k < rounds; ++k) {
      const uint32_t j = j0 + k;
      if (j >= m) break;
      const uint64_t v = a[j], u = j ? a[j - 1] : 0ull;
      const bool run_start = j == 0 || ((v ^ u) & smask & ~0xFFFFull) != 0;
      if (run_start) {
        atomicOr(&s_rb[j >> 6], 1ull << (j & 63));
      } else if ((v >> 16) != (u >> 16)) {
        mixed |= 1u << k;
        atomicOr(&s_mb[j >> 6], 1ull << (j & 63));
      }
    }
    __syncthreads();
    auto run_start_at = [&](uint32_t j) -> bool { return (s_rb[j >> 6] >> (j & 63)) & 1ull; };
    auto mixed_at = [&](uint32_t j) -> bool { return (s_mb[j >> 6] >> (j & 63)) & 1ull; };
    for (uint32_t k = 0; k < rounds; ++k) {
      if (!((mixed >> k) & 1u)) continue;
      const uint32_t j = j0 + k;
      uint32_t rs = j;
      while (!run_start_at(rs)) --rs;
      // the first mixed element of the run sorts it
      bool first = true;
      for (uint32_t x = rs + 1; x < j && first; ++x) first = !mixed_at(x);
      if (!first) continue;
      uint32_t re = j + 1;
      while (re < m && !run_start_at(re)) ++re;
      if (re - rs > 64) {
        s_bad_bucket = 1;
        continue;
      }
      for (uint32_t x = rs + 1; x < re; ++x) {
        const uint64_t v = a[x];
        uint32_t y = x;
        while (y > rs && a[y - 1] > v) {
          a[y] = a[y - 1];
          --y;
        }
        a[y] = v;
      }
    }
    __syncthreads();
    if (s_bad_bucket) {
      if (tid == 0) raise_flag(st.hdr, FLAG_BUCKET);
      return;
    }
  }
  // Each thread owns the sorted values [j0, j0 + per): their head flags
  // (first of a run of equal key bits) go to an LDS bitmask, and their
  // probability and check hash are gathered at once (independent loads)
  // into the two sort buffers, now free: p over a, check hash over b.
  const uint32_t per = rounds;  // at most kPer
  const uint32_t j0 = tid * per;
  uint32_t hmask = 0;
  uint32_t pos[kPer];
  uint32_t idx[kPer];  // index within the bucket (the pair's slot)
#pragma unroll
  for (int k = 0; k < int(kPer); ++k) {
    const uint32_t j = j0 + k;
    pos[k] = 0;
    idx[k] = 0;
    if (uint32_t(k) < per && j < m) {
      const uint64_t v = a[j];
      if (j == 0 || (v >> 16) != (a[j - 1] >> 16)) hmask |= 1u << k;
      idx[k] = uint32_t(v & 0xFFFFu);
      pos[k] = vals[start + idx[k]];
    }
  }
  if (hmask) {
    const uint32_t wd = j0 >> 6, sh = j0 & 63;
    atomicOr(&s_hb[wd], uint64_t(hmask) << sh);
    if (sh + per > 64) atomicOr(&s_hb[wd + 1], uint64_t(hmask) >> (64 - sh));
  }
  // each pair's record was moved into the bucket's range by the partition
  // pass: read within the bucket instead of gathered across all faults
  FaultRec rec[kPer];
#pragma unroll
  for (int k = 0; k < int(kPer); ++k)
    if (uint32_t(k) < per && j0 + k < m) {
      rec[k] = st.crp[start + idx[k]];
      mem[start + j0 + k] = pos[k];  // the class members, kept for refreshes and the adjoint
    }
  __syncthreads();  // every a[j] has been read
  double* sp = reinterpret_cast<double*>(a);
  uint64_t* sc = b;
#pragma unroll
  for (int k = 0; k < int(kPer); ++k)
    if (uint32_t(k) < per && j0 + k < m) {
      sp[j0 + k] = rec[k].p;
      sc[j0 + k] = rec[k].chk;
    }
  __syncthreads();
  auto head_at = [&](uint32_t j) -> bool { return (s_hb[j >> 6] >> (j & 63)) & 1ull; };
  // classes whose head this thread owns, in order: Eq. 3 over the members
  // in position order (runs longer than kBigSegment go to the block below);
  // the head is the class's lowest position, its representative
#pragma unroll
  for (int k = 0; k < int(kPer); ++k) {
    if (!((hmask >> k) & 1u)) continue;
    const uint32_t j = j0 + k;
    const uint32_t rep = pos[k];
    double q = sp[j];
    const uint64_t c0 = sc[j];
    bool bad = false;
    uint32_t i = j + 1;
    for (; i < m && i - j <= kBigSegment && !head_at(i); ++i) {
      bad |= sc[i] != c0;
      q = fma(sp[i], 1.0 - 2.0 * q, q);  // Eq. 3: q(1-p) + p(1-q)
    }
    if (i < m && i - j > kBigSegment && !head_at(i)) {
      const uint32_t g = atomicAdd(&s_nbig, 1u);
      s_big[2 * g] = rep;
      s_big[2 * g + 1] = j;
    } else {
      put_rep(st, rep, q, start + j, i - j);
      if (bad) s_bad = 1;
    }
  }
  __syncthreads();
  // large classes: strided partial merges over the whole run, then a
  // fixed-shape tree
  const uint32_t nbig = s_nbig;
  for (uint32_t g = 0; g < nbig; ++g) {
    const uint32_t rep = s_big[2 * g], j = s_big[2 * g + 1];
    if (tid == 0) {
      uint32_t e = j + 1;
      while (e < m && !head_at(e)) ++e;
      s_big_end = e;
    }
    __syncthreads();
    const uint32_t e = s_big_end;
    const uint64_t c0 = sc[j];
    bool bad = false;
    double q = 0.0;
    for (uint32_t i = j + tid; i < e; i += kBlk) {
      bad |= sc[i] != c0;
      q = fma(sp[i], 1.0 - 2.0 * q, q);
    }
    if (bad) s_bad = 1;
    s_q[tid] = q;
    __syncthreads();
    for (int h = kBlk / 2; h > 0; h >>= 1) {
      if (tid < h) {
        const double x = s_q[tid], y = s_q[tid + h];
        s_q[tid] = fma(y, 1.0 - 2.0 * x, x);
      }
      __syncthreads();
    }
    if (tid == 0) put_rep(st, rep, s_q[0], start + j, e - j);
    __syncthreads();
  }
  if (tid == 0 && s_bad) raise_flag(st.hdr, FLAG_COLLISION);
}

// 16-bit bucket of a key: its top two digits (the two partition passes).
__device__ __forceinline__ uint32_t bucket16_of(uint64_t k, uint32_t msd) {
  return uint32_t(k >> (8 * (msd - 1))) & 0xFFFFu;
}

// Sorted index range [b16_lo[b], b16_hi[b]) of every non-empty 16-bit bucket
// (empty buckets keep the cleared 0, 0): the first and last key of each run.
__global__ __launch_bounds__(kBlock) void k_bucket_bounds(DevState st, const uint64_t* __restrict__ keys) {
  if (grouping_aborted(st.hdr)) return;
  const uint32_t n = st.hdr->n_live;
  const uint32_t msd = st.n_pass - 1;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const uint32_t b = bucket16_of(keys[i], msd);
    if (i == 0 || bucket16_of(keys[i - 1], msd) != b) st.b16_lo[b] = i;
    if (i + 1 == n || bucket16_of(keys[i + 1], msd) != b) st.b16_hi[b] = i + 1;
  }
}

// ------------------------------------------------------------------ output

// Hyperedges in representative-position order. Output tiles of kTile
// positions; thread t of a tile's block owns positions [16t, 16t + 16), a
// quarter of one representative-bitmap word.
constexpr int kOutPer = kTile / kBlock;
static_assert(kOutPer == 16, "a thread owns 16 positions of a 64-bit bitmap word");

__device__ __forceinline__ uint32_t rep_bits16(const DevState& st, uint32_t p0) {
  return p0 < st.n_faults ? uint32_t(st.rep_bm[p0 >> 6] >> (p0 & 63)) & 0xFFFFu : 0u;
}

// The signature weights of a thread's 16 positions, loaded at once (64
// contiguous bytes; positions past the last fault read as zero).
__device__ __forceinline__ void weights16(const DevState& st, uint32_t p0, uint32_t (&pc)[kOutPer]) {
  if (p0 + uint32_t(kOutPer) <= st.n_faults) {
    const uint4* src = reinterpret_cast<const uint4*>(st.popc + p0);
#pragma unroll
    for (int j = 0; j < kOutPer / 4; ++j) {
      const uint4 x = src[j];
      pc[4 * j] = x.x;
      pc[4 * j + 1] = x.y;
      pc[4 * j + 2] = x.z;
      pc[4 * j + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kOutPer; ++k) pc[k] = p0 + uint32_t(k) < st.n_faults ? st.popc[p0 + k] : 0u;
  }
}

// Packed count of this thread's positions: representatives << kRepShift |
// their signature bits.
__device__ __forceinline__ uint64_t rep_count16(uint32_t m, const uint32_t (&pc)[kOutPer]) {
  uint64_t v = uint64_t(__popc(m)) << kRepShift;
#pragma unroll
  for (int k = 0; k < kOutPer; ++k) v += ((m >> k) & 1u) ? pc[k] : 0u;
  return v;
}

// Exclusive block scan of 64-bit values (kBlock threads); s needs kBlock / 64
// + 1 entries and ends holding the block total at [kBlock / 64].
__device__ __forceinline__ uint64_t block_exclusive_scan64(uint64_t v, unsigned long long* s) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint64_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t u = __shfl_up(inc, d, 64);
    if (lane >= d) inc += u;
  }
  if (lane == 63) s[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int k = 0; k < kBlock / 64; ++k) {
      const unsigned long long x = s[k];
      s[k] = run;
      run += x;
    }
    s[kBlock / 64] = run;
  }
  __syncthreads();
  return s[wv] + inc - v;
}

// Look-back words of the output pass (64-bit: status in the top two bits).
constexpr uint64_t kOutAgg = 1ull << 62;   // the tile's own count is published
constexpr uint64_t kOutPre = 2ull << 62;   // the inclusive prefix up to the tile is published
constexpr uint64_t kOutMask = kOutAgg - 1;
constexpr uint32_t kOutLookbackBit = 1u << 31;  // lookback_passes bit of the output pass

// Numbering of the hyperedges over tiles of kTile positions (tiles taken in
// dispatch order from a ticket). A tile counts its representatives and their
// signature bits, publishes both counts and looks back at the tiles before it
// for their prefixes (two chains, hyperedges and bits, each on half of wave
// 0, 32 predecessors per round), so it knows its first hyperedge and
// first bit. Each thread then lists its representatives (their positions in
// hyperedge order and their first bits) and gives every circuit whose first
// fault position falls in its positions that circuit's first hyperedge; the
// last tile writes the totals.
__global__ __launch_bounds__(kBlock) void k_rep_list(DevState st, uint32_t ntiles) {
  __shared__ unsigned long long s[kBlock / 64 + 1];
  __shared__ uint32_t s_bfb[kBranchLds];  // first fault of each circuit of the batch
  __shared__ uint64_t s_excl[2];
  __shared__ uint32_t s_tile;
  if (grouping_aborted(st.hdr)) return;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid == 0) s_tile = atomicAdd(st.out_ctr, 1u);
  const bool bfb_lds = st.n_branch <= uint32_t(kBranchLds);
  if (bfb_lds)
    for (uint32_t k = tid; k < st.n_branch; k += blockDim.x) s_bfb[k] = st.branch[k].fb;
  __syncthreads();
  const uint32_t tile = s_tile;
  if (tile >= ntiles) return;
  auto FB = [&](uint32_t k) -> uint32_t { return bfb_lds ? s_bfb[k] : st.branch[k].fb; };
  const uint32_t p0 = tile * kTile + tid * kOutPer;
  const uint32_t m = rep_bits16(st, p0);
  uint32_t pc[kOutPer];
  weights16(st, p0, pc);
  const uint64_t local = block_exclusive_scan64(rep_count16(m, pc), s);
  const uint64_t agg = s[kBlock / 64];
  const uint32_t nrep = uint32_t(agg >> kRepShift);
  const uint64_t nbits = agg & ((1ull << kRepShift) - 1);
  if (tid < 64) {
    // lanes 0-31: the hyperedge chain; lanes 32-63: the bit chain
    const int chain = lane >> 5, q = lane & 31;
    uint64_t* lb = st.out_lb + size_t(chain) * st.max_tiles;
    const uint64_t val = chain == 0 ? uint64_t(nrep) : nbits;
    if (q == 0)
      __hip_atomic_store(&lb[tile], (tile == 0 ? kOutPre : kOutAgg) | val, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    bool done = tile == 0;
    int jt = int(tile) - 1;
    uint32_t spins = 0;
    const uint64_t half = chain == 0 ? 0xFFFFFFFFull : 0xFFFFFFFF00000000ull;
    // the whole wave runs the loop until both chains are done (the ballots
    // and the give-up are wave-wide)
    while (__ballot(!done) != 0) {
      if (__ballot(spins >= st.spin_limit) != 0) {
        // gave up: the prefix is partial (every number it gives stays below
        // the true one, so in bounds) and the fetch redoes the compile
        if (lane == 0) {
          raise_flag(st.hdr, FLAG_LOOKBACK);
          atomicOr(&st.hdr->lookback_passes, kOutLookbackBit);
        }
        break;
      }
      // tiles jt, jt-1, ... (lane q: tile jt - q); before tile 0 an inclusive
      // prefix of zero, so a walk always ends at tile 0 at the latest
      uint64_t x = kOutPre;
      if (!done && jt - q >= 0) x = __hip_atomic_load(&lb[jt - q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // (__ballot takes an int: test the status bits as booleans, never the 64-bit word)
      const uint64_t pre = __ballot((x & kOutPre) != 0ull) & half;
      const uint64_t stall = __ballot((x & ~kOutMask) == 0ull) & half;
      // the nearest published prefix, and the nearest tile not yet published
      const int fp = pre ? int(__builtin_ctzll(pre >> (32 * chain))) : 32;
      const int fs = stall ? int(__builtin_ctzll(stall >> (32 * chain))) : 32;
      const int take = done ? 0 : (fp < fs ? fp + 1 : fs);  // predecessors summed this round
      uint64_t add = (q < take) ? (x & kOutMask) : 0ull;
#pragma unroll
      for (int d = 1; d < 32; d <<= 1) add += __shfl_xor(add, d, 32);
      if (!done) {
        excl += add;
        if (fp < fs) done = true;
        else jt -= take;
        if (fs < 32 && fp > fs) {
          ++spins;
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    if (q == 0) {
      if (tile > 0)
        __hip_atomic_store(&lb[tile], kOutPre | (excl + val), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_excl[chain] = excl;
    }
  }
  __syncthreads();
  const uint32_t e0 = uint32_t(s_excl[0]);
  const uint64_t o0 = s_excl[1];
  uint32_t e = e0 + uint32_t(local >> kRepShift);
  uint64_t o = o0 + (local & ((1ull << kRepShift) - 1));
  if (p0 < st.n_faults) {
    // circuits whose first position falls in this thread's positions
    uint32_t lo = 0, hi = st.n_branch;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) / 2;
      if (FB(mid) < p0) lo = mid + 1;
      else hi = mid;
    }
    for (uint32_t k = lo; k < st.n_branch; ++k) {
      const uint32_t fb = FB(k);
      if (fb >= p0 + uint32_t(kOutPer) || fb >= st.n_faults) break;
      st.circ_eoff[k] = e + uint32_t(__popc(m & ((1u << (fb - p0)) - 1u)));
    }
  }
#pragma unroll
  for (int k = 0; k < kOutPer; ++k)
    if ((m >> k) & 1u) {
      st.rep_pos[e] = p0 + uint32_t(k);
      st.edge_off32[e] = uint32_t(o);
      o += pc[k];
      ++e;
    }
  if (tile + 1 == ntiles && tid == 0) {
    const uint64_t U = e0 + uint64_t(nrep), NB = o0 + nbits;
    st.hdr->n_seg = uint32_t(U);
    st.hdr->n_edges = uint32_t(U);
    st.hdr->n_bits = NB;
    st.edge_off32[U] = uint32_t(NB);
    if (NB > st.bits_cap) raise_flag(st.hdr, FLAG_OVERFLOW);
    // circuits that start at or past the last fault position begin at the end
    for (uint32_t k = 0; k <= st.n_branch; ++k)
      if (k == st.n_branch || FB(k) >= st.n_faults) st.circ_eoff[k] = uint32_t(U);
  }
}

// Hyperedge e = the class of the e-th representative in position order (one
// thread per hyperedge, consecutive threads on increasing positions): its
// probability, members and bits in external numbering (detector d -> d,
// observable k -> D + k). The representative's boundary row, weight and
// non-zero-word mask come from its edge record; its non-zero signature words
// from the column slabs that cover that boundary.
__global__ __launch_bounds__(kBlock) void k_edge_write(DevState st) {
  __shared__ uint32_t s_bfb[kBranchLds];  // first fault of each circuit of the batch
  if (grouping_aborted(st.hdr)) return;
  const bool bfb_lds = st.n_branch <= uint32_t(kBranchLds);
  if (bfb_lds)
    for (uint32_t k = threadIdx.x; k < st.n_branch; k += blockDim.x) s_bfb[k] = st.branch[k].fb;
  __syncthreads();
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= st.hdr->n_edges) return;
  const uint32_t pos = st.rep_pos[e];
  const RepRec rr = st.rrec[pos];
  const EdgeRec er = st.erec[pos];
  const uint64_t o0 = st.edge_off32[e];
  st.edge_q[e] = rr.q;
  st.e_first[e] = rr.first;
  st.e_cnt[e] = rr.cnt;
  if (o0 + er.popc > st.bits_cap) return;
  // the representative's circuit (last one whose first fault is <= pos)
  uint32_t bi = 0;
  {
    uint32_t lo = 0, hi = st.n_branch;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if ((bfb_lds ? s_bfb[mid] : st.branch[mid].fb) <= pos) lo = mid;
      else hi = mid;
    }
    bi = lo;
  }
  const BranchDesc& br = st.branch[bi];
  const uint32_t b = er.bnd;  // the representative's boundary row
  const uint32_t n = st.ncov[b];
  const uint32_t* cl = st.cov + size_t(b) * st.w_max;
  uint64_t o = o0;
  const uint32_t obs0 = br.wd * 64, wb = br.wb, n_det = br.n_det;
  auto emit = [&](uint32_t w) {
    uint64_t v = st.slab[st.col_base[w] + pos];
    while (v) {
      const uint32_t bit = (w - wb) * 64 + uint32_t(__builtin_ctzll(v));
      st.edge_bits[o++] = bit < obs0 ? bit : n_det + (bit - obs0);
      v &= v - 1;
    }
  };
  if (n <= 64) {
    // the mask names the covered columns that hold non-zero words
    uint64_t mask = er.nzm;
    while (mask) {
      const uint32_t k = uint32_t(__builtin_ctzll(mask));
      mask &= mask - 1;
      emit(cl[k]);
    }
  } else {
    // more covered columns than mask bits: the bitmaps say which words are stored
    const uint32_t ib = pos - st.bnd_fault_off[b];  // b is the batch's boundary row
    const uint64_t* bm = st.bm + st.bnd_bm_off[b] + (ib >> 6);
    for (uint32_t k = 0; k < n; ++k)
      if ((bm[st.col_bm_base[cl[k]]] >> (ib & 63)) & 1ull) emit(cl[k]);
  }
}

// ------------------------------------------------------------------ rates

// Rate of lowered channel c: from the driver's table, or (rates != null) from
// a device array in program order.
__device__ __forceinline__ double channel_rate(const DevState& st, const double* rates, uint32_t c) {
  return rates ? rates[st.chan_src[c]] : st.chan_rate[c];
}

// Per-fault probabilities from the channel rates.
__global__ __launch_bounds__(kBlock) void k_fault_p(DevState st, const double* __restrict__ rates) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= st.n_chan) return;
  const double p = fault_probability(st.chan_kind[c], channel_rate(st, rates, c));
  for (uint32_t f = st.chan_foff[c]; f < st.chan_foff[c + 1]; ++f) st.frp[f].p = p;
}

// Eq. 3 again over each hyperedge's cached members (position order), with the
// compile's shape: up to kBigSegment + 1 members one thread folds them in
// order; larger classes are listed for k_remerge_big. Thread j serves
// hyperedge j and
// writes out[j].
__global__ __launch_bounds__(kBlock) void k_remerge(DevState st, const uint32_t* __restrict__ ord, uint32_t n_edges,
                                                    double* __restrict__ out) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_edges) return;
  const uint32_t e = j;
  const uint32_t i0 = st.e_first[e], cnt = st.e_cnt[e];
  if (cnt > kBigSegment + 1) {
    st.big[atomicAdd(&st.hdr->n_big, 1u)] = j;
    return;
  }
  double q = st.frp[ord[i0]].p;
  for (uint32_t i = 1; i < cnt; ++i) q = fma(st.frp[ord[i0 + i]].p, 1.0 - 2.0 * q, q);
  out[j] = q;
}

// One block of kBucketBlock threads per listed hyperedge: strided partial
// merges, then the fixed tree the bucket grouping uses.
__global__ __launch_bounds__(kBucketBlock) void k_remerge_big(DevState st, const uint32_t* __restrict__ ord,
                                                             double* __restrict__ out) {
  __shared__ double s_q[kBucketBlock];
  const int tid = threadIdx.x;
  const uint32_t nb = st.hdr->n_big;
  for (uint32_t g = blockIdx.x; g < nb; g += gridDim.x) {
    const uint32_t j = st.big[g];
    const uint32_t e = j;
    const uint32_t i0 = st.e_first[e], cnt = st.e_cnt[e];
    double q = 0.0;
    for (uint32_t i = tid; i < cnt; i += kBucketBlock) q = fma(st.frp[ord[i0 + i]].p, 1.0 - 2.0 * q, q);
    s_q[tid] = q;
    __syncthreads();
    for (int h = kBucketBlock / 2; h > 0; h >>= 1) {
      if (tid < h) {
        const double x = s_q[tid], y = s_q[tid + h];
        s_q[tid] = fma(y, 1.0 - 2.0 * x, x);
      }
      __syncthreads();
    }
    if (tid == 0) out[j] = s_q[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_clear_big(DevState st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st.hdr->n_big = 0;
}

// Adjoint, per hyperedge: q = 1/2 (1 - prod_j (1 - 2 p_j)) over the members,
// so dq/dp_i = prod_{j != i} (1 - 2 p_j): the product of the members other
// than those with p = 1/2, divided by (1 - 2 p_i); with one member at p = 1/2
// only that member's derivative is non-zero, with two or more none is.
// Thread j: dL/dq = gq[j] of hyperedge j.
__global__ __launch_bounds__(kBlock) void k_adj_edges(DevState st, const uint32_t* __restrict__ ord,
                                                      uint32_t n_edges, const double* __restrict__ gq,
                                                      double* __restrict__ gfault) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_edges) return;
  const uint32_t e = j;
  const uint32_t i0 = st.e_first[e], cnt = st.e_cnt[e];
  uint32_t half = 0;
  double prod = 1.0;
  for (uint32_t i = 0; i < cnt; ++i) {
    const double p = st.frp[ord[i0 + i]].p;
    if (p == 0.5) half++;
    else prod *= 1.0 - 2.0 * p;
  }
  const double g = gq[j];
  for (uint32_t i = 0; i < cnt; ++i) {
    const uint32_t pos = ord[i0 + i];
    const double p = st.frp[pos].p;
    const double d = half == 0 ? prod / (1.0 - 2.0 * p) : (half == 1 && p == 0.5 ? prod : 0.0);
    gfault[pos] = g * d;
  }
}

// dp/dr of a fault's split: (1-2p)^k = 1 - x, x = a r, so dp/dr =
// (a / 2k)(1 - x)^(1/k - 1): DEPOLARIZE1 (1/3)(1 - 4r/3)^(-1/2), DEPOLARIZE2
// (1/15)(1 - 16r/15)^(-7/8), a Pauli flip 1.
__device__ __forceinline__ double fault_dp_dr(uint32_t kind, double r) {
  if (kind == CH_DEP1) return (1.0 / 3.0) / sqrt(1.0 - 4.0 * r / 3.0);
  if (kind == CH_DEP2) return (1.0 / 15.0) * exp(-0.875 * log1p(-16.0 * r / 15.0));
  return 1.0;
}

// Per channel: its faults' dL/dp summed in fault order, times dp/dr; into
// st.gr (lowered order) or, with `out`, out[program-order channel].
__global__ __launch_bounds__(kBlock) void k_adj_channels(DevState st, const double* __restrict__ rates,
                                                         const double* __restrict__ gfault, double* __restrict__ out) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= st.n_chan) return;
  double sum = 0.0;
  for (uint32_t f = st.chan_foff[c]; f < st.chan_foff[c + 1]; ++f) sum += gfault[f];
  const double g = sum * fault_dp_dr(st.chan_kind[c], channel_rate(st, rates, c));
  if (out) out[st.chan_src[c]] = g;
  else st.gr[c] = g;
}

__global__ __launch_bounds__(kBlock) void k_zero_f64(double* __restrict__ a, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = 0.0;
}

inline uint32_t cdiv(uint64_t a, uint64_t b) { return uint32_t((a + b - 1) / b); }

}  // namespace

const char* kernel_name(int id) {
  static const char* names[K_COUNT] = {"k_prepare",    "k_sweep",       "k_hash",   "k_scan_single", "k_compact",
                                       "k_onesweep",   "k_heads_count", "k_heads_apply", "k_reduce",  "k_reduce_big",
                                       "k_edge_write",  "k_bucket",     "k_bucket_bounds", "k_rep_list"};
  return (id >= 0 && id < K_COUNT) ? names[id] : "?";
}

uint32_t sort_passes(uint64_t n) {
  uint32_t lg = 1;
  while ((1ull << lg) < n && lg < 40) lg++;
  uint32_t bits = 2 * lg + 12;
  if (bits < 16) bits = 16;
  uint32_t p = (bits + 7) / 8;
  return p > uint32_t(kMaxPasses) ? uint32_t(kMaxPasses) : p;
}

uint32_t class_key_bits(uint64_t n, uint32_t cap) {
  const uint32_t b = 8 * sort_passes(n);
  return cap < b ? cap : b;
}

size_t hash_lds_bytes(uint32_t w) { return (size_t(w) + 1) * 8 + size_t(w) * (8 + 8 + 8 * kHashBmw + 4); }

// LDS of one sweep work-group, in the order k_sweep lays it out: the frame
// (2n words) and the two pending-leaf buffers (2n words), the injection
// words, then the 32-bit tables (op windows, layer / fault / bitmap offsets,
// injection layers, qubits and group ends, the window table).
template <int kBlk>
static size_t sweep_lds_shape(uint32_t n_qubits) {
  using S = SweepShape<kBlk>;
  return (size_t(4) * n_qubits + S::kInj) * sizeof(uint64_t) +
         (size_t(2) * S::kWin + 3 * S::kLofs + 2 + 3 * S::kInj + 3 * S::kWinTab) * sizeof(uint32_t);
}

size_t sweep_lds_bytes(uint32_t n_qubits) { return sweep_lds_shape<1024>(n_qubits); }

// The small shape is used when there are enough items to give each CU
// several, its tables hold the circuit and two of its work-groups fit in one
// CU's LDS.
bool sweep_small_fits(const DevState& st) {
  using S = SweepShape<256>;
  return st.n_layers + 2 <= uint32_t(S::kLofs) && st.n_win <= uint32_t(S::kWinTab) &&
         st.max_win_ops <= uint32_t(S::kWin) &&
         2 * (sweep_lds_shape<256>(st.n_qubits) + 1024) <= 160 * 1024;
}

static size_t g_lds_limit = 64 * 1024;
static uint32_t g_n_cus = 0;  // compute units of the device (0: unknown)
static bool g_bucket_ok = false;

size_t sweep_lds_limit() { return g_lds_limit; }
bool bucket_grouping_available() { return g_bucket_ok; }
static constexpr size_t kBucketDynLds = 2 * size_t(kBucketCap) * sizeof(uint64_t);

hipError_t configure_kernels() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int lds = 0;
  e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  g_n_cus = cus > 0 ? uint32_t(cus) : 0u;
  // leave room for the sweep's static shared words
  size_t lim = size_t(lds) > 1024 ? size_t(lds) - 1024 : size_t(lds);
  if (lim > 64 * 1024) {
    const void* variants[3] = {reinterpret_cast<const void*>(&k_sweep<true, 1024>),
                               reinterpret_cast<const void*>(&k_sweep<false, 1024>),
                               reinterpret_cast<const void*>(&k_sweep<true, 256>)};
    for (const void* f : variants)
      if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lim));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      lim = 64 * 1024 - 1024;
    }
  }
  g_lds_limit = lim;
  // the hash stages its cover list and bitmap words (at most kMaxHashWords columns)
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hash), hipFuncAttributeMaxDynamicSharedMemorySize,
                          int(hash_lds_bytes(kMaxHashWords))) != hipSuccess)
    (void)hipGetLastError();
  // the bucket grouping needs its two sort buffers next to its static arrays
  g_bucket_ok = false;
  hipFuncAttributes fa{};
  const void* bucket8 = reinterpret_cast<const void*>(&k_bucket<kBucketBlock, kBucketCap, false>);
  if (hipFuncGetAttributes(&fa, bucket8) == hipSuccess && fa.sharedSizeBytes + kBucketDynLds <= size_t(lds)) {
    g_bucket_ok = hipFuncSetAttribute(bucket8,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, int(kBucketDynLds)) == hipSuccess;
  }
  (void)hipGetLastError();
  return hipSuccess;
}

#define GP_LAUNCH(id, ...)                      \
  do {                                          \
    if (hook.before) hook.before(hook.ctx, id); \
    __VA_ARGS__;                                \
    if (hook.after) hook.after(hook.ctx, id);   \
    hipError_t _e = hipGetLastError();          \
    if (_e != hipSuccess) return _e;            \
  } while (0)

hipError_t enqueue_compile(DevState& st_io, hipStream_t stream, const LaunchHook& hook) {
  DevState st = st_io;
  st_io.ord = st.val[0];
  const uint32_t n = st.n_faults;
  const uint32_t ntiles = cdiv(n ? n : 1, kTile);
  // passes: enough key bits for the faults; every bit after a collision
  if (st.key_mode == 1) {
    st.n_pass = kMaxPasses;
    st.key_bits = 64;
  } else {
    st.n_pass = sort_passes(n);
    st.key_bits = class_key_bits(n, st.key_bits);
  }
  // 16-bit buckets: from kBucket16MinFaults faults (or when forced), while
  // the key has two digits above the ones sorted in LDS
  st.use_b16 = st.key_mode == 0 && n <= kBucket16MaxFaults && st.n_pass >= 3 &&
                       (st.sort_mode == SORT_BUCKET16 || (st.sort_mode == SORT_AUTO && n >= kBucket16MinFaults))
                   ? 1u
                   : 0u;
  {
    // a block per kPrepChan channels, or per kBlock look-back words to clear
    const uint32_t g_chan = cdiv(st.n_chan ? st.n_chan : 1, kPrepChan);
    const uint32_t g_clear = cdiv(st.n_pass * ntiles * 256, kBlock);
    uint32_t g = g_chan > g_clear ? g_chan : g_clear;
    if (g > 4096) g = 4096;
    GP_LAUNCH(K_PREPARE, k_prepare<<<g, kBlock, 0, stream>>>(st));
  }
  if (st.n_items) {
    // the small shape for many items of small circuits (several per CU)
    const bool small = st.sweep_shape == 2 || (st.sweep_shape == 0 && st.n_items >= 512 && sweep_small_fits(st));
    // one 1024-thread item per CU: the XCD-contiguous item order when they
    // all fit at once
    st.item_xcd = !small && st.n_items <= g_n_cus ? 1u : 0u;
    if (small && sweep_small_fits(st)) {
      GP_LAUNCH(K_SWEEP, k_sweep<true, 256><<<st.n_items, 256, sweep_lds_shape<256>(st.n_qubits), stream>>>(st));
    } else if (st.n_layers + 2 <= uint32_t(kLofsMax) && st.n_win <= uint32_t(kWinTableLds)) {
      GP_LAUNCH(K_SWEEP,
                k_sweep<true, 1024><<<st.n_items, kSweepBlock, sweep_lds_bytes(st.n_qubits), stream>>>(st));
    } else {
      GP_LAUNCH(K_SWEEP,
                k_sweep<false, 1024><<<st.n_items, kSweepBlock, sweep_lds_bytes(st.n_qubits), stream>>>(st));
    }
  }
  // hyperedges in representative-position order (after any grouping): tile
  // counts, their prefix, the hyperedges, each circuit's first hyperedge
  auto output = [&]() -> hipError_t {
    GP_LAUNCH(K_REP_LIST, k_rep_list<<<ntiles, kBlock, 0, stream>>>(st, ntiles));
    GP_LAUNCH(K_EDGE_WRITE, k_edge_write<<<cdiv(n ? n : 1, kBlock), kBlock, 0, stream>>>(st));
    return hipSuccess;
  };
  if (n == 0) return output();
  GP_LAUNCH(K_HASH, k_hash<<<st.n_hchunks, kBlock, hash_lds_bytes(st.w_max), stream>>>(st));
  if (st.use_b16) {
    // two stable passes on the top two digits (the second carries the fault
    // records), the bucket ranges, then each bucket in LDS
    const uint32_t msd = st.n_pass - 1;
    const uint32_t g = cdiv(n, kBlock) < 8192u ? cdiv(n, kBlock) : 8192u;
    GP_LAUNCH(K_COMPACT, k_compact<<<ntiles, kCompactBlock, 0, stream>>>(st, msd - 1));
    GP_LAUNCH(K_ONESWEEP, k_onesweep<<<ntiles, kSortBlock, 0, stream>>>(st, msd - 1, st.key[0], st.val[0], st.key[1],
                                                                     st.val[1], nullptr, nullptr));
    GP_LAUNCH(K_ONESWEEP, k_onesweep<<<ntiles, kSortBlock, 0, stream>>>(st, msd, st.key[1], st.val[1], st.key[0],
                                                                     st.val[0], st.frp, st.crp));
    GP_LAUNCH(K_BUCKET_BOUNDS, k_bucket_bounds<<<g, kBlock, 0, stream>>>(st, st.key[0]));
    GP_LAUNCH(K_BUCKET, k_bucket<256, kBucket16Cap, true><<<kBuckets16, 256, 2 * kBucket16Cap * sizeof(uint64_t),
                                                            stream>>>(st, st.key[0], st.val[0], st.val[1]));
    st_io.ord = st.val[1];
    return output();
  }
  // buckets: one stable pass on the top digit, then each bucket in LDS
  const bool bucketed = st.sort_mode == SORT_AUTO && st.key_mode == 0 && g_bucket_ok && n <= kBucketMaxFaults &&
                        st.n_pass >= 2 && st.n_pass <= 7;
  if (bucketed) {
    const uint32_t msd = st.n_pass - 1;
    GP_LAUNCH(K_COMPACT, k_compact<<<ntiles, kCompactBlock, 0, stream>>>(st, msd));
    GP_LAUNCH(K_ONESWEEP, k_onesweep<<<ntiles, kSortBlock, 0, stream>>>(st, msd, st.key[0], st.val[0], st.key[1],
                                                                     st.val[1], st.frp, st.crp));
    GP_LAUNCH(K_BUCKET, k_bucket<kBucketBlock, kBucketCap, false><<<kBuckets, kBucketBlock, kBucketDynLds, stream>>>(
                            st, st.key[1], st.val[1], st.val[0]));
    return output();
  }
  GP_LAUNCH(K_COMPACT, k_compact<<<ntiles, kCompactBlock, 0, stream>>>(st, 0));
  for (uint32_t pass = 0; pass < st.n_pass; ++pass) {
    const int src = pass & 1, dst = src ^ 1;
    GP_LAUNCH(K_ONESWEEP, k_onesweep<<<ntiles, kSortBlock, 0, stream>>>(st, pass, st.key[src], st.val[src], st.key[dst],
                                                                     st.val[dst], nullptr, nullptr));
  }
  const int fin = st.n_pass & 1;
  st_io.ord = st.val[fin];
  GP_LAUNCH(K_HEADS_COUNT, k_heads_count<<<ntiles, kBlock, 0, stream>>>(st.key[fin], st.hdr, st.tile_sum));
  GP_LAUNCH(K_SCAN_SINGLE,
            k_scan_single<uint32_t><<<1, kScanSingleBlock, 0, stream>>>(st.tile_sum, ntiles, nullptr, &st.hdr->n_seg));
  GP_LAUNCH(K_HEADS_APPLY, k_heads_apply<<<ntiles, kBlock, 0, stream>>>(st.key[fin], st.hdr, st.tile_sum,
                                                                         st.segstart));
  GP_LAUNCH(K_REDUCE, k_reduce<<<cdiv(n, kBlock), kBlock, 0, stream>>>(st, st.val[fin]));
  GP_LAUNCH(K_REDUCE_BIG, k_reduce_big<<<256, kBlock, 0, stream>>>(st, st.val[fin]));
  return output();
}

hipError_t enqueue_refresh(const DevState& st, uint32_t n_edges, hipStream_t stream) {
  return enqueue_aggregate(st, n_edges, nullptr, st.edge_q, stream);
}

hipError_t enqueue_rates_gradient(const DevState& st, uint32_t n_edges, hipStream_t stream) {
  if (st.n_faults) k_zero_f64<<<min(cdiv(st.n_faults, kBlock), 4096u), kBlock, 0, stream>>>(st.gfault, st.n_faults);
  if (n_edges) k_adj_edges<<<cdiv(n_edges, kBlock), kBlock, 0, stream>>>(st, st.ord, n_edges, st.gq, st.gfault);
  if (st.n_chan) k_adj_channels<<<cdiv(st.n_chan, kBlock), kBlock, 0, stream>>>(st, nullptr, st.gfault, nullptr);
  return hipGetLastError();
}

hipError_t enqueue_aggregate(const DevState& st, uint32_t n_edges, const double* rates,
                             double* q, hipStream_t stream) {
  if (st.n_chan) k_fault_p<<<cdiv(st.n_chan, kBlock), kBlock, 0, stream>>>(st, rates);
  k_clear_big<<<1, kBlock, 0, stream>>>(st);
  if (n_edges) {
    k_remerge<<<cdiv(n_edges, kBlock), kBlock, 0, stream>>>(st, st.ord, n_edges, q);
    k_remerge_big<<<64, kBucketBlock, 0, stream>>>(st, st.ord, q);
  }
  return hipGetLastError();
}

hipError_t enqueue_aggregate_backward(const DevState& st, uint32_t n_edges, const double* rates,
                                      const double* gq, double* grates, double* gfault,
                                      hipStream_t stream) {
  if (!gfault) gfault = st.gfault;
  if (st.n_chan) k_fault_p<<<cdiv(st.n_chan, kBlock), kBlock, 0, stream>>>(st, rates);
  // faults outside every hyperedge (empty signature) keep dL/dp = 0
  if (st.n_faults) k_zero_f64<<<min(cdiv(st.n_faults, kBlock), 4096u), kBlock, 0, stream>>>(gfault, st.n_faults);
  if (n_edges) k_adj_edges<<<cdiv(n_edges, kBlock), kBlock, 0, stream>>>(st, st.ord, n_edges, gq, gfault);
  if (st.n_chan) k_adj_channels<<<cdiv(st.n_chan, kBlock), kBlock, 0, stream>>>(st, rates, gfault, grates);
  return hipGetLastError();
}

// ------------------------------------------------------------ static scratch

// Per-fault dL/dp of the allocation-free adjoint. In host code `scratch`
// names a host-side stand-in, not device memory: kernels receive the device
// address that hipGetSymbolAddress gives for the current device, kept per
// device by scratch_init.
static __device__ __align__(256) double scratch[kScratchFaults];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return hipSuccess;
}

double* scratch_for(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace gp
