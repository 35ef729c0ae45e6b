// Test-only CPU interpreter of the lowered tables produced by the compiler's
// host lowering (paper_2604_16613_amd/csrc/lower.cpp). It replays the stage-1
// work items exactly as the device sweep schedules them -- same tables, same
// per-column slab addressing, same early stop -- with every table and slab
// access bounds-checked, and returns each fault's signature. Tests compare
// those signatures with the oracle's before any kernel runs on a GPU.
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "gp.h"
#include "lower.h"

using namespace gp;

namespace {
std::string g_msg;
int bad(const char* what) {
  g_msg = what;
  return -100;
}
}  // namespace

extern "C" const char* hc_error() { return g_msg.c_str(); }

// per work item of the last hc_run: layers swept, words emitted
static std::vector<uint64_t> g_item_stats;
extern "C" uint64_t hc_item_stats(uint64_t* out, uint64_t cap) {
  for (size_t i = 0; i < g_item_stats.size() && i < cap; i++) out[i] = g_item_stats[i];
  return g_item_stats.size();
}

// Replay the lowered tables (one circuit, or a merged batch) as the device
// addresses them: every circuit through its descriptor, every access checked.
// Signature bits use each circuit's own numbering.
// stats: [0] faults, [1] items, [2] slab words, [3] layers (most of any circuit),
//        [4] gauge flag, [5] words written, [6] columns, [7] qubits (most),
//        [8] injection entries of the longest column list
static int replay(const Lowered& lw, uint64_t* off, uint32_t* bits, uint64_t bits_cap, uint32_t* src,
                  uint32_t* code, uint64_t* stats, uint64_t max_faults) {
  const uint32_t W = lw.w;
  const uint64_t F = lw.n_faults;
  if (F > max_faults) return bad("fault capacity too small");
  if (lw.branches.empty()) return bad("no circuit descriptor");
  // descriptors tile the batch's tables in order
  {
    uint32_t lob = 0, bb = 0, wb = 0, wib = 0, fb = 0;
    for (const BranchDesc& br : lw.branches) {
      if (br.lob != lob || br.bb != bb || br.wb != wb || br.wib != wib || br.fb != fb || br.fe < br.fb)
        return bad("descriptor bases do not tile the tables");
      if (br.nw > lw.w_max || br.wd > br.nw) return bad("descriptor columns");
      lob += br.n_layers + 1;
      bb += br.n_layers + 2;
      wb += br.nw;
      wib += br.n_win;
      fb = br.fe;
    }
    if (lob != lw.layer_off.size() || lob != lw.layer_win.size() || bb != lw.bnd_fault_off.size() ||
        bb != lw.bnd_chan_off.size() || bb != lw.bnd_bm_off.size() || wb != W || wib != lw.win_lo.size() ||
        fb != F)
      return bad("descriptors do not cover the tables");
  }
  if (lw.item_branch.size() != lw.item_col.size() || lw.hchunk_branch.size() != lw.hchunk_pos.size())
    return bad("per-item circuit tables");
  if (lw.fnv_pow.size() < lw.w_max + 1u) return bad("fnv powers");
  for (const BranchDesc& br : lw.branches) {
    const uint32_t n = br.n_qubits, L = br.n_layers;
    const uint32_t* layer_off = lw.layer_off.data() + br.lob;
    if (layer_off[L] - layer_off[0] > lw.ops.size()) return bad("layer_off");
    for (uint32_t t = 0; t < L; t++) {
      // the layer lies inside its op window
      const uint32_t k = lw.layer_win[br.lob + t];
      if (k >= br.n_win) return bad("layer window index");
      const uint32_t ob = lw.win_obase[br.wib + k], oc = lw.win_cnt[br.wib + k];
      if (oc > kSweepWinOps || ob + oc > lw.ops32.size()) return bad("op window out of range");
      if (layer_off[t] < ob || layer_off[t + 1] > ob + oc || lw.win_lo[br.wib + k] > t)
        return bad("layer outside its op window");
      std::vector<char> seen(n, 0);
      for (uint32_t o = layer_off[t]; o < layer_off[t + 1]; o++) {
        uint64_t op = lw.ops[o];
        uint32_t kind = uint32_t(op >> 56), a = uint32_t(op >> 28) & kField, b = uint32_t(op) & kField;
        if (a >= n || seen[a]++) return bad("layer touches a qubit twice or out of range");
        if (kind == OP_CX || kind == OP_CZ || kind == OP_SWAP) {
          if (b >= n || seen[b]++) return bad("layer touches a qubit twice (pair)");
        }
      }
    }
    if (lw.bnd_fault_off[br.bb] != br.fb || lw.bnd_fault_off[br.bb + L + 1] != br.fe) return bad("bnd_fault_off");
    for (uint32_t c = lw.bnd_chan_off[br.bb]; c < lw.bnd_chan_off[br.bb + L + 1]; c++) {
      if (lw.chan_qa[c] >= n) return bad("channel qubit");
      if (lw.chan_kind[c] == CH_DEP2 && lw.chan_qb[c] >= n) return bad("channel qubit b");
      if (lw.chan_foff[c] < br.fb || lw.chan_foff[c + 1] > br.fe) return bad("channel faults outside the circuit");
    }
  }
  // bitmap regions: column w at boundary b owns ceil(faults at b / 64) words
  {
    std::vector<char> owned(lw.bm_words, 0);
    for (const BranchDesc& br : lw.branches)
      for (uint32_t w = br.wb; w < br.wb + br.nw; w++) {
        const int top = lw.col_top[w];
        for (int b = 0; b <= top; b++) {
          const uint32_t nf = lw.bnd_fault_off[br.bb + b + 1] - lw.bnd_fault_off[br.bb + b];
          const uint64_t o = lw.col_bm_base[w] + lw.bnd_bm_off[br.bb + b];
          if (lw.bnd_bm_off[br.bb + b + 1] - lw.bnd_bm_off[br.bb + b] != (nf + 63) / 64)
            return bad("bitmap words of a boundary");
          for (uint64_t i = o; i < o + (nf + 63) / 64; i++) {
            if (i >= lw.bm_words) return bad("bitmap word out of range");
            if (owned[i]++) return bad("bitmap regions overlap");
          }
        }
      }
  }
  std::vector<uint64_t> slab(lw.slab_words, 0);
  std::vector<char> written(lw.slab_words, 0);
  std::vector<int32_t> cover_lo(W, 0);
  uint64_t nwritten = 0;
  int gauge = 0;
  if (lw.ops32.size() != lw.ops.size() || lw.inj_off.size() != W + 1u) return bad("device tables missing");
  g_item_stats.assign(2 * lw.item_col.size(), 0);
  for (size_t it = 0; it < lw.item_col.size(); it++) {
    if (lw.item_branch[it] >= lw.branches.size()) return bad("item circuit");
    const BranchDesc& br = lw.branches[lw.item_branch[it]];
    const uint32_t n = br.n_qubits;
    const uint32_t* layer_off = lw.layer_off.data() + br.lob;
    const uint32_t* bnd_chan_off = lw.bnd_chan_off.data() + br.bb;
    const uint32_t w = lw.item_col[it];
    if (w < br.wb || w >= br.wb + br.nw) return bad("item column outside its circuit");
    const int top = lw.col_top[w], clo = lw.col_lo[w];
    const int blo = int(lw.item_blo[it]), bhi = int(lw.item_bhi[it]);
    if (top < 0 || top >= int(br.n_layers) || bhi > top || blo > bhi) return bad("item range");
    const uint64_t base = lw.col_base[w];
    const uint64_t cap = lw.bnd_fault_off[br.bb + top + 1];
    std::vector<uint64_t> fr(2 * size_t(n), 0);
    std::vector<uint64_t> pend(n, 0);
    uint32_t ip = lw.inj_off[w];
    const uint32_t ip_end = lw.inj_off[w + 1];
    if (ip_end > lw.inj_layer.size()) return bad("injection range");
    auto scatter = [&](int layer) -> int {
      while (ip < ip_end && int(lw.inj_layer[ip]) == layer) {
        const uint32_t q = lw.inj_qubit[ip];
        if (q >= n) return bad("injection qubit");
        if (pend[q]) return bad("two injections for one qubit in one layer");
        pend[q] = lw.inj_word[ip];
        ip++;
      }
      if (ip < ip_end && int(lw.inj_layer[ip]) > layer) return bad("injections out of order");
      return 0;
    };
    if (ip < ip_end && int(lw.inj_layer[ip]) != top) return bad("first injection is not at the top layer");
    if (scatter(top)) return -100;
    int nz = 0;
    bool dead = false;
    for (int t = top; t >= blo; --t) {
      g_item_stats[2 * it]++;
      int dnz = 0;
      auto nzd = [](uint64_t a, uint64_t b) { return int(a != 0) - int(b != 0); };
      for (uint32_t o = layer_off[t]; o < layer_off[t + 1]; o++) {
        const uint32_t op = lw.ops32[o];
        if (op == 0xFFFFFFFFu) return bad("qubit index too large for the compact op word");
        const uint32_t kind = op >> 28, a = (op >> kQubitBits) & kQField, b = op & kQField;
        if ((lw.ops[o] >> 56) != kind) return bad("compact op kind differs");
        uint64_t& xa = fr[2 * a];
        uint64_t& za = fr[2 * a + 1];
        const uint64_t x0 = xa, z0 = za;
        switch (kind) {
          case OP_H: xa = z0; za = x0; break;
          case OP_S: xa = x0 ^ z0; dnz += nzd(xa, x0); break;
          case OP_SQRTX: za = x0 ^ z0; dnz += nzd(za, z0); break;
          case OP_CX: {
            uint64_t& xb = fr[2 * b]; uint64_t& zb = fr[2 * b + 1];
            uint64_t x1 = xb, z1 = zb;
            xa = x0 ^ x1; zb = z1 ^ z0;
            dnz += nzd(xa, x0) + nzd(zb, z1);
            break;
          }
          case OP_CZ: {
            uint64_t& xb = fr[2 * b]; uint64_t& zb = fr[2 * b + 1];
            uint64_t x1 = xb, z1 = zb;
            xa = x0 ^ z1; xb = x1 ^ z0;
            dnz += nzd(xa, x0) + nzd(xb, x1);
            break;
          }
          case OP_SWAP: {
            uint64_t& xb = fr[2 * b]; uint64_t& zb = fr[2 * b + 1];
            std::swap(xa, xb); std::swap(za, zb);
            break;
          }
          case OP_R: gauge |= z0 != 0; xa = 0; za = 0; dnz -= int(x0 != 0) + int(z0 != 0); break;
          case OP_RX: gauge |= x0 != 0; xa = 0; za = 0; dnz -= int(x0 != 0) + int(z0 != 0); break;
          case OP_M: gauge |= z0 != 0; xa = x0 ^ pend[a]; pend[a] = 0; dnz += nzd(xa, x0); break;
          case OP_MX: gauge |= x0 != 0; za = z0 ^ pend[a]; pend[a] = 0; dnz += nzd(za, z0); break;
          case OP_MR: gauge |= z0 != 0; xa = pend[a]; za = 0; pend[a] = 0; dnz += nzd(xa, x0) - int(z0 != 0); break;
          case OP_MRX: gauge |= x0 != 0; za = pend[a]; xa = 0; pend[a] = 0; dnz += nzd(za, z0) - int(x0 != 0); break;
          default: return bad("op kind");
        }
      }
      for (uint32_t q = 0; q < n; q++)
        if (pend[q]) return bad("an injection was not consumed by a measurement of its layer");
      nz += dnz;
      int full = 0;
      for (uint64_t v : fr) full += v != 0;
      if (full != nz) return bad("incremental non-zero count disagrees with a full count");
      if (t <= bhi) {
        for (uint32_t c = bnd_chan_off[t]; c < bnd_chan_off[t + 1]; c++) {
          const uint64_t x0 = fr[2 * lw.chan_qa[c]], z0 = fr[2 * lw.chan_qa[c] + 1];
          uint64_t words[15];
          int nwd = 0;
          switch (lw.chan_kind[c]) {
            case CH_X: words[nwd++] = x0; break;
            case CH_Y: words[nwd++] = x0 ^ z0; break;
            case CH_Z: words[nwd++] = z0; break;
            case CH_DEP1: words[nwd++] = x0; words[nwd++] = x0 ^ z0; words[nwd++] = z0; break;
            case CH_DEP2: {
              const uint64_t x1 = fr[2 * lw.chan_qb[c]], z1 = fr[2 * lw.chan_qb[c] + 1];
              const uint64_t A[4] = {0, x0, z0, x0 ^ z0}, B[4] = {0, x1, z1, x1 ^ z1};
              for (int k = 1; k < 16; k++) words[nwd++] = A[k & 3] ^ B[k >> 2];
              break;
            }
            default: return bad("channel kind");
          }
          for (int k = 0; k < nwd; k++) {
            uint64_t pos = lw.chan_foff[c] + k;
            if (pos >= cap) return bad("emission beyond the column's slab");
            uint64_t idx = base + pos;
            if (idx >= lw.slab_words) return bad("slab index out of range");
            if (written[idx]) return bad("slab word written twice");
            written[idx] = 1;
            slab[idx] = words[k];
            nwritten++;
            g_item_stats[2 * it + 1]++;
          }
        }
      }
      if (t > 0 && scatter(t - 1)) return -100;
      if (nz == 0 && t <= clo) {
        if (t <= bhi) cover_lo[w] = t;
        dead = true;
        break;
      }
    }
    if (!dead && blo == 0)
      for (uint32_t q = 0; q < n; q++) gauge |= fr[2 * q + 1] != 0;
  }
  // hash chunks cover every position once, each inside one boundary of its circuit
  {
    std::vector<char> seen(F, 0);
    if (lw.hchunk_pos.size() != lw.hchunk_bnd.size()) return bad("hash chunk arrays");
    for (size_t k = 0; k < lw.hchunk_pos.size(); k++) {
      if (lw.hchunk_branch[k] >= lw.branches.size()) return bad("hash chunk circuit");
      const BranchDesc& br = lw.branches[lw.hchunk_branch[k]];
      const uint32_t b = lw.hchunk_bnd[k], p0 = lw.hchunk_pos[k];
      if (b > br.n_layers || p0 < lw.bnd_fault_off[br.bb + b] || p0 >= lw.bnd_fault_off[br.bb + b + 1])
        return bad("hash chunk boundary");
      const uint32_t p1 = std::min<uint32_t>(p0 + 256, lw.bnd_fault_off[br.bb + b + 1]);
      for (uint32_t p = p0; p < p1; p++) {
        if (seen[p]) return bad("hash chunks overlap");
        seen[p] = 1;
      }
    }
    for (uint64_t p = 0; p < F; p++)
      if (!seen[p]) return bad("hash chunks miss a position");
  }
  // signatures of every fault position from its circuit's covered columns
  uint64_t nb = 0;
  off[0] = 0;
  for (const BranchDesc& br : lw.branches) {
    for (uint32_t b = 0; b <= br.n_layers; b++) {
      for (uint32_t c = lw.bnd_chan_off[br.bb + b]; c < lw.bnd_chan_off[br.bb + b + 1]; c++) {
        for (uint32_t pos = lw.chan_foff[c]; pos < lw.chan_foff[c + 1]; pos++) {
          for (uint32_t w = br.wb; w < br.wb + br.nw; w++) {
            const int top = lw.col_top[w];
            if (top < 0 || int(b) > top || int(b) < cover_lo[w]) continue;
            uint64_t idx = lw.col_base[w] + pos;
            if (!written[idx]) return bad("covered slab word never written");
            uint64_t v = slab[idx];
            while (v) {
              uint32_t bit = (w - br.wb) * 64 + uint32_t(__builtin_ctzll(v));
              if (nb >= bits_cap) return bad("bit capacity");
              bits[nb++] = bit < br.wd * 64 ? bit : br.n_det + (bit - br.wd * 64);
              v &= v - 1;
            }
          }
          off[pos + 1] = nb;
          src[pos] = lw.chan_src[c];
          uint32_t k = pos - lw.chan_foff[c];
          code[pos] = kept_code(lw.chan_kind[c], lw.level, k);
        }
      }
    }
  }
  uint32_t L = 0, nq = 0;
  for (const BranchDesc& br : lw.branches) {
    L = std::max(L, br.n_layers);
    nq = std::max(nq, br.n_qubits);
  }
  stats[0] = F;
  stats[1] = lw.item_col.size();
  stats[2] = lw.slab_words;
  stats[3] = L;
  stats[4] = uint64_t(gauge);
  stats[5] = nwritten;
  stats[6] = W;
  stats[7] = nq;
  uint64_t mi = 0;
  for (size_t w = 0; w + 1 < lw.inj_off.size(); w++) mi = std::max<uint64_t>(mi, lw.inj_off[w + 1] - lw.inj_off[w]);
  stats[8] = mi;
  return 0;
}

// the observable range cut used by hc_run (the lowering's cost per fault)
static double g_fault_cost = kDefaultFaultCost;
extern "C" void hc_set_fault_cost(double c) { g_fault_cost = c; }

extern "C" int hc_run(const char* text, size_t len, const double* rates, size_t n_rates, uint64_t* off,
                      uint32_t* bits, uint64_t bits_cap, uint32_t* src, uint32_t* code, uint64_t* stats,
                      uint64_t max_faults) {
  Lowered lw;
  LowerError err{};
  int rc = lower_circuit(text, len, rates, n_rates, kSweepSlots, lw, err, 2, g_fault_cost);
  if (rc) {
    g_msg = err.msg;
    return rc;
  }
  return replay(lw, off, bits, bits_cap, src, code, stats, max_faults);
}

// The same for a batch: each circuit lowered with `slots` sweep slots, then
// merged. Positions (and so off, src, code) run over the batch in circuit order;
// src is the batch's channel number.
extern "C" int hc_run_batch(const char* const* texts, const size_t* lens, size_t n_texts, uint32_t slots,
                            uint64_t* off, uint32_t* bits, uint64_t bits_cap, uint32_t* src, uint32_t* code,
                            uint64_t* stats, uint64_t max_faults, uint32_t* fault_circuit) {
  std::vector<Lowered> parts(n_texts);
  for (size_t k = 0; k < n_texts; k++) {
    LowerError err{};
    int rc = lower_circuit(texts[k], lens[k], nullptr, 0, slots, parts[k], err);
    if (rc) {
      g_msg = err.msg;
      return rc;
    }
  }
  Lowered lw;
  merge_branches(parts, lw);
  if (lw.n_faults > max_faults) return bad("fault capacity too small");
  for (size_t k = 0; k < lw.branches.size(); k++)
    for (uint32_t p = lw.branches[k].fb; p < lw.branches[k].fe; p++) fault_circuit[p] = uint32_t(k);
  return replay(lw, off, bits, bits_cap, src, code, stats, max_faults);
}

// A digest (FNV-1a over the bytes) of every table of a lowering, lowered into
// a Lowered kept across calls (reuse != 0) or into a fresh one: the kept one
// must give the fresh one's tables whatever was lowered into it before.
static uint64_t digest_bytes(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; i++) h = (h ^ c[i]) * 1099511628211ull;
  return (h ^ n) * 1099511628211ull;
}
template <typename V>
static uint64_t digest_vec(uint64_t h, const V& v) {
  return digest_bytes(h, v.data(), v.size() * sizeof(v[0]));
}
extern "C" int hc_lower_digest(const char* text, size_t len, int reuse, uint64_t* out) {
  static Lowered kept;
  Lowered fresh;
  Lowered& lw = reuse ? kept : fresh;
  LowerError err{0, ""};
  const int rc = lower_circuit(text, len, nullptr, 0, kSweepSlots, lw, err, 2, g_fault_cost);
  if (rc) {
    g_msg = err.msg;
    return rc;
  }
  uint64_t h = 1469598103934665603ull;
  const uint64_t scal[] = {lw.n_qubits, lw.n_layers, lw.n_meas, lw.n_det, lw.n_obs, lw.wd, lw.wo, lw.w,
                           lw.n_faults, lw.slab_words, lw.level, lw.bm_words, lw.w_max};
  h = digest_bytes(h, scal, sizeof scal);
  h = digest_vec(h, lw.ops), h = digest_vec(h, lw.layer_off), h = digest_vec(h, lw.leaf_off);
  h = digest_vec(h, lw.leaf_bits), h = digest_vec(h, lw.meas_layer), h = digest_vec(h, lw.chan_qa);
  h = digest_vec(h, lw.chan_qb), h = digest_vec(h, lw.chan_kind), h = digest_vec(h, lw.chan_rate);
  h = digest_vec(h, lw.chan_src), h = digest_vec(h, lw.chan_foff), h = digest_vec(h, lw.bnd_chan_off);
  h = digest_vec(h, lw.bnd_fault_off), h = digest_vec(h, lw.col_top), h = digest_vec(h, lw.col_lo);
  h = digest_vec(h, lw.col_base), h = digest_vec(h, lw.item_col), h = digest_vec(h, lw.item_blo);
  h = digest_vec(h, lw.item_bhi), h = digest_vec(h, lw.fnv_pow), h = digest_vec(h, lw.ops32);
  h = digest_vec(h, lw.inj_off), h = digest_vec(h, lw.inj_layer), h = digest_vec(h, lw.inj_qubit);
  h = digest_vec(h, lw.inj_word), h = digest_vec(h, lw.inj_next), h = digest_vec(h, lw.hchunk_pos);
  h = digest_vec(h, lw.hchunk_bnd), h = digest_vec(h, lw.layer_win), h = digest_vec(h, lw.win_lo);
  h = digest_vec(h, lw.win_obase), h = digest_vec(h, lw.win_cnt), h = digest_vec(h, lw.bnd_bm_off);
  h = digest_vec(h, lw.col_bm_base), h = digest_vec(h, lw.item_branch), h = digest_vec(h, lw.hchunk_branch);
  h = digest_bytes(h, lw.branches.data(), lw.branches.size() * sizeof(BranchDesc));
  *out = h;
  return 0;
}
