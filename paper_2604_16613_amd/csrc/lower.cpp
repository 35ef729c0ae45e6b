// Host lowering of circuit text to the device tables (see lower.h).
#include "lower.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <thread>

#include "gp.h"

namespace gp {
namespace {

enum Cls : uint8_t { G_1Q = 1, G_2Q, G_MEAS, G_RESET, G_PAULI, G_N1, G_N2, G_DET, G_OBS, G_IGNORE };

struct Gate {
  const char* name;
  uint8_t cls;
  uint8_t kind;
};

const Gate kGates[] = {
    {"CX", G_2Q, OP_CX},          {"CNOT", G_2Q, OP_CX},       {"ZCX", G_2Q, OP_CX},
    {"CZ", G_2Q, OP_CZ},          {"ZCZ", G_2Q, OP_CZ},        {"SWAP", G_2Q, OP_SWAP},
    {"H", G_1Q, OP_H},            {"H_XZ", G_1Q, OP_H},        {"S", G_1Q, OP_S},
    {"S_DAG", G_1Q, OP_S},        {"SQRT_Z", G_1Q, OP_S},      {"SQRT_Z_DAG", G_1Q, OP_S},
    {"SQRT_X", G_1Q, OP_SQRTX},   {"SQRT_X_DAG", G_1Q, OP_SQRTX},
    {"I", G_PAULI, 0},            {"X", G_PAULI, 0},           {"Y", G_PAULI, 0},
    {"Z", G_PAULI, 0},            {"R", G_RESET, OP_R},        {"RZ", G_RESET, OP_R},
    {"RX", G_RESET, OP_RX},       {"M", G_MEAS, OP_M},         {"MZ", G_MEAS, OP_M},
    {"MX", G_MEAS, OP_MX},        {"MR", G_MEAS, OP_MR},       {"MRZ", G_MEAS, OP_MR},
    {"MRX", G_MEAS, OP_MRX},      {"X_ERROR", G_N1, CH_X},     {"Y_ERROR", G_N1, CH_Y},
    {"Z_ERROR", G_N1, CH_Z},      {"DEPOLARIZE1", G_N1, CH_DEP1},
    {"DEPOLARIZE2", G_N2, CH_DEP2}, {"DETECTOR", G_DET, 0},    {"OBSERVABLE_INCLUDE", G_OBS, 0},
    {"TICK", G_IGNORE, 0},        {"QUBIT_COORDS", G_IGNORE, 0}, {"SHIFT_COORDS", G_IGNORE, 0},
};

constexpr uint32_t kObsFlag = 0x80000000u;
constexpr uint32_t kMaxIndex = (1u << 28) - 1;

// Instruction name -> gate: open addressing over a 128-slot table, built once
// (a linear scan per line cost a third of the parse on detector-heavy text).
const Gate* find_gate(const char* name, size_t nl) {
  struct Table {
    const Gate* slot[128] = {};
    static uint32_t hash(const char* s, size_t n) {
      uint32_t h = 2166136261u;
      for (size_t i = 0; i < n; i++) h = (h ^ uint8_t(s[i])) * 16777619u;
      return h;
    }
    Table() {
      for (const Gate& g : kGates) {
        uint32_t h = hash(g.name, std::strlen(g.name)) & 127u;
        while (slot[h]) h = (h + 1) & 127u;
        slot[h] = &g;
      }
    }
  };
  static const Table t;
  static_assert(sizeof(kGates) / sizeof(kGates[0]) < 96, "gate table load");
  for (uint32_t h = Table::hash(name, nl) & 127u; t.slot[h]; h = (h + 1) & 127u)
    if (!std::strcmp(t.slot[h]->name, name)) return t.slot[h];
  return nullptr;
}

// One instruction line, tokenized: its gate, arguments and targets (record
// targets flagged), with its line number within the chunk of text it came from.
struct Tok {
  const Gate* g;
  uint32_t line;
  uint32_t t0, t1;  // targets [t0, t1) of the chunk
  int nargs;
  double arg0;
};

// A chunk of whole lines, tokenized on its own thread. Tokenizing stops at
// the chunk's first syntax error, which is reported after the instructions
// before it have been applied (so errors keep program order).
struct TokChunk {
  std::vector<Tok> toks;
  std::vector<uint32_t> targets;
  std::vector<uint8_t> is_rec;
  uint32_t lines = 0;
  int err_code = 0;
  uint32_t err_line = 0;
  const char* err_fmt = nullptr;
  std::string err_what;
};

void tokenize_text(const char* p, const char* end, TokChunk& c);

// Tokenize a chunk; an allocation failure is recorded as the chunk's error
// (this runs on its own thread, so nothing may be thrown out of it).
void tokenize(const char* p, const char* end, TokChunk& c) {
  try {
    tokenize_text(p, end, c);
  } catch (...) {
    c.err_code = GP_E_OOM;
    c.err_line = 0;
    c.err_what.clear();
    c.err_fmt = "host memory allocation failed while tokenizing%s";
  }
}

void tokenize_text(const char* p, const char* end, TokChunk& c) {
  auto fail = [&](int code, uint32_t line, const char* fmt, const char* what) {
    c.err_code = code;
    c.err_line = line;
    c.err_fmt = fmt;
    c.err_what = what;
  };
  uint32_t line = 0;
  while (p < end) {
    line++;
    c.lines = line;
    const char* eol = static_cast<const char*>(std::memchr(p, '\n', size_t(end - p)));
    if (!eol) eol = end;
    const char* s = p;
    p = eol + 1;
    const char* hash = static_cast<const char*>(std::memchr(s, '#', size_t(eol - s)));
    const char* e = hash ? hash : eol;
    while (s < e && (*s == ' ' || *s == '\t' || *s == '\r')) s++;
    if (s == e) continue;
    char name[40];
    size_t nl = 0;
    while (s < e && *s != '(' && *s != ' ' && *s != '\t' && *s != '\r') {
      if (nl >= sizeof(name) - 1) return fail(GP_E_UNSUPPORTED, line, "unknown instruction %s", "(too long)");
      char ch = *s++;
      name[nl++] = (ch >= 'a' && ch <= 'z') ? char(ch - 32) : ch;
    }
    name[nl] = 0;
    if (!std::strcmp(name, "REPEAT") || name[0] == '{' || name[0] == '}')
      return fail(GP_E_UNSUPPORTED, line, "%s blocks are not supported", "REPEAT");
    const Gate* g = find_gate(name, nl);
    if (!g) return fail(GP_E_UNSUPPORTED, line, "unsupported instruction %s", name);
    Tok t{g, line, uint32_t(c.targets.size()), 0, 0, 0.0};
    if (s < e && *s == '(') {
      s++;
      for (;;) {
        while (s < e && (*s == ' ' || *s == '\t')) s++;
        if (s < e && *s == ')') {
          s++;
          break;
        }
        char buf[64];
        size_t bl = 0;
        while (s < e && *s != ',' && *s != ')' && bl < sizeof(buf) - 1) buf[bl++] = *s++;
        buf[bl] = 0;
        char* ep;
        double v = std::strtod(buf, &ep);
        if (ep == buf) return fail(GP_E_PARSE, line, "bad argument in %s", g->name);
        if (t.nargs == 0) t.arg0 = v;
        t.nargs++;
        if (s < e && *s == ',') s++;
        else if (s >= e) return fail(GP_E_PARSE, line, "unterminated arguments in %s", g->name);
      }
    }
    while (s < e) {
      while (s < e && (*s == ' ' || *s == '\t' || *s == '\r')) s++;
      if (s >= e) break;
      if (*s >= '0' && *s <= '9') {
        uint64_t v = 0;
        while (s < e && *s >= '0' && *s <= '9') {
          v = v * 10 + uint64_t(*s - '0');
          if (v > kMaxIndex) return fail(GP_E_BOUNDS, line, "target index too large in %s", g->name);
          s++;
        }
        if (s < e && *s != ' ' && *s != '\t' && *s != '\r')
          return fail(GP_E_UNSUPPORTED, line, "unsupported target in %s", g->name);
        c.targets.push_back(uint32_t(v));
        c.is_rec.push_back(0);
      } else if (e - s >= 6 && !std::strncmp(s, "rec[-", 5)) {
        s += 5;
        uint64_t v = 0;
        int nd = 0;
        while (s < e && *s >= '0' && *s <= '9') {
          v = v * 10 + uint64_t(*s - '0');
          if (v > kMaxIndex) return fail(GP_E_PARSE, line, "record offset too large in %s", g->name);
          s++;
          nd++;
        }
        if (!nd || s >= e || *s != ']' || v == 0) return fail(GP_E_PARSE, line, "bad record target in %s", g->name);
        s++;
        c.targets.push_back(uint32_t(v));
        c.is_rec.push_back(1);
      } else {
        return fail(GP_E_UNSUPPORTED, line, "unsupported target in %s", g->name);
      }
    }
    t.t1 = uint32_t(c.targets.size());
    const bool qubit_targets = g->cls != G_DET && g->cls != G_OBS && g->cls != G_IGNORE;
    if (qubit_targets) {
      for (uint32_t k = t.t0; k < t.t1; k++)
        if (c.is_rec[k]) return fail(GP_E_PARSE, line, "record target on %s", g->name);
      if (t.nargs && g->cls != G_N1 && g->cls != G_N2)
        return fail(GP_E_UNSUPPORTED, line, "arguments on %s are not supported", g->name);
    }
    c.toks.push_back(t);
  }
}

// Whole-line chunks of about equal size (at most kMaxTokChunks; one below
// kTokChunkMin bytes of text per chunk), tokenized on one thread per
// kTokThreadMin bytes of text, at most kMaxTokThreads, the scheduling thread
// included (texts lowered side by side, as a batch's or a server's, are
// mostly below that size and so start no threads of their own).
constexpr size_t kMaxTokThreads = 8;
constexpr size_t kTokThreadMin = 1 << 17;
constexpr size_t kMaxTokChunks = 64;
constexpr size_t kTokChunkMin = 1 << 15;
// The channel tables are built on up to this many threads, one per this many
// channels at least.
constexpr size_t kMaxChanThreads = 4;
constexpr size_t kChanChunkMin = 1 << 15;

double rate_limit(uint8_t kind) {
  return kind == CH_DEP1 ? 0.75 : kind == CH_DEP2 ? 15.0 / 16.0 : 0.5;
}



int set_err(LowerError& err, int code, int line, const char* fmt, const char* what) {
  char buf[256];
  std::snprintf(buf, sizeof buf, fmt, what);
  char full[320];
  if (line > 0)
    std::snprintf(full, sizeof full, "line %d: %s", line, buf);
  else
    std::snprintf(full, sizeof full, "%s", buf);
  err.code = code;
  err.msg = full;
  return code;
}

struct RawChan {
  uint32_t boundary, qa, qb;
  uint8_t kind;
  double rate;
};

}  // namespace

namespace {

// The program-order scheduling of one circuit, fed one elementary operation
// at a time by either front end (circuit text or the binary form): ASAP
// layers, measurement records, noise channels at their boundary, and the
// (measurement, detector-or-observable) memberships of the leaves (Eq. 2).
// Each call returns 0 or a GP_E_* status with a message in `msg`.
struct Sched {
  std::vector<uint32_t> ready;     // per qubit: the first layer it is free in
  std::vector<uint32_t> op_layer;
  std::vector<uint64_t> op_word;
  std::vector<RawChan> chans;
  std::vector<uint64_t> pairs;     // (measurement << 32) | detector index or kObsFlag | observable
  std::vector<uint32_t> meas_layer;
  std::vector<uint32_t> meas_qubit;  // per measurement: its qubit
  uint32_t n_meas = 0, n_det = 0, n_obs = 0;
  const char* msg = nullptr;

  int bad(int code, const char* m) {
    msg = m;
    return code;
  }
  int touch(uint32_t q) {
    if (q > kMaxIndex) return bad(GP_E_BOUNDS, "qubit index too large");
    if (q >= ready.size()) ready.resize(size_t(q) + 1, 0);
    return 0;
  }
  // a one-qubit gate or a reset
  int gate1(uint8_t kind, uint32_t q) {
    if (int rc = touch(q)) return rc;
    op_layer.push_back(ready[q]);
    op_word.push_back(pack_op(kind, q, 0));
    ready[q]++;
    return 0;
  }
  int gate2(uint8_t kind, uint32_t a, uint32_t b) {
    if (a == b) return bad(GP_E_PARSE, "repeated qubit in a two-qubit gate");
    if (int rc = touch(a)) return rc;
    if (int rc = touch(b)) return rc;
    const uint32_t l = std::max(ready[a], ready[b]);
    op_layer.push_back(l);
    op_word.push_back(pack_op(kind, a, b));
    ready[a] = ready[b] = l + 1;
    return 0;
  }
  int measure(uint8_t kind, uint32_t q) {
    if (int rc = touch(q)) return rc;
    if (n_meas > kMaxIndex) return bad(GP_E_BOUNDS, "too many measurements");
    op_layer.push_back(ready[q]);
    op_word.push_back(pack_op(kind, q, n_meas));
    meas_layer.push_back(ready[q]);
    meas_qubit.push_back(q);
    ready[q]++;
    n_meas++;
    return 0;
  }
  int noise1(uint8_t kind, uint32_t q, double r) {
    if (!(r >= 0.0 && r <= rate_limit(kind))) return bad(GP_E_NOISE, "rate out of range");
    if (int rc = touch(q)) return rc;
    chans.push_back(RawChan{ready[q], q, UINT32_MAX, kind, r});
    return 0;
  }
  int noise2(uint8_t kind, uint32_t a, uint32_t b, double r) {
    if (!(r >= 0.0 && r <= rate_limit(kind))) return bad(GP_E_NOISE, "rate out of range");
    if (a == b) return bad(GP_E_PARSE, "repeated qubit in a two-qubit channel");
    if (int rc = touch(a)) return rc;
    if (int rc = touch(b)) return rc;
    // both halves of the fault must sit at one boundary: later operations on
    // either qubit may not be scheduled before it
    const uint32_t bnd = std::max(ready[a], ready[b]);
    ready[a] = ready[b] = bnd;
    chans.push_back(RawChan{bnd, a, b, kind, r});
    return 0;
  }
  // a new detector / an observable's membership code
  int detector(uint32_t& code) {
    if (n_det >= kMaxIndex) return bad(GP_E_BOUNDS, "too many detectors");
    code = n_det++;
    return 0;
  }
  int observable(uint32_t k, uint32_t& code) {
    if (k > 65535) return bad(GP_E_PARSE, "observable index above 65535");
    n_obs = std::max(n_obs, k + 1);
    code = kObsFlag | k;
    return 0;
  }
  // measurement m (absolute, program order) belongs to `code`
  int member(uint32_t m, uint32_t code) {
    if (m >= n_meas) return bad(GP_E_PARSE, "record names a measurement that has not happened yet");
    pairs.push_back((uint64_t(m) << 32) | code);
    return 0;
  }
};

int finish_lowering(Sched& S, const double* rates, size_t n_rates, uint32_t sweep_slots, Lowered& lw,
                    LowerError& err, double fault_cost);

}  // namespace

void Lowered::reset() {
  // every field; the size check below fails when one is added, so that it is
  // added here too
  static_assert(sizeof(Lowered) == 960, "a field of Lowered is missing from reset()");
  n_qubits = n_layers = n_meas = n_det = n_obs = 0;
  wd = wo = w = 0;
  n_faults = 0;
  slab_words = 0;
  level = 2;
  bm_words = 0;
  w_max = 0;
  for (auto* v : {&layer_off, &leaf_off, &leaf_bits, &meas_layer, &chan_qa, &chan_qb, &chan_src, &chan_foff,
                  &bnd_chan_off, &bnd_fault_off, &item_col, &item_blo, &item_bhi, &ops32, &inj_off, &inj_layer,
                  &inj_qubit, &inj_next, &hchunk_pos, &hchunk_bnd, &layer_win, &win_lo, &win_obase, &win_cnt,
                  &bnd_bm_off, &item_branch, &hchunk_branch})
    v->clear();
  for (auto* v : {&ops, &col_base, &fnv_pow, &inj_word, &col_bm_base}) v->clear();
  col_top.clear();
  col_lo.clear();
  chan_kind.clear();
  chan_rate.clear();
  branches.clear();
}

int lower_circuit(const char* text, size_t len, const double* rates, size_t n_rates,
                  uint32_t sweep_slots, Lowered& lw, LowerError& err, uint32_t level, double fault_cost) {
  lw.reset();
  if (level > 2) return set_err(err, GP_E_ARG, 0, "%s", "correlation level must be 0, 1 or 2");
  if (!(fault_cost >= 0.0 && fault_cost < 1.0)) return set_err(err, GP_E_ARG, 0, "%s", "fault cost must be in [0, 1)");
  lw.level = level;
  Sched S;
  // sized from the text (typical circuits spend about four characters per
  // target) so that the vectors rarely regrow
  S.op_layer.reserve(len / 4);
  S.op_word.reserve(len / 4);
  S.chans.reserve(len / 8);
  S.pairs.reserve(len / 8);
  S.meas_layer.reserve(len / 8);
  S.meas_qubit.reserve(len / 8);

  // Tokenize whole-line chunks on up to kMaxTokThreads threads while this
  // thread schedules them (ASAP layers, measurement records, channels) in
  // program order: chunks are claimed in order from one counter, a chunk is
  // scheduled as soon as it is tokenized, and this thread tokenizes the next
  // unclaimed chunk itself while the one it needs is still being tokenized.
  const size_t n_chunks = std::max<size_t>(1, std::min(kMaxTokChunks, len / kTokChunkMin));
  std::vector<const char*> cut(n_chunks + 1, text + len);
  cut[0] = text;
  for (size_t k = 1; k < n_chunks; k++) {
    const char* c = text + len * k / n_chunks;
    if (c < cut[k - 1]) c = cut[k - 1];
    const char* nl = static_cast<const char*>(std::memchr(c, '\n', size_t(text + len - c)));
    cut[k] = nl ? nl + 1 : text + len;
  }
  std::vector<TokChunk> chunks(n_chunks);
  std::unique_ptr<std::atomic<uint8_t>[]> ready(new std::atomic<uint8_t>[n_chunks]);
  for (size_t k = 0; k < n_chunks; k++) ready[k].store(0, std::memory_order_relaxed);
  std::atomic<size_t> next_chunk{0};
  std::atomic<bool> stop{false};
  // tokenize the next unclaimed chunk; false once none is left or the
  // schedule has stopped on an error
  auto claim = [&]() -> bool {
    if (stop.load(std::memory_order_relaxed)) return false;
    const size_t k = next_chunk.fetch_add(1, std::memory_order_relaxed);
    if (k >= n_chunks) return false;
    tokenize(cut[k], cut[k + 1], chunks[k]);
    ready[k].store(1, std::memory_order_release);
    return true;
  };
  std::vector<std::thread> pool;
  // joins the tokenizer threads on every return below, before the chunks
  // they write go away
  struct Joiner {
    std::vector<std::thread>& pool;
    std::atomic<bool>& stop;
    ~Joiner() {
      stop.store(true, std::memory_order_relaxed);
      for (std::thread& th : pool) th.join();
    }
  } joiner{pool, stop};
  const size_t n_workers = std::min(std::min(kMaxTokThreads, std::max<size_t>(1, len / kTokThreadMin)), n_chunks) - 1;
  for (size_t w = 0; w < n_workers; w++) {
    try {
      pool.emplace_back([&claim] {
        while (claim()) {
        }
      });
    } catch (...) {
      break;  // could not start a thread: this thread claims the rest itself
    }
  }
  uint32_t line_base = 0;
  for (size_t ci = 0; ci < n_chunks; ci++) {
    while (!ready[ci].load(std::memory_order_acquire))
      if (!claim()) std::this_thread::yield();
    const TokChunk& ck = chunks[ci];
    for (const Tok& t : ck.toks) {
      const Gate* g = t.g;
      const int line = int(line_base + t.line);
      const size_t nt = t.t1 - t.t0;
      const uint32_t* targets = ck.targets.data() + t.t0;
      const uint8_t* is_rec = ck.is_rec.data() + t.t0;
      const char* name = g->name;
      int rc = 0;
      switch (g->cls) {
        case G_PAULI:
          for (size_t k = 0; k < nt && !rc; k++) rc = S.touch(targets[k]);
          break;
        case G_1Q:
        case G_RESET:
          for (size_t k = 0; k < nt && !rc; k++) rc = S.gate1(g->kind, targets[k]);
          break;
        case G_2Q:
          if (nt % 2) return set_err(err, GP_E_PARSE, line, "odd number of targets in %s", name);
          for (size_t k = 0; k < nt && !rc; k += 2) rc = S.gate2(g->kind, targets[k], targets[k + 1]);
          break;
        case G_MEAS:
          for (size_t k = 0; k < nt && !rc; k++) rc = S.measure(g->kind, targets[k]);
          break;
        case G_N1:
        case G_N2: {
          if (t.nargs != 1) return set_err(err, GP_E_PARSE, line, "%s takes one probability", name);
          const double r = t.arg0;
          if (!(r >= 0.0 && r <= rate_limit(g->kind)))
            return set_err(err, GP_E_NOISE, line, "rate out of range in %s", name);
          if (g->cls == G_N1) {
            for (size_t k = 0; k < nt && !rc; k++) rc = S.noise1(g->kind, targets[k], r);
          } else {
            if (nt % 2) return set_err(err, GP_E_PARSE, line, "odd number of targets in %s", name);
            for (size_t k = 0; k < nt && !rc; k += 2) rc = S.noise2(g->kind, targets[k], targets[k + 1], r);
          }
          break;
        }
        case G_DET:
        case G_OBS: {
          uint32_t code = 0;
          if (g->cls == G_DET) {
            rc = S.detector(code);
          } else {
            if (t.nargs != 1 || t.arg0 < 0 || t.arg0 != std::floor(t.arg0) || t.arg0 > 65535)
              return set_err(err, GP_E_PARSE, line, "%s needs one observable index", name);
            rc = S.observable(uint32_t(t.arg0), code);
          }
          for (size_t k = 0; k < nt && !rc; k++) {
            if (!is_rec[k]) return set_err(err, GP_E_PARSE, line, "%s takes record targets", name);
            if (targets[k] > S.n_meas) return set_err(err, GP_E_PARSE, line, "record looks back too far in %s", name);
            rc = S.member(S.n_meas - targets[k], code);
          }
          break;
        }
        default:
          break;
      }
      if (rc) return set_err(err, rc, line, "%s", S.msg);
    }
    if (ck.err_code) return set_err(err, ck.err_code, int(line_base + ck.err_line), ck.err_fmt, ck.err_what.c_str());
    line_base += ck.lines;
  }
  return finish_lowering(S, rates, n_rates, sweep_slots, lw, err, fault_cost);
}

int lower_ir(const gp_circuit_ir& ir, const double* rates, size_t n_rates, uint32_t sweep_slots, Lowered& lw,
             LowerError& err, uint32_t level, double fault_cost) {
  lw.reset();
  if (level > 2) return set_err(err, GP_E_ARG, 0, "%s", "correlation level must be 0, 1 or 2");
  if (!(fault_cost >= 0.0 && fault_cost < 1.0)) return set_err(err, GP_E_ARG, 0, "%s", "fault cost must be in [0, 1)");
  if (ir.n_ops && !ir.code) return set_err(err, GP_E_ARG, 0, "%s", "operation codes missing");
  lw.level = level;
  Sched S;
  // upper bounds, so that the vectors never regrow (untouched capacity costs
  // no memory traffic)
  S.op_layer.reserve(ir.n_ops);
  S.op_word.reserve(ir.n_ops);
  S.chans.reserve(ir.n_ops);
  S.meas_layer.reserve(ir.n_ops);
  S.meas_qubit.reserve(ir.n_ops);
  S.pairs.reserve(ir.n_rec);
  uint64_t ri = 0;  // next entry of ir.rec
  char buf[160];
  auto op_err = [&](uint64_t k, int code, const char* what) {
    std::snprintf(buf, sizeof buf, "operation %llu: %s", (unsigned long long)k, what);
    return set_err(err, code, 0, "%s", buf);
  };
  for (uint64_t k = 0; k < ir.n_ops; k++) {
    const uint8_t c = ir.code[k];
    const bool needs_q0 = c != GP_IR_DETECTOR;
    const bool needs_q1 = c == GP_IR_CX || c == GP_IR_CZ || c == GP_IR_SWAP || c == GP_IR_DEPOLARIZE2 ||
                          c == GP_IR_DETECTOR || c == GP_IR_OBSERVABLE;
    const bool needs_rate = c >= GP_IR_X_ERROR && c <= GP_IR_DEPOLARIZE2;
    if ((needs_q0 && !ir.q0) || (needs_q1 && !ir.q1) || (needs_rate && !ir.rate))
      return op_err(k, GP_E_ARG, "an array this operation needs is missing");
    int rc = 0;
    switch (c) {
      case GP_IR_PAULI: rc = S.touch(ir.q0[k]); break;
      case GP_IR_H: rc = S.gate1(OP_H, ir.q0[k]); break;
      case GP_IR_S: rc = S.gate1(OP_S, ir.q0[k]); break;
      case GP_IR_SQRT_X: rc = S.gate1(OP_SQRTX, ir.q0[k]); break;
      case GP_IR_R: rc = S.gate1(OP_R, ir.q0[k]); break;
      case GP_IR_RX: rc = S.gate1(OP_RX, ir.q0[k]); break;
      case GP_IR_CX: rc = S.gate2(OP_CX, ir.q0[k], ir.q1[k]); break;
      case GP_IR_CZ: rc = S.gate2(OP_CZ, ir.q0[k], ir.q1[k]); break;
      case GP_IR_SWAP: rc = S.gate2(OP_SWAP, ir.q0[k], ir.q1[k]); break;
      case GP_IR_M: rc = S.measure(OP_M, ir.q0[k]); break;
      case GP_IR_MX: rc = S.measure(OP_MX, ir.q0[k]); break;
      case GP_IR_MR: rc = S.measure(OP_MR, ir.q0[k]); break;
      case GP_IR_MRX: rc = S.measure(OP_MRX, ir.q0[k]); break;
      case GP_IR_X_ERROR: rc = S.noise1(CH_X, ir.q0[k], ir.rate[k]); break;
      case GP_IR_Y_ERROR: rc = S.noise1(CH_Y, ir.q0[k], ir.rate[k]); break;
      case GP_IR_Z_ERROR: rc = S.noise1(CH_Z, ir.q0[k], ir.rate[k]); break;
      case GP_IR_DEPOLARIZE1: rc = S.noise1(CH_DEP1, ir.q0[k], ir.rate[k]); break;
      case GP_IR_DEPOLARIZE2: rc = S.noise2(CH_DEP2, ir.q0[k], ir.q1[k], ir.rate[k]); break;
      case GP_IR_DETECTOR:
      case GP_IR_OBSERVABLE: {
        uint32_t code = 0;
        rc = c == GP_IR_DETECTOR ? S.detector(code) : S.observable(ir.q0[k], code);
        const uint64_t n = ir.q1[k];
        if (!rc && n && !ir.rec) return op_err(k, GP_E_ARG, "record array missing");
        if (!rc && ri + n > ir.n_rec) return op_err(k, GP_E_ARG, "records run past the record array");
        for (uint64_t j = 0; j < n && !rc; j++) rc = S.member(ir.rec[ri + j], code);
        ri += n;
        break;
      }
      default:
        return op_err(k, GP_E_UNSUPPORTED, "unknown operation code");
    }
    if (rc) return op_err(k, rc, S.msg);
  }
  if (ri != ir.n_rec) return set_err(err, GP_E_ARG, 0, "%s", "record array longer than the annotations use");
  return finish_lowering(S, rates, n_rates, sweep_slots, lw, err, fault_cost);
}

namespace {

// Everything after the program-order pass: channel and fault tables, layers,
// leaves, word columns, sweep items, windows and hash chunks.
int finish_lowering(Sched& S, const double* rates, size_t n_rates, uint32_t sweep_slots, Lowered& lw,
                    LowerError& err, double fault_cost) {
  std::vector<uint32_t>& ready = S.ready;
  std::vector<uint32_t>& op_layer = S.op_layer;
  std::vector<uint64_t>& op_word = S.op_word;
  std::vector<RawChan>& chans = S.chans;
  std::vector<uint64_t>& pairs = S.pairs;
  const uint32_t n_meas = S.n_meas, n_det = S.n_det, n_obs = S.n_obs;
  lw.meas_layer.swap(S.meas_layer);

  // ---- sizes
  lw.n_qubits = uint32_t(ready.size());
  uint32_t L = 0;
  for (uint32_t r : ready) L = std::max(L, r);
  lw.n_layers = L;
  lw.n_meas = n_meas;
  lw.n_det = n_det;
  lw.n_obs = n_obs;
  lw.wd = (n_det + 63) / 64;
  lw.wo = (n_obs + 63) / 64;
  lw.w = lw.wd + lw.wo;

  // ---- channels sorted by boundary (stable), fault positions; on a second
  // thread for large circuits, beside the op sort and the leaves
  auto channel_phase = [&](LowerError& e) -> int {
    const size_t C = chans.size();
    if (rates) {
      if (n_rates != C) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "rate array has %zu entries, circuit has %zu channels", n_rates, C);
        return set_err(e, GP_E_NOISE, 0, "%s", buf);
      }
      for (size_t k = 0; k < C; k++) {
        double r = rates[k];
        if (!(r >= 0.0 && r <= rate_limit(chans[k].kind))) return set_err(e, GP_E_NOISE, 0, "%s", "rate out of range");
        chans[k].rate = r;
      }
    }
    lw.chan_qa.resize(C);
    lw.chan_qb.resize(C);
    lw.chan_kind.resize(C);
    lw.chan_rate.resize(C);
    lw.chan_src.resize(C);
    // stable counting sort by boundary; large circuits split the channels
    // over a few threads (per-thread boundary counts, one prefix over
    // (boundary, thread), then each thread scatters its own range)
    const size_t T = std::max<size_t>(1, std::min<size_t>(kMaxChanThreads, C / kChanChunkMin));
    const size_t nb = size_t(L) + 1;
    std::vector<uint32_t> cnt(T * nb, 0);
    auto part = [&](size_t t) { return std::make_pair(C * t / T, C * (t + 1) / T); };
    auto count = [&](size_t t) {
      uint32_t* c = cnt.data() + t * nb;
      const auto r = part(t);
      for (size_t k = r.first; k < r.second; k++) c[chans[k].boundary]++;
    };
    auto scatter = [&](size_t t) {
      uint32_t* f = cnt.data() + t * nb;
      const auto r = part(t);
      for (size_t k = r.first; k < r.second; k++) {
        const uint32_t d = f[chans[k].boundary]++;
        lw.chan_qa[d] = chans[k].qa;
        lw.chan_qb[d] = chans[k].qb;
        lw.chan_kind[d] = chans[k].kind;
        lw.chan_rate[d] = chans[k].rate;
        lw.chan_src[d] = uint32_t(k);
      }
    };
    auto on_threads = [&](auto&& fn) {
      std::vector<std::thread> pool;
      for (size_t t = 1; t < T; t++) {
        try {
          pool.emplace_back(fn, t);
        } catch (...) {
          fn(t);  // could not start a thread: do its part here
        }
      }
      fn(size_t(0));
      for (std::thread& th : pool) th.join();
    };
    on_threads(count);
    lw.bnd_chan_off.assign(size_t(L) + 2, 0);
    {
      uint32_t run = 0;
      for (size_t b = 0; b < nb; b++) {
        lw.bnd_chan_off[b] = run;
        for (size_t t = 0; t < T; t++) {
          const uint32_t x = cnt[t * nb + b];
          cnt[t * nb + b] = run;
          run += x;
        }
      }
      lw.bnd_chan_off[nb] = run;
    }
    on_threads(scatter);
    uint64_t total_faults = 0;
    for (size_t c = 0; c < C; c++) total_faults += kKeptCodes.n[lw.chan_kind[c]][lw.level];
    if (total_faults >= (1ull << 32)) return set_err(e, GP_E_BOUNDS, 0, "%s", "more than 2^32 - 1 faults");
    lw.chan_foff.assign(C + 1, 0);
    for (size_t c = 0; c < C; c++) lw.chan_foff[c + 1] = lw.chan_foff[c] + kKeptCodes.n[lw.chan_kind[c]][lw.level];
    lw.n_faults = total_faults;
    lw.bnd_fault_off.assign(size_t(L) + 2, 0);
    for (uint32_t b = 0; b <= L + 1; b++) lw.bnd_fault_off[b] = lw.chan_foff[lw.bnd_chan_off[b]];
    return 0;
  };
  LowerError ch_err{};
  int ch_rc = 0;
  const bool two_threads = chans.size() + op_word.size() > (size_t(1) << 16);
  std::thread ch_thread;
  bool ch_done = false;
  // the phases on other threads may not throw: an allocation failure there
  // becomes their status
  auto channel_phase_safe = [&]() {
    try {
      ch_rc = channel_phase(ch_err);
    } catch (...) {
      ch_rc = set_err(ch_err, GP_E_OOM, 0, "%s", "host memory allocation failed while lowering");
    }
  };
  if (two_threads) {
    try {
      ch_thread = std::thread(channel_phase_safe);
    } catch (...) {
      channel_phase_safe();  // could not start a thread: build the channel tables here
      ch_done = true;
    }
  }
  // joined on every way out of this function, exceptions included
  struct Joiner {
    std::thread& t;
    ~Joiner() {
      if (t.joinable()) t.join();
    }
  } ch_join{ch_thread};

  // ---- operations sorted by layer (counting sort keeps program order)
  lw.layer_off.assign(size_t(L) + 1, 0);
  for (uint32_t l : op_layer) lw.layer_off[l + 1]++;
  for (uint32_t l = 0; l < L; l++) lw.layer_off[l + 1] += lw.layer_off[l];
  lw.ops.resize(op_word.size());
  {
    std::vector<uint32_t> fill(lw.layer_off.begin(), lw.layer_off.end() - 1);
    for (size_t k = 0; k < op_word.size(); k++) lw.ops[fill[op_layer[k]]++] = op_word[k];
  }

  // ---- leaves (Eq. 2), XOR semantics for repeated memberships
  {
    // (measurement, code) pairs in ascending order: a counting sort by
    // measurement, then each measurement's few codes sorted
    std::vector<uint32_t> cnt(size_t(n_meas) + 1, 0);
    for (uint64_t pr : pairs) cnt[(pr >> 32) + 1]++;
    for (uint32_t m = 0; m < n_meas; m++) cnt[m + 1] += cnt[m];
    std::vector<uint64_t> sorted(pairs.size());
    std::vector<uint32_t> fill(cnt.begin(), cnt.end() - 1);
    for (uint64_t pr : pairs) sorted[fill[pr >> 32]++] = pr;
    for (uint32_t m = 0; m < n_meas; m++)
      if (cnt[m + 1] - cnt[m] > 1) std::sort(sorted.begin() + cnt[m], sorted.begin() + cnt[m + 1]);
    pairs.swap(sorted);
  }
  lw.leaf_off.assign(size_t(n_meas) + 1, 0);
  lw.leaf_bits.clear();
  for (size_t i = 0; i < pairs.size();) {
    size_t j = i;
    while (j < pairs.size() && pairs[j] == pairs[i]) j++;
    if ((j - i) & 1) {
      uint32_t m = uint32_t(pairs[i] >> 32);
      uint32_t code = uint32_t(pairs[i]);
      uint32_t bit = (code & kObsFlag) ? lw.wd * 64 + (code & ~kObsFlag) : code;
      lw.leaf_off[m + 1]++;
      lw.leaf_bits.push_back(bit);
    }
    i = j;
  }
  for (uint32_t m = 0; m < n_meas; m++) lw.leaf_off[m + 1] += lw.leaf_off[m];

  if (ch_thread.joinable()) ch_thread.join();
  else if (!ch_done) ch_rc = channel_phase(ch_err);
  if (ch_rc) {
    err = ch_err;
    return ch_rc;
  }

  // ---- word columns: static live range from the layers of their leaves
  lw.col_top.assign(lw.w, -1);
  lw.col_lo.assign(lw.w, INT32_MAX);
  for (uint32_t m = 0; m < n_meas; m++) {
    for (uint32_t k = lw.leaf_off[m]; k < lw.leaf_off[m + 1]; k++) {
      uint32_t w = lw.leaf_bits[k] >> 6;
      lw.col_top[w] = std::max<int32_t>(lw.col_top[w], int32_t(lw.meas_layer[m]));
      lw.col_lo[w] = std::min<int32_t>(lw.col_lo[w], int32_t(lw.meas_layer[m]));
    }
  }
  lw.col_base.assign(lw.w, 0);
  uint64_t base = 0;
  for (uint32_t w = 0; w < lw.w; w++) {
    lw.col_base[w] = base;
    if (lw.col_top[w] >= 0) base += lw.bnd_fault_off[lw.col_top[w] + 1];
    else lw.col_lo[w] = -1;
  }
  lw.slab_words = base;
  lw.bnd_bm_off.assign(size_t(L) + 2, 0);
  for (uint32_t b = 0; b <= L; b++)
    lw.bnd_bm_off[b + 1] = lw.bnd_bm_off[b] + (lw.bnd_fault_off[b + 1] - lw.bnd_fault_off[b] + 63) / 64;
  lw.col_bm_base.assign(lw.w, 0);
  uint64_t bm = 0;
  for (uint32_t w = 0; w < lw.w; w++) {
    lw.col_bm_base[w] = bm;
    if (lw.col_top[w] >= 0) bm += lw.bnd_bm_off[lw.col_top[w] + 1];
  }
  lw.bm_words = bm;

  // ---- per-column leaf injections, top layer first (on a second thread for
  // large circuits, beside the items, windows and compact ops)
  auto injection_phase = [&]() {
    {
      const std::vector<uint32_t>& meas_qubit = S.meas_qubit;
      // one entry per (measurement, column) that the measurement's leaves
      // hit; a measurement's leaf bits ascend, so those of one column are
      // adjacent. Counted per column, then placed straight into the tables.
      lw.inj_off.assign(size_t(lw.w) + 1, 0);
      for (uint32_t m = 0; m < n_meas; m++)
        for (uint32_t k = lw.leaf_off[m]; k < lw.leaf_off[m + 1]; k++)
          if (k == lw.leaf_off[m] || (lw.leaf_bits[k] >> 6) != (lw.leaf_bits[k - 1] >> 6))
            lw.inj_off[(lw.leaf_bits[k] >> 6) + 1]++;
      for (uint32_t w = 0; w < lw.w; w++) lw.inj_off[w + 1] += lw.inj_off[w];
      const size_t n_inj = lw.inj_off[lw.w];
      lw.inj_layer.resize(n_inj);
      lw.inj_qubit.resize(n_inj);
      lw.inj_word.resize(n_inj);
      // placed in descending measurement order, which lists a column top
      // layer first wherever its measurements come in layer order
      std::vector<uint32_t> fill(lw.inj_off.begin(), lw.inj_off.end() - 1);
      for (uint32_t m = n_meas; m-- > 0;) {
        for (uint32_t k = lw.leaf_off[m], e = lw.leaf_off[m + 1]; k < e;) {
          const uint32_t w = lw.leaf_bits[k] >> 6;
          uint64_t word = 0;
          for (; k < e && (lw.leaf_bits[k] >> 6) == w; k++) word |= 1ull << (lw.leaf_bits[k] & 63);
          const uint32_t pos = fill[w]++;
          lw.inj_layer[pos] = lw.meas_layer[m];
          lw.inj_qubit[pos] = meas_qubit[m];
          lw.inj_word[pos] = word;
        }
      }
      // within each column: top layer first, the entries of one layer in
      // measurement order (a stable sort by layer where the column is not in
      // layer order already, then each run of one layer reversed)
      std::vector<uint32_t> perm;
      std::vector<uint32_t> tmp32;
      std::vector<uint64_t> tmp64;
      for (uint32_t w = 0; w < lw.w; w++) {
        const uint32_t a = lw.inj_off[w], e = lw.inj_off[w + 1];
        uint32_t* layer = lw.inj_layer.data();
        if (!std::is_sorted(layer + a, layer + e, [](uint32_t x, uint32_t y) { return x > y; })) {
          perm.resize(e - a);
          for (uint32_t i = 0; i < e - a; i++) perm[i] = a + i;
          std::stable_sort(perm.begin(), perm.end(), [&](uint32_t x, uint32_t y) { return layer[x] > layer[y]; });
          auto gather32 = [&](std::vector<uint32_t>& v) {
            tmp32.resize(e - a);
            for (uint32_t i = 0; i < e - a; i++) tmp32[i] = v[perm[i]];
            std::copy(tmp32.begin(), tmp32.end(), v.begin() + a);
          };
          gather32(lw.inj_layer);
          gather32(lw.inj_qubit);
          tmp64.resize(e - a);
          for (uint32_t i = 0; i < e - a; i++) tmp64[i] = lw.inj_word[perm[i]];
          std::copy(tmp64.begin(), tmp64.end(), lw.inj_word.begin() + a);
        }
        for (uint32_t r = a; r < e;) {
          uint32_t q = r + 1;
          while (q < e && layer[q] == layer[r]) q++;
          std::reverse(lw.inj_qubit.begin() + r, lw.inj_qubit.begin() + q);
          std::reverse(lw.inj_word.begin() + r, lw.inj_word.begin() + q);
          r = q;
        }
      }
      lw.inj_next.resize(n_inj);
      for (uint32_t w = 0; w < lw.w; w++) {
        const uint32_t a = lw.inj_off[w], e = lw.inj_off[w + 1];
        uint32_t next = e - a;
        for (uint32_t k = e; k-- > a;) {
          if (k + 1 < e && lw.inj_layer[k + 1] != lw.inj_layer[k]) next = k + 1 - a;
          lw.inj_next[k] = next;
        }
      }
    }
  };
  bool inj_oom = false;
  auto injection_phase_safe = [&]() {
    try {
      injection_phase();
    } catch (...) {
      inj_oom = true;
    }
  };
  std::thread inj_thread;
  if (two_threads) {
    try {
      inj_thread = std::thread(injection_phase_safe);
    } catch (...) {
      injection_phase_safe();  // could not start a thread: build the lists here
    }
  } else {
    injection_phase_safe();
  }
  Joiner inj_join{inj_thread};

  // ---- sweep items: one per detector column; observable columns, which stay
  // live over the whole circuit, are cut into boundary ranges so that their
  // emission spreads over the slots left after the detector columns (one
  // slot = one CU running one item). Each range re-sweeps from the column's
  // top, so the lowest ranges run longest; they are listed first so that
  // they start first.
  {
    uint32_t n_det_items = 0, n_obs_live = 0;
    for (uint32_t w = 0; w < lw.w; w++)
      if (lw.col_top[w] >= 0) (w < lw.wd ? n_det_items : n_obs_live)++;
    const uint32_t slots = std::max<uint32_t>(sweep_slots, 1);
    const uint32_t per_obs =
        n_obs_live && slots > n_det_items ? std::max<uint32_t>((slots - n_det_items) / n_obs_live, 1) : 1;
    // A range [lo, hi] costs (top - hi) transform-only layers plus its own
    // layers with their faults (relative weights of a transform-only layer
    // and of one emitted fault, measured on gfx950). Every range re-sweeps
    // from the top, so the lowest ranges get few boundaries and the upper
    // ones many: the smallest makespan T that the greedy cut from the
    // bottom fits into per_obs ranges is found by bisection.
    constexpr double kLayerCost = 1.0;
    const double kFaultCost = fault_cost > 0 ? fault_cost : kDefaultFaultCost;
    for (uint32_t w = lw.wd; w < lw.w; w++) {
      const int32_t top = lw.col_top[w];
      if (top < 0) continue;
      auto emit_cost = [&](int32_t t) {
        return kLayerCost + kFaultCost * double(lw.bnd_fault_off[t + 1] - lw.bnd_fault_off[t]);
      };
      // greedy cut for makespan T: ranges from the bottom up, or empty if a
      // range would exceed per_obs
      auto cut = [&](double T, std::vector<std::pair<uint32_t, uint32_t>>& out) {
        out.clear();
        int32_t lo = 0;
        while (lo <= top) {
          if (out.size() == per_obs) return false;
          double c = kLayerCost * double(top - lo) + emit_cost(lo);
          int32_t hi = lo;
          while (hi < top) {
            const double nc = c - kLayerCost + emit_cost(hi + 1);
            if (nc > T) break;
            c = nc;
            hi++;
          }
          out.emplace_back(uint32_t(lo), uint32_t(hi));
          lo = hi + 1;
        }
        return true;
      };
      double total = 0;
      for (int32_t t = 0; t <= top; t++) total += emit_cost(t);
      double lo_T = 0, hi_T = total + kLayerCost * double(top + 1);
      std::vector<std::pair<uint32_t, uint32_t>> ranges;
      for (int it = 0; it < 60; it++) {
        const double mid = 0.5 * (lo_T + hi_T);
        if (cut(mid, ranges)) hi_T = mid;
        else lo_T = mid;
      }
      cut(hi_T, ranges);
      // ranges are bottom-up: the lowest (longest-running) first
      for (const auto& r : ranges) {
        lw.item_col.push_back(w);
        lw.item_blo.push_back(r.first);
        lw.item_bhi.push_back(r.second);
      }
    }
  }
  for (uint32_t w = 0; w < lw.wd; w++) {
    if (lw.col_top[w] < 0) continue;
    lw.item_col.push_back(w);
    lw.item_blo.push_back(0);
    lw.item_bhi.push_back(uint32_t(lw.col_top[w]));
  }

  // ---- op windows (a layer has at most n ops; the driver rejects circuits
  // whose largest layer exceeds a window). A circuit of a batch (fewer sweep
  // slots than the device has) with at most kSmallWinOps qubits gets windows
  // the 256-thread sweep holds; a circuit lowered alone runs on the
  // 1024-thread sweep, whose larger windows mean fewer window swaps on the
  // layer chain.
  lw.layer_win.assign(L, 0);
  const uint32_t win_ops =
      (lw.n_qubits <= kSmallWinOps && sweep_slots < kSweepSlots) ? kSmallWinOps : kSweepWinOps;
  for (int32_t hi = int32_t(L) - 1; hi >= 0;) {
    int32_t lo = hi;
    while (lo > 0 && lw.layer_off[hi + 1] - lw.layer_off[lo - 1] <= win_ops) lo--;
    const uint32_t id = uint32_t(lw.win_lo.size());
    lw.win_lo.push_back(uint32_t(lo));
    lw.win_obase.push_back(lw.layer_off[lo]);
    lw.win_cnt.push_back(lw.layer_off[hi + 1] - lw.layer_off[lo]);
    for (int32_t t = lo; t <= hi; t++) lw.layer_win[t] = id;
    hi = lo - 1;
  }

  // ---- compact sweep ops (qubit indices must fit the compact word)
  lw.ops32.resize(lw.ops.size());
  for (size_t k = 0; k < lw.ops.size(); k++) {
    const uint64_t op = lw.ops[k];
    const uint32_t kind = uint32_t(op >> 56), a = uint32_t(op >> 28) & kField, b = uint32_t(op) & kField;
    const bool two = kind == OP_CX || kind == OP_CZ || kind == OP_SWAP;
    lw.ops32[k] = (a < kMaxSweepQubits && (!two || b < kMaxSweepQubits)) ? pack_op32(kind, a, two ? b : 0)
                                                                         : 0xFFFFFFFFu;
  }

  // ---- hash chunks: 256 positions of one boundary at most
  for (uint32_t b = 0; b <= L; b++)
    for (uint32_t p0 = lw.bnd_fault_off[b]; p0 < lw.bnd_fault_off[b + 1]; p0 += 256) {
      lw.hchunk_pos.push_back(p0);
      lw.hchunk_bnd.push_back(b);
    }

  // ---- FNV-1a over the 8W octets of a signature: a run of k zero words
  // multiplies the state by prime^(8k)
  uint64_t p8 = 1;
  for (int k = 0; k < 8; k++) p8 *= kFnvPrime;
  lw.fnv_pow.assign(size_t(lw.w) + 1, 1);
  for (uint32_t k = 1; k <= lw.w; k++) lw.fnv_pow[k] = lw.fnv_pow[k - 1] * p8;
  // a single circuit is a batch of one
  lw.w_max = lw.w;
  BranchDesc bd{};
  bd.n_qubits = lw.n_qubits;
  bd.n_layers = lw.n_layers;
  bd.lob = 0;
  bd.bb = 0;
  bd.wb = 0;
  bd.nw = lw.w;
  bd.wd = lw.wd;
  bd.n_det = lw.n_det;
  bd.n_obs = lw.n_obs;
  bd.wib = 0;
  bd.n_win = uint32_t(lw.win_lo.size());
  bd.fb = 0;
  bd.fe = uint32_t(lw.n_faults);
  lw.branches.assign(1, bd);
  lw.item_branch.assign(lw.item_col.size(), 0);
  lw.hchunk_branch.assign(lw.hchunk_pos.size(), 0);
  // layer windows share the layer-offset indexing (n_layers + 1 entries)
  lw.layer_win.resize(size_t(lw.n_layers) + 1, 0);
  if (inj_thread.joinable()) inj_thread.join();
  if (inj_oom) return set_err(err, GP_E_OOM, 0, "%s", "host memory allocation failed while lowering");
  return 0;
}

}  // namespace

void merge_branches(const std::vector<Lowered>& in, Lowered& out) {
  std::vector<const Lowered*> ptrs;
  for (const Lowered& a : in) ptrs.push_back(&a);
  merge_branches(ptrs, out);
}

namespace {

template <typename T>
void append(std::vector<T>& dst, const std::vector<T>& src) {
  dst.insert(dst.end(), src.begin(), src.end());
}

template <typename T, typename U>
void append_plus(std::vector<T>& dst, const std::vector<T>& src, U add) {
  const size_t n0 = dst.size();
  dst.resize(n0 + src.size());
  T* o = dst.data() + n0;
  for (size_t i = 0; i < src.size(); i++) o[i] = T(src[i] + add);
}

}  // namespace

void merge_branches(const std::vector<const Lowered*>& in, Lowered& out) {
  out = Lowered();
  // every table is sized once, then filled by bulk appends
  size_t n_ops = 0, n_lay = 0, n_leafo = 0, n_leaf = 0, n_meas = 0, n_ch = 0, n_bnd = 0, n_col = 0, n_inj = 0,
         n_item = 0, n_hc = 0, n_win = 0;
  for (const Lowered* a : in) {
    n_ops += a->ops.size();
    n_lay += a->layer_off.size();
    n_leafo += a->leaf_off.size();
    n_leaf += a->leaf_bits.size();
    n_meas += a->meas_layer.size();
    n_ch += a->chan_kind.size();
    n_bnd += a->bnd_fault_off.size();
    n_col += a->w;
    n_inj += a->inj_layer.size();
    n_item += a->item_col.size();
    n_hc += a->hchunk_pos.size();
    n_win += a->win_lo.size();
  }
  out.ops.reserve(n_ops);
  out.ops32.reserve(n_ops);
  out.layer_off.reserve(n_lay);
  out.layer_win.reserve(n_lay);
  out.leaf_off.reserve(n_leafo);
  out.leaf_bits.reserve(n_leaf);
  out.meas_layer.reserve(n_meas);
  for (auto* v : {&out.chan_qa, &out.chan_qb, &out.chan_src}) v->reserve(n_ch);
  out.chan_kind.reserve(n_ch);
  out.chan_rate.reserve(n_ch);
  out.chan_foff.reserve(n_ch + 1);
  for (auto* v : {&out.bnd_chan_off, &out.bnd_fault_off, &out.bnd_bm_off}) v->reserve(n_bnd);
  out.col_top.reserve(n_col);
  out.col_lo.reserve(n_col);
  out.col_base.reserve(n_col);
  out.col_bm_base.reserve(n_col);
  out.inj_off.reserve(n_col + 1);
  for (auto* v : {&out.inj_layer, &out.inj_qubit, &out.inj_next}) v->reserve(n_inj);
  out.inj_word.reserve(n_inj);
  for (auto* v : {&out.item_col, &out.item_blo, &out.item_bhi, &out.item_branch}) v->reserve(n_item);
  for (auto* v : {&out.hchunk_pos, &out.hchunk_bnd, &out.hchunk_branch}) v->reserve(n_hc);
  for (auto* v : {&out.win_lo, &out.win_obase, &out.win_cnt}) v->reserve(n_win);
  out.branches.reserve(in.size());

  uint32_t ob = 0, cb = 0, fb = 0, wb = 0, ib = 0, wib = 0, mb = 0;
  uint64_t sb = 0, bmb = 0;
  std::vector<uint32_t> item_order_span;
  item_order_span.reserve(n_item);
  for (size_t k = 0; k < in.size(); k++) {
    const Lowered& a = *in[k];
    out.n_qubits = std::max(out.n_qubits, a.n_qubits);
    out.n_layers = std::max(out.n_layers, a.n_layers);
    out.n_det = std::max(out.n_det, a.n_det);
    out.n_obs = std::max(out.n_obs, a.n_obs);
    out.w_max = std::max(out.w_max, a.w);
    out.level = a.level;
    BranchDesc bd{};
    bd.n_qubits = a.n_qubits;
    bd.n_layers = a.n_layers;
    bd.lob = uint32_t(out.layer_off.size());
    bd.bb = uint32_t(out.bnd_fault_off.size());
    bd.wb = wb;
    bd.nw = a.w;
    bd.wd = a.wd;
    bd.n_det = a.n_det;
    bd.n_obs = a.n_obs;
    bd.wib = wib;
    bd.n_win = uint32_t(a.win_lo.size());
    bd.fb = fb;
    bd.fe = fb + uint32_t(a.n_faults);
    out.branches.push_back(bd);
    append(out.ops, a.ops);
    append(out.ops32, a.ops32);
    append_plus(out.layer_off, a.layer_off, ob);
    append(out.layer_win, a.layer_win);
    append(out.leaf_off, a.leaf_off);
    append(out.leaf_bits, a.leaf_bits);
    append(out.meas_layer, a.meas_layer);
    append(out.chan_qa, a.chan_qa);
    append(out.chan_qb, a.chan_qb);
    append(out.chan_kind, a.chan_kind);
    append(out.chan_rate, a.chan_rate);
    append_plus(out.chan_src, a.chan_src, cb);
    {
      // chan_foff holds C + 1 entries per circuit; the batch keeps one closing entry
      const size_t C = a.chan_kind.size();
      const size_t n0 = out.chan_foff.size();
      out.chan_foff.resize(n0 + C);
      for (size_t c = 0; c < C; c++) out.chan_foff[n0 + c] = a.chan_foff[c] + fb;
    }
    append_plus(out.bnd_chan_off, a.bnd_chan_off, cb);
    append_plus(out.bnd_fault_off, a.bnd_fault_off, fb);
    append(out.bnd_bm_off, a.bnd_bm_off);
    // slab words are addressed by base + (batch) fault position: the circuit's
    // slab starts at sb >= fb, so its bases (sb - fb + own base) stay >= 0
    sb = std::max<uint64_t>(sb, fb);
    append(out.col_top, a.col_top);
    append(out.col_lo, a.col_lo);
    append_plus(out.col_base, a.col_base, sb - fb);
    append_plus(out.col_bm_base, a.col_bm_base, bmb);
    {
      const size_t n0 = out.inj_off.size();
      out.inj_off.resize(n0 + a.w);
      for (uint32_t w = 0; w < a.w; w++) out.inj_off[n0 + w] = a.inj_off[w] + ib;
    }
    append(out.inj_layer, a.inj_layer);
    append(out.inj_qubit, a.inj_qubit);
    append(out.inj_word, a.inj_word);
    append(out.inj_next, a.inj_next);
    append_plus(out.item_col, a.item_col, wb);
    append(out.item_blo, a.item_blo);
    append(out.item_bhi, a.item_bhi);
    out.item_branch.resize(out.item_branch.size() + a.item_col.size(), uint32_t(k));
    for (size_t t = 0; t < a.item_col.size(); t++)
      item_order_span.push_back(uint32_t(a.col_top[a.item_col[t]] - int32_t(a.item_blo[t]) + 1));
    append_plus(out.hchunk_pos, a.hchunk_pos, fb);
    append(out.hchunk_bnd, a.hchunk_bnd);
    out.hchunk_branch.resize(out.hchunk_branch.size() + a.hchunk_pos.size(), uint32_t(k));
    append(out.win_lo, a.win_lo);
    append_plus(out.win_obase, a.win_obase, ob);
    append(out.win_cnt, a.win_cnt);
    if (a.fnv_pow.size() > out.fnv_pow.size()) out.fnv_pow = a.fnv_pow;
    ob += uint32_t(a.ops32.size());
    cb += uint32_t(a.chan_kind.size());
    fb += uint32_t(a.n_faults);
    wb += a.w;
    ib += uint32_t(a.inj_layer.size());
    wib += uint32_t(a.win_lo.size());
    mb += a.n_meas;
    sb += a.slab_words;
    bmb += a.bm_words;
  }
  out.chan_foff.push_back(fb);
  out.inj_off.push_back(ib);
  out.n_meas = mb;
  out.n_faults = fb;
  out.w = wb;
  out.slab_words = sb;
  out.bm_words = bmb;
  // the longest sweeps first (stable: a circuit's own order is kept among equals)
  std::vector<uint32_t> idx(out.item_col.size());
  for (uint32_t i = 0; i < idx.size(); i++) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](uint32_t x, uint32_t y) { return item_order_span[x] > item_order_span[y]; });
  auto permute = [&](std::vector<uint32_t>& v) {
    std::vector<uint32_t> t(v.size());
    for (size_t i = 0; i < idx.size(); i++) t[i] = v[idx[i]];
    v.swap(t);
  };
  permute(out.item_col);
  permute(out.item_blo);
  permute(out.item_bhi);
  permute(out.item_branch);
}

int apply_rates(Lowered& lw, const double* rates, size_t n_rates, LowerError& err) {
  const size_t C = lw.chan_kind.size();
  if (n_rates != C) return set_err(err, GP_E_NOISE, 0, "%s", "rate array length differs from the channel count");
  for (size_t d = 0; d < C; d++) {
    double r = rates[lw.chan_src[d]];
    if (!(r >= 0.0 && r <= rate_limit(lw.chan_kind[d]))) return set_err(err, GP_E_NOISE, 0, "%s", "rate out of range");
    lw.chan_rate[d] = r;
  }
  return 0;
}

}  // namespace gp
