// C ABI of the compiler: driver lifetime, buffers sized from bounds (paper
// Sec. 3.4), host lowering + upload, device stages, result download.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "driver_internal.h"
#include "gp.h"
#include "kernels.h"
#include "lower.h"

namespace {

thread_local std::string g_error = "no error";

int fail(int code, const char* msg) noexcept {
  try {
    g_error = msg;
  } catch (...) {
    // no memory for the message: the previous one stays
  }
  return code;
}

int fail(int code, const std::string& msg) noexcept { return fail(code, msg.c_str()); }

int hip_fail(hipError_t e, const char* what) {
  return fail(GP_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

uint32_t words_for(uint32_t det, uint32_t obs) { return (det + 63) / 64 + (obs + 63) / 64; }

// Layout of the per-compile input tables inside one device arena and one
// pinned host buffer of the same shape, so one copy uploads them all.
struct TableLayout {
  size_t layer_off, chan_qa, chan_qb, chan_kind, chan_rate, chan_src, chan_foff, bnd_chan_off,
      bnd_fault_off, col_top, col_lo, col_base, item_col, item_blo, item_bhi, fnv_pow, ops32, inj_off, inj_layer,
      inj_qubit, inj_word, inj_next, hchunk_pos, hchunk_bnd, bnd_bm_off, col_bm_base, layer_win, win_lo, win_obase,
      win_cnt, branch, item_branch, hchunk_branch, total;
};

// Entry counts of the tables: exact for a lowering, upper bounds for a driver.
struct TableSizes {
  uint64_t ops, layer_entries, inj, chans, bnd_entries, cols, items, fnv, hchunks, windows, branches;
};

TableSizes sizes_of(const gp::Lowered& lw) {
  return {lw.ops32.size(), lw.layer_off.size(), lw.inj_layer.size(), lw.chan_kind.size(), lw.bnd_fault_off.size(),
          lw.col_top.size(), lw.item_col.size(), lw.fnv_pow.size(), lw.hchunk_pos.size(), lw.win_lo.size(),
          lw.branches.size()};
}

TableLayout layout_for(const TableSizes& z) {
  TableLayout t{};
  size_t o = 0;
  auto take = [&](size_t& f, size_t bytes) {
    f = o;
    o += align_up(bytes ? bytes : 1);
  };
  take(t.layer_off, z.layer_entries * 4);
  take(t.chan_qa, z.chans * 4);
  take(t.chan_qb, z.chans * 4);
  take(t.chan_kind, z.chans);
  take(t.chan_rate, z.chans * 8);
  take(t.chan_src, z.chans * 4);
  take(t.chan_foff, (z.chans + 1) * 4);
  take(t.bnd_chan_off, z.bnd_entries * 4);
  take(t.bnd_fault_off, z.bnd_entries * 4);
  take(t.col_top, z.cols * 4);
  take(t.col_lo, z.cols * 4);
  take(t.col_base, z.cols * 8);
  take(t.item_col, z.items * 4);
  take(t.item_blo, z.items * 4);
  take(t.item_bhi, z.items * 4);
  take(t.fnv_pow, z.fnv * 8);
  take(t.ops32, z.ops * 4);
  take(t.inj_off, (z.cols + 1) * 4);
  take(t.inj_layer, z.inj * 4);
  take(t.inj_qubit, z.inj * 4);
  take(t.inj_word, z.inj * 8);
  take(t.inj_next, z.inj * 4);
  take(t.hchunk_pos, z.hchunks * 4);
  take(t.hchunk_bnd, z.hchunks * 4);
  take(t.bnd_bm_off, z.bnd_entries * 4);
  take(t.col_bm_base, z.cols * 8);
  take(t.layer_win, z.layer_entries * 4);
  take(t.win_lo, z.windows * 4);
  take(t.win_obase, z.windows * 4);
  take(t.win_cnt, z.windows * 4);
  take(t.branch, z.branches * sizeof(gp::BranchDesc));
  take(t.item_branch, z.items * 4);
  take(t.hchunk_branch, z.hchunks * 4);
  t.total = o;
  return t;
}

struct TimedLaunch {
  int id;
  hipEvent_t a, b;
};

// Host threads for splitting a result of U hyperedges (one per 64 Ki, at most 16).
size_t split_threads(uint64_t U) {
  return std::min<size_t>({16, std::max<size_t>(1, std::thread::hardware_concurrency()),
                           std::max<uint64_t>(1, U / 65536)});
}

// Run fn(0 .. T-1) on T threads (inline when T is 1) and wait for all; an
// exception thrown by any share is rethrown here once every thread has ended.
template <typename F>
void run_threads(size_t T, F&& fn) {
  if (T <= 1) {
    fn(size_t(0));
    return;
  }
  std::vector<std::exception_ptr> errs(T);
  auto share = [&](size_t t) {
    try {
      fn(t);
    } catch (...) {
      errs[t] = std::current_exception();
    }
  };
  // a thread that cannot be started runs its share here instead
  std::vector<std::thread> pool;
  pool.reserve(T);
  for (size_t t = 0; t < T; t++) {
    try {
      pool.emplace_back(share, t);
    } catch (...) {
      share(t);
    }
  }
  for (std::thread& th : pool) th.join();
  for (const std::exception_ptr& e : errs)
    if (e) std::rethrow_exception(e);
}


}  // namespace

struct gp_edges {
  uint32_t n_det = 0, n_obs = 0;      // most detectors / observables of any circuit
  // packed form of the signatures, made on the first request (gp_edges_signatures)
  std::once_flag words_once;
  uint32_t n_words = 0;
  std::vector<uint64_t> words;
  int words_rc = GP_OK;
  std::vector<uint64_t> off;
  std::vector<uint32_t> bits;
  std::vector<double> q;
  std::vector<uint32_t> circuit;      // per hyperedge: its circuit in the batch
  std::vector<uint32_t> c_det, c_obs; // per circuit: detectors, observables
  std::vector<uint64_t> c_off;        // per circuit: its hyperedges [c_off[k], c_off[k+1])
};

struct gp_driver {
  int device = 0;
  hipStream_t stream = nullptr;
  gp_bounds bounds{};
  uint32_t max_w = 1;
  uint64_t bits_cap = 0;
  uint32_t max_tiles = 1;

  std::vector<void*> allocations;
  char* d_tables = nullptr;
  size_t tables_cap = 0;
  char* h_tables = nullptr;  // pinned
  void* h_out = nullptr;     // pinned download staging
  size_t h_out_cap = 0;
  gp::DevHeader* h_hdr = nullptr;  // pinned

  gp::Lowered lw;
  bool lowered = false;
  bool ran = false;
  bool structured = false;     // a fetched compile left its class structure on the device
  uint64_t struct_edges = 0;   // hyperedges of that compile
  uint64_t struct_id = 0;      // bumped by every fetch that leaves a structure (gp_structure_id)
  hipEvent_t ev_drv = nullptr, ev_user = nullptr;  // orders the caller's stream against the driver's
  // a downloaded single-circuit result in the pinned staging buffer (gp_fetch_sizes)
  bool staged_ok = false;
  uint64_t staged_U = 0, staged_nb = 0;
  const uint32_t* staged_off = nullptr;
  const uint32_t* staged_bits = nullptr;
  const double* staged_q = nullptr;
  const uint32_t* staged_ceoff = nullptr;
  gp::DevState st{};

  uint32_t key_bits = 64;      // test hook: class keys cut to this many bits
  uint32_t sort_mode = gp::SORT_AUTO;  // test hook: force the full radix sort
  uint32_t sweep_shape = 0;            // test hook: force a stage-1 work-group shape
  uint64_t bm_cap = 0;                 // non-zero-word bitmap words allocated
  uint32_t level = 2;                  // correlation level for the next lowering
  double fault_cost = gp::kDefaultFaultCost;  // observable range cut (set by gp_autotune)
  uint32_t spin_limit = gp::kSpinLimit;  // test hook: look-back rounds before a sort tile gives up
  uint64_t collision_retries = 0, bucket_retries = 0, lookback_retries = 0;
  // test hook: each gp_run copies the per-position class keys here once the
  // hash kernel has written them (the grouping passes overwrite them after)
  bool capture_keys = false;
  uint64_t* key_copy = nullptr;
  uint32_t captured_key_bits = 0;
  uint64_t captured_faults = 0;

  // optionally, the compile's launch sequence captured as a HIP graph and
  // replayed while the lowering and the modes it was captured with stay the same
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  uint64_t lower_gen = 0;      // bumped by every upload of a lowering
  uint64_t graph_gen = ~0ull;  // the lowering generation the graph was captured for
  uint32_t graph_key_bits = 0, graph_sort_mode = 0, graph_shape = 0, graph_spin = 0;

  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<TimedLaunch> pending;
  double total_ms[gp::K_COUNT] = {};
  uint64_t launches[gp::K_COUNT] = {};
};

namespace {

template <typename T>
int dev_alloc(gp_driver* d, T** p, size_t count, const char* what) {
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(count * sizeof(T), 256));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? GP_E_OOM : GP_E_HIP,
                std::string("device allocation of ") + what + " failed: " + hipGetErrorString(e));
  }
  d->allocations.push_back(v);
  *p = static_cast<T*>(v);
  return GP_OK;
}

void hook_before(void* ctx, int id) {
  gp_driver* d = static_cast<gp_driver*>(ctx);
  TimedLaunch t{id, nullptr, nullptr};
  for (hipEvent_t* e : {&t.a, &t.b}) {
    if (!d->ev_free.empty()) {
      *e = d->ev_free.back();
      d->ev_free.pop_back();
    } else if (hipEventCreate(e) != hipSuccess) {
      *e = nullptr;
    }
  }
  if (t.a) (void)hipEventRecord(t.a, d->stream);
  d->pending.push_back(t);
}

void hook_after(void* ctx, int) {
  gp_driver* d = static_cast<gp_driver*>(ctx);
  if (!d->pending.empty() && d->pending.back().b) (void)hipEventRecord(d->pending.back().b, d->stream);
}

void hook_after_keys(void* ctx, int id) {
  gp_driver* d = static_cast<gp_driver*>(ctx);
  if (d->timing) hook_after(ctx, id);
  if (id == gp::K_HASH && d->st.n_faults)
    (void)hipMemcpyAsync(d->key_copy, d->st.key[1], size_t(d->st.n_faults) * sizeof(uint64_t),
                         hipMemcpyDeviceToDevice, d->stream);
}

void collect_timing(gp_driver* d) {
  for (TimedLaunch& t : d->pending) {
    float ms = 0.f;
    if (t.a && t.b && hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      d->total_ms[t.id] += ms;
      d->launches[t.id]++;
    }
    if (t.a) d->ev_free.push_back(t.a);
    if (t.b) d->ev_free.push_back(t.b);
  }
  d->pending.clear();
}

uint32_t branches_of(const gp_bounds& b) { return std::max<uint32_t>(b.max_branches, 1); }

uint64_t hash_chunk_cap(const gp_bounds& b) {
  return b.max_faults / 256 + uint64_t(branches_of(b)) * (uint64_t(b.max_layers) + 2);
}

// Table capacities of a driver: per-circuit maxima times the circuits of a batch.
TableSizes sizes_cap(const gp_bounds& b, uint32_t max_w) {
  const uint64_t B = branches_of(b), L = b.max_layers;
  // injection entries: one per (column, measurement) pair, so at most one per leaf bit
  return {b.max_ops, B * (L + 1), b.max_leaf_bits, b.max_channels, B * (L + 2), B * max_w, b.max_items,
          uint64_t(max_w) + 1, hash_chunk_cap(b), B * (L + 1), B};
}

int check_bounds(const gp_driver* d, const gp::Lowered& lw) {
  const gp_bounds& b = d->bounds;
  char msg[256];
  auto over = [&](const char* what, uint64_t have, uint64_t cap) {
    std::snprintf(msg, sizeof msg, "circuit exceeds the driver bounds: %s %" PRIu64 " > %" PRIu64, what, have, cap);
    return fail(GP_E_BOUNDS, msg);
  };
  if (lw.branches.size() > branches_of(b)) return over("circuits in a batch", lw.branches.size(), branches_of(b));
  if (lw.n_qubits > b.max_qubits) return over("qubits", lw.n_qubits, b.max_qubits);
  if (lw.n_layers > b.max_layers) return over("layers", lw.n_layers, b.max_layers);
  if (lw.n_meas > b.max_measurements) return over("measurements", lw.n_meas, b.max_measurements);
  if (lw.n_det > b.max_detectors) return over("detectors", lw.n_det, b.max_detectors);
  if (lw.n_obs > b.max_observables) return over("observables", lw.n_obs, b.max_observables);
  if (lw.chan_kind.size() > b.max_channels) return over("channels", lw.chan_kind.size(), b.max_channels);
  if (lw.n_faults > b.max_faults) return over("faults", lw.n_faults, b.max_faults);
  if (lw.ops.size() > b.max_ops) return over("operations", lw.ops.size(), b.max_ops);
  if (lw.leaf_bits.size() > b.max_leaf_bits) return over("leaf bits", lw.leaf_bits.size(), b.max_leaf_bits);
  if (lw.slab_words > b.max_slab_words) return over("slab words", lw.slab_words, b.max_slab_words);
  if (lw.item_col.size() > b.max_items) return over("sweep items", lw.item_col.size(), b.max_items);
  if (lw.bm_words > d->bm_cap) return over("non-zero-word bitmap words", lw.bm_words, d->bm_cap);
  for (uint32_t c : lw.win_cnt)
    if (c > gp::kSweepWinOps) return over("operations in one layer (sweep op window)", c, gp::kSweepWinOps);
  if (lw.w_max > d->max_w) return over("signature words", lw.w_max, d->max_w);
  if (lw.w_max > gp::kMaxHashWords) return over("signature words for the hash kernel", lw.w_max, gp::kMaxHashWords);
  if (lw.n_qubits > gp::kMaxSweepQubits) return over("qubits for the compact op words", lw.n_qubits, gp::kMaxSweepQubits);
  if (lw.hchunk_pos.size() > hash_chunk_cap(b)) return over("hash chunks", lw.hchunk_pos.size(), hash_chunk_cap(b));
  if (layout_for(sizes_of(lw)).total > d->tables_cap)
    return over("table bytes", layout_for(sizes_of(lw)).total, d->tables_cap);
  if (gp::sweep_lds_bytes(lw.n_qubits) > gp::sweep_lds_limit())
    return over("LDS bytes for the qubit frame", gp::sweep_lds_bytes(lw.n_qubits), gp::sweep_lds_limit());
  return GP_OK;
}

void fill_bounds(const gp::Lowered& lw, gp_bounds* out) {
  gp_bounds b{};
  b.max_qubits = lw.n_qubits;
  b.max_layers = lw.n_layers;
  b.max_measurements = lw.n_meas;
  b.max_detectors = lw.n_det;
  b.max_observables = lw.n_obs;
  b.max_channels = uint32_t(lw.chan_kind.size());
  b.max_faults = lw.n_faults;
  b.max_ops = lw.ops.size();
  b.max_leaf_bits = lw.leaf_bits.size();
  b.max_branches = uint32_t(lw.branches.size());
  // any circuit within these bounds needs at most one word per (fault, column)
  b.max_slab_words = std::max<uint64_t>(lw.slab_words, lw.n_faults * uint64_t(lw.w_max));
  // detector columns one item each; observable ranges fill the slots left
  b.max_items = uint64_t(b.max_branches) * (std::max<uint64_t>(gp::kSweepSlots, lw.w_max) + 16);
  *out = b;
}

// Lower every circuit of a batch, each on its own (on up to 16 host threads,
// each circuit with its share of the sweep slots), and merge them.
// lower_one(k, slots, out, err) lowers circuit k and returns its status.
template <typename LowerOne>
int lower_batch_with(size_t n, LowerOne&& lower_one, gp::Lowered& out) {
  if (n == 0) return fail(GP_E_ARG, "a batch needs at least one circuit");
  if (n > (1u << 20)) return fail(GP_E_BOUNDS, "at most 2^20 circuits in one batch");
  const uint32_t slots = std::max<uint32_t>(1, uint32_t((gp::kSweepSlots + n - 1) / n));
  std::vector<gp::Lowered> parts(n);
  std::vector<gp::LowerError> errs(n);
  std::vector<int> rcs(n, 0);
  auto lower_range = [&](size_t lo, size_t hi) {
    for (size_t k = lo; k < hi; k++) {
      try {
        rcs[k] = lower_one(k, slots, parts[k], errs[k]);
      } catch (...) {
        // on a lowering thread: nothing may be thrown out of it
        rcs[k] = GP_E_OOM;
        errs[k].code = GP_E_OOM;
        errs[k].msg = "host memory allocation failed while lowering";
      }
    }
  };
  const size_t n_threads = std::min<size_t>({n, 16, std::max<size_t>(1, std::thread::hardware_concurrency())});
  if (n_threads <= 1) {
    lower_range(0, n);
  } else {
    std::vector<std::thread> pool;
    pool.reserve(n_threads);
    for (size_t t = 0; t < n_threads; t++) {
      const size_t a = n * t / n_threads, b = n * (t + 1) / n_threads;
      try {
        pool.emplace_back(lower_range, a, b);
      } catch (...) {
        lower_range(a, b);  // could not start a thread: lower this share here
      }
    }
    for (std::thread& th : pool) th.join();
  }
  for (size_t k = 0; k < n; k++)
    if (rcs[k]) return fail(rcs[k], "circuit " + std::to_string(k) + " of the batch: " + errs[k].msg);
  uint64_t faults = 0;
  for (const gp::Lowered& a : parts) faults += a.n_faults;
  if (faults >= (1ull << 30)) return fail(GP_E_BOUNDS, "at most 2^30 - 1 faults in one batch");
  gp::merge_branches(parts, out);
  return GP_OK;
}

// Batch of circuit texts; `rates` may be null (rates written in the texts),
// as may any rates[k].
int lower_batch(const char* const* texts, const size_t* lens, const double* const* rates, const size_t* n_rates,
                size_t n, uint32_t level, gp::Lowered& out, double fault_cost = gp::kDefaultFaultCost) {
  if ((!texts || !lens) && n) return fail(GP_E_ARG, "null argument");
  if (rates && !n_rates) return fail(GP_E_ARG, "rate arrays without their lengths");
  for (size_t k = 0; k < n; k++)
    if (!texts[k]) return fail(GP_E_ARG, "null circuit text in the batch");
  return lower_batch_with(
      n,
      [&](size_t k, uint32_t slots, gp::Lowered& lw, gp::LowerError& err) {
        const double* r = rates ? rates[k] : nullptr;
        return gp::lower_circuit(texts[k], lens[k], r, r ? n_rates[k] : 0, slots, lw, err, level, fault_cost);
      },
      out);
}

// Batch of circuits in binary form (irs[k], k < n).
int lower_batch_ir(const gp_circuit_ir* irs, const double* const* rates, const size_t* n_rates, size_t n,
                   uint32_t level, gp::Lowered& out, double fault_cost = gp::kDefaultFaultCost) {
  if (!irs && n) return fail(GP_E_ARG, "null argument");
  if (rates && !n_rates) return fail(GP_E_ARG, "rate arrays without their lengths");
  return lower_batch_with(
      n,
      [&](size_t k, uint32_t slots, gp::Lowered& lw, gp::LowerError& err) {
        const double* r = rates ? rates[k] : nullptr;
        return gp::lower_ir(irs[k], r, r ? n_rates[k] : 0, slots, lw, err, level, fault_cost);
      },
      out);
}

}  // namespace

extern "C" {

const char* gp_last_error(void) { return g_error.c_str(); }

static int gp_bounds_from_circuit_impl(const char* text, size_t len, gp_bounds* out) {
  if (!text || !out) return fail(GP_E_ARG, "null argument");
  gp::Lowered lw;
  gp::LowerError err{};
  int rc = gp::lower_circuit(text, len, nullptr, 0, gp::kSweepSlots, lw, err);
  if (rc) return fail(rc, err.msg);
  fill_bounds(lw, out);
  return GP_OK;
}

static int gp_bounds_from_ir_impl(const gp_circuit_ir* ir, gp_bounds* out) {
  if (!ir || !out) return fail(GP_E_ARG, "null argument");
  gp::Lowered lw;
  gp::LowerError err{};
  int rc = gp::lower_ir(*ir, nullptr, 0, gp::kSweepSlots, lw, err);
  if (rc) return fail(rc, err.msg);
  fill_bounds(lw, out);
  return GP_OK;
}

static int gp_bounds_from_batch_ir_impl(const gp_circuit_ir* irs, size_t n, gp_bounds* out) {
  if (!out) return fail(GP_E_ARG, "null argument");
  gp::Lowered lw;
  int rc = lower_batch_ir(irs, nullptr, nullptr, n, 2, lw);
  if (rc) return rc;
  fill_bounds(lw, out);
  return GP_OK;
}

void gp_driver_destroy(gp_driver* d) {
  if (!d) return;
  (void)hipSetDevice(d->device);
  if (d->stream) (void)hipStreamSynchronize(d->stream);
  for (void* p : d->allocations) (void)hipFree(p);
  if (d->h_tables) (void)hipHostFree(d->h_tables);
  if (d->h_out) (void)hipHostFree(d->h_out);
  if (d->h_hdr) (void)hipHostFree(d->h_hdr);
  if (d->gexec) (void)hipGraphExecDestroy(d->gexec);
  if (d->ev_drv) (void)hipEventDestroy(d->ev_drv);
  if (d->ev_user) (void)hipEventDestroy(d->ev_user);
  for (TimedLaunch& t : d->pending) {
    if (t.a) (void)hipEventDestroy(t.a);
    if (t.b) (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : d->ev_free) (void)hipEventDestroy(e);
  if (d->stream) (void)hipStreamDestroy(d->stream);
  delete d;
}

static int gp_driver_create_impl(const gp_bounds* bounds, int device, gp_driver** out) {
  if (!bounds || !out) return fail(GP_E_ARG, "null argument");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(GP_E_HIP, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(GP_E_ARG, "device index out of range");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GP_E_HIP, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  HIP_TRY(hipSetDevice(device), "hipSetDevice");
  HIP_TRY(gp::configure_kernels(), "configure kernels");
  HIP_TRY(gp::scratch_init(device), "static scratch address");

  gp_driver* d = new gp_driver();
  d->device = device;
  d->bounds = *bounds;
  gp_bounds& b = d->bounds;
  b.max_layers = std::max<uint32_t>(b.max_layers, 1);
  b.max_faults = std::max<uint64_t>(b.max_faults, 1);
  b.max_branches = branches_of(b);
  if (b.max_faults >= (1ull << 30)) {
    delete d;
    return fail(GP_E_BOUNDS, "at most 2^30 - 1 faults per compile");
  }
  d->max_w = std::max<uint32_t>(words_for(b.max_detectors, b.max_observables), 1);
  if (!b.max_slab_words) b.max_slab_words = b.max_faults * d->max_w;
  if (!b.max_items) b.max_items = uint64_t(branches_of(b)) * (std::max<uint64_t>(gp::kSweepSlots, d->max_w) + 16);
  d->bits_cap = std::max<uint64_t>(b.max_faults * 8, 1u << 20);
  d->max_tiles = uint32_t((b.max_faults + 4095) / 4096) + 1;

  int rc = GP_OK;
  auto cleanup = [&](int code) {
    gp_driver_destroy(d);
    return code;
  };
  if (hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking) != hipSuccess)
    return cleanup(hip_fail(hipGetLastError(), "hipStreamCreate"));

  TableLayout tl = layout_for(sizes_cap(b, d->max_w));
  d->tables_cap = tl.total;
  if ((rc = dev_alloc(d, &d->d_tables, d->tables_cap, "tables"))) return cleanup(rc);
  if (hipHostMalloc(reinterpret_cast<void**>(&d->h_tables), d->tables_cap, hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(GP_E_OOM, "pinned host allocation failed"));
  if (hipHostMalloc(reinterpret_cast<void**>(&d->h_hdr), sizeof(gp::DevHeader), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(GP_E_OOM, "pinned host allocation failed"));

  gp::DevState& st = d->st;
  const uint64_t F = b.max_faults;
  uint64_t* slab = nullptr;
  if ((rc = dev_alloc(d, &slab, b.max_slab_words, "signature slab"))) return cleanup(rc);
  st.slab = slab;
  // a column's bitmaps take at most (its slab words) / 64 + (boundaries) words
  d->bm_cap = b.max_slab_words / 64 + uint64_t(branches_of(b)) * d->max_w * (uint64_t(b.max_layers) + 2);
  if ((rc = dev_alloc(d, &st.bm, d->bm_cap, "non-zero-word bitmaps"))) return cleanup(rc);
  const size_t bnd_rows = size_t(branches_of(b)) * (size_t(b.max_layers) + 2);
  if ((rc = dev_alloc(d, &st.cover_lo, size_t(branches_of(b)) * d->max_w, "cover_lo"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.cov, bnd_rows * d->max_w, "cover lists"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.ncov, bnd_rows, "cover counts"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.frp, F, "fault probabilities and check hashes"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.crp, F, "partitioned fault records"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.frec, F, "fault records"))) return cleanup(rc);
  for (int k = 0; k < 2; k++) {
    if ((rc = dev_alloc(d, &st.key[k], F, "keys"))) return cleanup(rc);
    if ((rc = dev_alloc(d, &st.val[k], F, "values"))) return cleanup(rc);
  }
  if ((rc = dev_alloc(d, &st.popc, F, "signature weights"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.erec, F, "edge records"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.tile_cnt, size_t(d->max_tiles) + 1, "tile counts"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.tile_nzw, size_t(d->max_tiles) + 1, "tile word counts"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.digit_tot, size_t(gp::kMaxPasses) * 256, "digit totals"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.lookback, size_t(gp::kMaxPasses) * d->max_tiles * 256, "look-back words")))
    return cleanup(rc);
  if ((rc = dev_alloc(d, &st.tile_ctr, gp::kMaxPasses, "tile tickets"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.tile_sum, size_t(d->max_tiles) + 1, "tile sums"))) return cleanup(rc);
  st.max_tiles = d->max_tiles;
  if ((rc = dev_alloc(d, &st.segstart, F, "class starts"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.big, F / 64 + 1, "large classes"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.b16_lo, size_t(gp::kBuckets16), "16-bit bucket starts")) ||
      (rc = dev_alloc(d, &st.b16_hi, size_t(gp::kBuckets16), "16-bit bucket ends")))
    return cleanup(rc);
  if ((rc = dev_alloc(d, &st.rep_bm, F / 64 + 1, "representative bitmap"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.rrec, F, "representative records"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.out_lb, 2 * size_t(d->max_tiles), "output look-back words"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.out_ctr, 1, "output tile ticket"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.rep_pos, F, "representative positions"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.circ_eoff, size_t(b.max_branches) + 1, "circuit hyperedge offsets")))
    return cleanup(rc);
  if ((rc = dev_alloc(d, &st.e_first, F, "hyperedge member offsets"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.e_cnt, F, "hyperedge member counts"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.gfault, F, "fault gradients"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.gq, F, "hyperedge gradients"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.gr, std::max<uint64_t>(b.max_channels, 1), "channel gradients"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.edge_off32, F + 1, "edge offsets"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.edge_bits, d->bits_cap, "edge bits"))) return cleanup(rc);
  if ((rc = dev_alloc(d, &st.edge_q, F, "edge probabilities"))) return cleanup(rc);
  if (hipEventCreateWithFlags(&d->ev_drv, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&d->ev_user, hipEventDisableTiming) != hipSuccess)
    return cleanup(hip_fail(hipGetLastError(), "hipEventCreate"));
  if ((rc = dev_alloc(d, &st.hdr, 1, "header"))) return cleanup(rc);
  if (hipMemset(st.hdr, 0, sizeof(gp::DevHeader)) != hipSuccess)
    return cleanup(hip_fail(hipGetLastError(), "clearing the device header"));
  if ((rc = dev_alloc(d, &st.item_clock, 2 * b.max_items, "item clocks"))) return cleanup(rc);
  st.bits_cap = d->bits_cap;
  // download staging: offsets + bits + probabilities + circuits of the largest result
  d->h_out_cap = (F + 1) * 4 + d->bits_cap * 4 + F * 8 + (size_t(b.max_branches) + 1) * 4 + 4 * kAlign;
  if (hipHostMalloc(&d->h_out, d->h_out_cap, hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(GP_E_OOM, "pinned host allocation failed"));
  *out = d;
  return GP_OK;
}

static int gp_driver_create_from_circuit_impl(const char* text, size_t len, int device, gp_driver** out) {
  gp_bounds b;
  int rc = gp_bounds_from_circuit(text, len, &b);
  if (rc) return rc;
  return gp_driver_create(&b, device, out);
}

static int gp_bounds_from_batch_impl(const char* const* texts, const size_t* lens, size_t n, gp_bounds* out) {
  if (!out) return fail(GP_E_ARG, "null argument");
  gp::Lowered lw;
  int rc = lower_batch(texts, lens, nullptr, nullptr, n, 2, lw);
  if (rc) return rc;
  fill_bounds(lw, out);
  return GP_OK;
}

static int gp_driver_create_from_batch_impl(const char* const* texts, const size_t* lens, size_t n, int device,
                                gp_driver** out) {
  gp_bounds b;
  int rc = gp_bounds_from_batch(texts, lens, n, &b);
  if (rc) return rc;
  return gp_driver_create(&b, device, out);
}

// Upload a lowering (one circuit, or a merged batch) and point the device state at it.
static int upload_lowered(gp_driver* d) {
  int rc;
  if ((rc = check_bounds(d, d->lw))) return rc;
  const gp::Lowered& lw = d->lw;
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  // the previous compile may still read the pinned buffer
  HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  TableLayout tl = layout_for(sizes_of(lw));
  if (tl.total > d->tables_cap) return fail(GP_E_BOUNDS, "lowered tables exceed the driver's table arena");
  char* h = d->h_tables;
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(h + off, src, bytes);
  };
  put(tl.layer_off, lw.layer_off.data(), lw.layer_off.size() * 4);
  put(tl.chan_qa, lw.chan_qa.data(), lw.chan_qa.size() * 4);
  put(tl.chan_qb, lw.chan_qb.data(), lw.chan_qb.size() * 4);
  put(tl.chan_kind, lw.chan_kind.data(), lw.chan_kind.size());
  put(tl.chan_rate, lw.chan_rate.data(), lw.chan_rate.size() * 8);
  put(tl.chan_src, lw.chan_src.data(), lw.chan_src.size() * 4);
  put(tl.chan_foff, lw.chan_foff.data(), lw.chan_foff.size() * 4);
  put(tl.bnd_chan_off, lw.bnd_chan_off.data(), lw.bnd_chan_off.size() * 4);
  put(tl.bnd_fault_off, lw.bnd_fault_off.data(), lw.bnd_fault_off.size() * 4);
  put(tl.col_top, lw.col_top.data(), lw.col_top.size() * 4);
  put(tl.col_lo, lw.col_lo.data(), lw.col_lo.size() * 4);
  put(tl.col_base, lw.col_base.data(), lw.col_base.size() * 8);
  put(tl.item_col, lw.item_col.data(), lw.item_col.size() * 4);
  put(tl.item_blo, lw.item_blo.data(), lw.item_blo.size() * 4);
  put(tl.item_bhi, lw.item_bhi.data(), lw.item_bhi.size() * 4);
  put(tl.fnv_pow, lw.fnv_pow.data(), lw.fnv_pow.size() * 8);
  put(tl.ops32, lw.ops32.data(), lw.ops32.size() * 4);
  put(tl.inj_off, lw.inj_off.data(), lw.inj_off.size() * 4);
  put(tl.inj_layer, lw.inj_layer.data(), lw.inj_layer.size() * 4);
  put(tl.inj_qubit, lw.inj_qubit.data(), lw.inj_qubit.size() * 4);
  put(tl.inj_word, lw.inj_word.data(), lw.inj_word.size() * 8);
  put(tl.inj_next, lw.inj_next.data(), lw.inj_next.size() * 4);
  put(tl.hchunk_pos, lw.hchunk_pos.data(), lw.hchunk_pos.size() * 4);
  put(tl.hchunk_bnd, lw.hchunk_bnd.data(), lw.hchunk_bnd.size() * 4);
  put(tl.bnd_bm_off, lw.bnd_bm_off.data(), lw.bnd_bm_off.size() * 4);
  put(tl.col_bm_base, lw.col_bm_base.data(), lw.col_bm_base.size() * 8);
  put(tl.layer_win, lw.layer_win.data(), lw.layer_win.size() * 4);
  put(tl.win_lo, lw.win_lo.data(), lw.win_lo.size() * 4);
  put(tl.win_obase, lw.win_obase.data(), lw.win_obase.size() * 4);
  put(tl.win_cnt, lw.win_cnt.data(), lw.win_cnt.size() * 4);
  put(tl.branch, lw.branches.data(), lw.branches.size() * sizeof(gp::BranchDesc));
  put(tl.item_branch, lw.item_branch.data(), lw.item_branch.size() * 4);
  put(tl.hchunk_branch, lw.hchunk_branch.data(), lw.hchunk_branch.size() * 4);
  HIP_TRY(hipMemcpyAsync(d->d_tables, d->h_tables, tl.total, hipMemcpyHostToDevice, d->stream), "upload tables");

  gp::DevState& st = d->st;
  char* D = d->d_tables;
  st.layer_off = reinterpret_cast<const uint32_t*>(D + tl.layer_off);
  st.chan_qa = reinterpret_cast<const uint32_t*>(D + tl.chan_qa);
  st.chan_qb = reinterpret_cast<const uint32_t*>(D + tl.chan_qb);
  st.chan_kind = reinterpret_cast<const uint8_t*>(D + tl.chan_kind);
  st.chan_rate = reinterpret_cast<const double*>(D + tl.chan_rate);
  st.chan_src = reinterpret_cast<const uint32_t*>(D + tl.chan_src);
  st.chan_foff = reinterpret_cast<const uint32_t*>(D + tl.chan_foff);
  st.bnd_chan_off = reinterpret_cast<const uint32_t*>(D + tl.bnd_chan_off);
  st.bnd_fault_off = reinterpret_cast<const uint32_t*>(D + tl.bnd_fault_off);
  st.col_top = reinterpret_cast<const int32_t*>(D + tl.col_top);
  st.col_lo = reinterpret_cast<const int32_t*>(D + tl.col_lo);
  st.col_base = reinterpret_cast<const uint64_t*>(D + tl.col_base);
  st.item_col = reinterpret_cast<const uint32_t*>(D + tl.item_col);
  st.item_blo = reinterpret_cast<const uint32_t*>(D + tl.item_blo);
  st.item_bhi = reinterpret_cast<const uint32_t*>(D + tl.item_bhi);
  st.fnv_pow = reinterpret_cast<const uint64_t*>(D + tl.fnv_pow);
  st.ops32 = reinterpret_cast<const uint32_t*>(D + tl.ops32);
  st.inj_off = reinterpret_cast<const uint32_t*>(D + tl.inj_off);
  st.inj_layer = reinterpret_cast<const uint32_t*>(D + tl.inj_layer);
  st.inj_qubit = reinterpret_cast<const uint32_t*>(D + tl.inj_qubit);
  st.inj_word = reinterpret_cast<const uint64_t*>(D + tl.inj_word);
  st.inj_next = reinterpret_cast<const uint32_t*>(D + tl.inj_next);
  st.hchunk_pos = reinterpret_cast<const uint32_t*>(D + tl.hchunk_pos);
  st.hchunk_bnd = reinterpret_cast<const uint32_t*>(D + tl.hchunk_bnd);
  st.n_hchunks = uint32_t(lw.hchunk_pos.size());
  st.bnd_bm_off = reinterpret_cast<const uint32_t*>(D + tl.bnd_bm_off);
  st.col_bm_base = reinterpret_cast<const uint64_t*>(D + tl.col_bm_base);
  st.layer_win = reinterpret_cast<const uint32_t*>(D + tl.layer_win);
  st.win_lo = reinterpret_cast<const uint32_t*>(D + tl.win_lo);
  st.win_obase = reinterpret_cast<const uint32_t*>(D + tl.win_obase);
  st.win_cnt = reinterpret_cast<const uint32_t*>(D + tl.win_cnt);
  st.branch = reinterpret_cast<const gp::BranchDesc*>(D + tl.branch);
  st.item_branch = reinterpret_cast<const uint32_t*>(D + tl.item_branch);
  st.hchunk_branch = reinterpret_cast<const uint32_t*>(D + tl.hchunk_branch);
  st.n_branch = uint32_t(lw.branches.size());
  st.w_max = lw.w_max;
  st.n_win = 0;
  for (const gp::BranchDesc& bd : lw.branches) st.n_win = std::max(st.n_win, bd.n_win);
  st.max_win_ops = 0;
  for (uint32_t c : lw.win_cnt) st.max_win_ops = std::max(st.max_win_ops, c);
  st.n_qubits = lw.n_qubits;
  st.n_layers = lw.n_layers;
  st.n_det = lw.n_det;
  st.wd = lw.wd;
  st.w = lw.w;
  st.n_chan = uint32_t(lw.chan_kind.size());
  st.n_items = uint32_t(lw.item_col.size());
  st.n_faults = uint32_t(lw.n_faults);
  st.level = lw.level;
  d->lowered = true;
  d->lower_gen++;
  return GP_OK;
}


// A new lowering replaces whatever the driver held: nothing is staged, run
// or structured until it has been run and fetched.
static void forget_compile(gp_driver* d) {
  d->staged_ok = false;
  d->lowered = false;
  d->ran = false;
  d->structured = false;
}

static int lower_text_at(gp_driver* d, const char* text, size_t len, const double* rates, size_t n_rates,
                         uint32_t level) {
  if (!d || !text) return fail(GP_E_ARG, "null argument");
  forget_compile(d);
  gp::LowerError err{};
  int rc = gp::lower_circuit(text, len, rates, n_rates, gp::kSweepSlots, d->lw, err, level, d->fault_cost);
  if (rc) return fail(rc, err.msg);
  return upload_lowered(d);
}

static int lower_ir_at(gp_driver* d, const gp_circuit_ir* ir, const double* rates, size_t n_rates,
                       uint32_t level) {
  if (!d || !ir) return fail(GP_E_ARG, "null argument");
  forget_compile(d);
  gp::LowerError err{};
  int rc = gp::lower_ir(*ir, rates, n_rates, gp::kSweepSlots, d->lw, err, level, d->fault_cost);
  if (rc) return fail(rc, err.msg);
  return upload_lowered(d);
}

static int gp_lower_impl(gp_driver* d, const char* text, size_t len, const double* rates, size_t n_rates) {
  return lower_text_at(d, text, len, rates, n_rates, d ? d->level : 2u);
}

static int gp_lower_ir_impl(gp_driver* d, const gp_circuit_ir* ir, const double* rates, size_t n_rates) {
  return lower_ir_at(d, ir, rates, n_rates, d ? d->level : 2u);
}

static int gp_lower_batch_ir_impl(gp_driver* d, const gp_circuit_ir* irs, size_t n, const double* const* rates,
                                  const size_t* n_rates) {
  if (!d) return fail(GP_E_ARG, "null driver");
  forget_compile(d);
  int rc = lower_batch_ir(irs, rates, n_rates, n, d->level, d->lw, d->fault_cost);
  if (rc) return rc;
  return upload_lowered(d);
}

static int gp_lower_batch_impl(gp_driver* d, const char* const* texts, const size_t* lens, const double* const* rates,
                   const size_t* n_rates, size_t n) {
  if (!d) return fail(GP_E_ARG, "null driver");
  forget_compile(d);
  int rc = lower_batch(texts, lens, rates, n_rates, n, d->level, d->lw, d->fault_cost);
  if (rc) return rc;
  return upload_lowered(d);
}

static int gp_run_impl(gp_driver* d) {
  if (!d) return fail(GP_E_ARG, "null driver");
  if (!d->lowered) return fail(GP_E_STATE, "gp_run before gp_lower");
  d->staged_ok = false;
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  gp::LaunchHook hook;
  if (d->timing) {
    hook.before = hook_before;
    hook.after = hook_after;
    hook.ctx = d;
  }
  if (d->capture_keys) {
    hook.after = hook_after_keys;
    hook.ctx = d;
    d->captured_faults = d->st.n_faults;
    d->captured_key_bits = gp::class_key_bits(d->st.n_faults, d->key_bits);
  }
  d->st.key_mode = 0;
  d->st.key_bits = d->key_bits;
  d->st.sort_mode = d->sort_mode;
  d->st.sweep_shape = d->sweep_shape;
  d->st.spin_limit = d->spin_limit;
  d->structured = false;
  if (d->use_graph && !d->timing && !d->capture_keys) {
    // replay the captured launch sequence; capture it first if the lowering
    // or a mode changed since
    if (!d->gexec || d->graph_gen != d->lower_gen || d->graph_key_bits != d->key_bits ||
        d->graph_sort_mode != d->sort_mode || d->graph_shape != d->sweep_shape ||
        d->graph_spin != d->spin_limit) {
      if (d->gexec) {
        (void)hipGraphExecDestroy(d->gexec);
        d->gexec = nullptr;
      }
      hipGraph_t g = nullptr;
      gp::LaunchHook none;
      HIP_TRY(hipStreamBeginCapture(d->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      const hipError_t ce = gp::enqueue_compile(d->st, d->stream, none);
      const hipError_t ee = hipStreamEndCapture(d->stream, &g);
      hipError_t ie = hipSuccess;
      if (ce == hipSuccess && ee == hipSuccess) ie = hipGraphInstantiate(&d->gexec, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (ce != hipSuccess || ee != hipSuccess || ie != hipSuccess) {
        (void)hipGetLastError();
        d->gexec = nullptr;
        return hip_fail(ce != hipSuccess ? ce : ee != hipSuccess ? ee : ie, "capturing the compile as a graph");
      }
      d->graph_gen = d->lower_gen;
      d->graph_key_bits = d->key_bits;
      d->graph_sort_mode = d->sort_mode;
      d->graph_shape = d->sweep_shape;
      d->graph_spin = d->spin_limit;
    }
    HIP_TRY(hipGraphLaunch(d->gexec, d->stream), "hipGraphLaunch");
    d->ran = true;
    return GP_OK;
  }
  hipError_t e = gp::enqueue_compile(d->st, d->stream, hook);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  d->ran = true;
  return GP_OK;
}

int gp_set_fault_cost(gp_driver* d, double fault_cost) {
  if (!d) return fail(GP_E_ARG, "null driver");
  if (!(fault_cost > 0.0 && fault_cost < 1.0)) return fail(GP_E_ARG, "fault cost must be in (0, 1)");
  d->fault_cost = fault_cost;
  return GP_OK;
}

static int gp_debug_device_flags_impl(gp_driver* d, uint32_t* flags, uint32_t* flags_seen, int clear_seen);

}  // extern "C"

namespace {

// Tuned parameters by lowered shape, shared by every driver of the process.
std::mutex g_tune_mu;
std::map<std::tuple<uint32_t, uint32_t, uint32_t, uint64_t, uint32_t, uint32_t, uint32_t>, gp_tuning> g_tune;

std::tuple<uint32_t, uint32_t, uint32_t, uint64_t, uint32_t, uint32_t, uint32_t> tune_key(const gp_tuning& t) {
  return {t.n_circuits, t.n_qubits, t.n_layers, t.n_faults, t.n_det, t.n_obs, t.level};
}

void shape_of(const gp::Lowered& lw, gp_tuning& t) {
  t.n_circuits = uint32_t(lw.branches.size());
  t.n_qubits = lw.n_qubits;
  t.n_layers = lw.n_layers;
  t.n_faults = lw.n_faults;
  t.n_det = lw.n_det;
  t.n_obs = lw.n_obs;
  t.level = lw.level;
}

// Times every (fault cost, sweep work-group) candidate on what `lower`
// lowers and keeps the fastest; a shape already in the cache is taken from it.
template <typename Lower>
int autotune(gp_driver* d, Lower&& lower, int iters, gp_tuning* out) {
  if (iters < 1) return fail(GP_E_ARG, "iters must be at least 1");
  static const double kCandidates[] = {2.5e-4, 4.0e-4, 6.2e-4, 9.0e-4, 1.4e-3};
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  const double saved_cost = d->fault_cost;
  const uint32_t saved_shape = d->sweep_shape;
  gp_tuning best{};
  int rc = lower();
  if (rc) return rc;
  shape_of(d->lw, best);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(tune_key(best));
    if (it != g_tune.end()) {
      best = it->second;
      best.cached = 1;
    }
  }
  if (!best.cached) {
    hipEvent_t a = nullptr, b = nullptr;
    HIP_TRY(hipEventCreate(&a), "hipEventCreate");
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return hip_fail(hipGetLastError(), "hipEventCreate");
    }
    // the 256-thread work-group is a candidate when the circuit fits its tables
    const int n_blocks = gp::sweep_small_fits(d->st) ? 2 : 1;
    best.ms = -1.0;
    for (int blk = 0; blk < n_blocks && rc == GP_OK; blk++) {
      for (double c : kCandidates) {
        d->fault_cost = c;
        d->sweep_shape = blk == 0 ? 1u : 2u;
        if ((rc = lower()) || (rc = gp_run(d))) break;
        float ms = 0.f;
        if (hipEventRecord(a, d->stream) != hipSuccess) {
          rc = hip_fail(hipGetLastError(), "hipEventRecord");
          break;
        }
        for (int k = 0; k < iters && rc == GP_OK; k++) rc = gp_run(d);
        if (rc) break;
        if (hipEventRecord(b, d->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
            hipEventElapsedTime(&ms, a, b) != hipSuccess) {
          rc = hip_fail(hipGetLastError(), "timing the candidates");
          break;
        }
        const double per = double(ms) / iters;
        if (best.ms < 0 || per < best.ms) {
          best.ms = per;
          best.fault_cost = c;
          best.sweep_block = blk == 0 ? 1024 : 256;
        }
      }
    }
    // the grouping for the chosen stage-1 split: the mode the size picks, the
    // full radix sort, and the 65,536 buckets; a mode whose runs raise a
    // device flag (a bucket over its LDS capacity, a look-back give-up) would
    // need a re-run at fetch time and is not a candidate
    const uint32_t saved_sort = d->sort_mode;
    best.grouping = int32_t(gp::SORT_AUTO);
    if (rc == GP_OK) {
      d->fault_cost = best.fault_cost;
      d->sweep_shape = best.sweep_block == 256 ? 2u : 1u;
      rc = lower();
    }
    double auto_ms = -1.0;
    for (uint32_t mode : {uint32_t(gp::SORT_AUTO), uint32_t(gp::SORT_FULL), uint32_t(gp::SORT_BUCKET16)}) {
      if (rc) break;
      d->sort_mode = mode;
      uint32_t seen = 0;
      if ((rc = gp_debug_device_flags_impl(d, nullptr, nullptr, 1)) || (rc = gp_run(d))) break;
      float ms = 0.f;
      if (hipEventRecord(a, d->stream) != hipSuccess) {
        rc = hip_fail(hipGetLastError(), "hipEventRecord");
        break;
      }
      for (int k = 0; k < iters && rc == GP_OK; k++) rc = gp_run(d);
      if (rc) break;
      if (hipEventRecord(b, d->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
          hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        rc = hip_fail(hipGetLastError(), "timing the groupings");
        break;
      }
      if ((rc = gp_debug_device_flags_impl(d, nullptr, &seen, 1))) break;
      const double per = double(ms) / iters;
      if (mode == gp::SORT_AUTO) auto_ms = per;
      if (seen & (gp::FLAG_BUCKET | gp::FLAG_LOOKBACK | gp::FLAG_COLLISION)) continue;
      if (mode == gp::SORT_AUTO || per < best.ms) {
        best.ms = per;
        best.grouping = int32_t(mode);
      }
    }
    (void)auto_ms;
    d->sort_mode = saved_sort;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  d->lowered = false;  // the tables hold the last candidate's lowering
  d->ran = false;
  d->structured = false;
  if (rc) {
    d->fault_cost = saved_cost;
    d->sweep_shape = saved_shape;
    return rc;
  }
  d->fault_cost = best.fault_cost;
  d->sweep_shape = best.sweep_block == 256 ? 2u : 1u;
  d->sort_mode = uint32_t(best.grouping);
  if (!best.cached) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[tune_key(best)] = best;
  }
  if (out) *out = best;
  return GP_OK;
}

}  // namespace

extern "C" {

static int gp_autotune_impl(gp_driver* d, const char* text, size_t len, int iters, gp_tuning* out) {
  if (!d || !text) return fail(GP_E_ARG, "null argument");
  return autotune(d, [&]() { return gp_lower(d, text, len, nullptr, 0); }, iters, out);
}

static int gp_autotune_batch_impl(gp_driver* d, const char* const* texts, const size_t* lens, size_t n, int iters,
                      gp_tuning* out) {
  if (!d || !texts || !lens) return fail(GP_E_ARG, "null argument");
  return autotune(d, [&]() { return gp_lower_batch(d, texts, lens, nullptr, nullptr, n); }, iters, out);
}

size_t gp_tuning_cache_size(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  return g_tune.size();
}

int gp_tuning_cache_get(size_t i, gp_tuning* out) {
  if (!out) return fail(GP_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(g_tune_mu);
  if (i >= g_tune.size()) return fail(GP_E_ARG, "cache index out of range");
  auto it = g_tune.begin();
  std::advance(it, i);
  *out = it->second;
  out->cached = 1;
  return GP_OK;
}

static int gp_tuning_cache_put_impl(const gp_tuning* t) {
  if (!t) return fail(GP_E_ARG, "null argument");
  if (!(t->fault_cost > 0.0 && t->fault_cost < 1.0)) return fail(GP_E_ARG, "fault cost must lie in (0, 1)");
  if (t->sweep_block != 256 && t->sweep_block != 1024) return fail(GP_E_ARG, "sweep work-group must be 256 or 1024");
  if (t->level > 2) return fail(GP_E_ARG, "correlation level must be 0, 1 or 2");
  if (t->grouping < 0 || t->grouping > 2) return fail(GP_E_ARG, "grouping must be 0, 1 or 2");
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[tune_key(*t)] = *t;
  return GP_OK;
}

int gp_debug_set_sweep_shape(gp_driver* d, int shape) {
  if (!d) return fail(GP_E_ARG, "null driver");
  if (shape < 0 || shape > 2) return fail(GP_E_ARG, "sweep shape must be 0, 1 or 2");
  d->sweep_shape = uint32_t(shape);
  return GP_OK;
}

int gp_debug_set_graph(gp_driver* d, int enable) {
  if (!d) return fail(GP_E_ARG, "null driver");
  d->use_graph = enable != 0;
  return GP_OK;
}

static int gp_sync_impl(gp_driver* d) {
  if (!d) return fail(GP_E_ARG, "null driver");
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  collect_timing(d);
  return GP_OK;
}

// A fetched compile in the pinned staging buffer.
struct Staged {
  uint64_t U = 0, nb = 0;
  const uint32_t* off32 = nullptr;
  const uint32_t* bits32 = nullptr;
  const double* q64 = nullptr;
  const uint32_t* c_eoff = nullptr;  // per circuit: its first hyperedge (circuits + 1 entries)
  size_t n_circuits = 0;
  std::chrono::steady_clock::time_point t_ready;   // when the compile was seen finished
  std::chrono::steady_clock::time_point t_loaded;  // when the download had finished
};

// Wait for the compile (redoing it for the retry flags), check the device
// flags and download the hyperedges into the pinned staging buffer.
static int fetch_staged(gp_driver* d, Staged& out) {
  if (!d->ran) return fail(GP_E_STATE, "gp_fetch before gp_run");
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  HIP_TRY(hipMemcpyAsync(d->h_hdr, d->st.hdr, sizeof(gp::DevHeader), hipMemcpyDeviceToHost, d->stream),
          "download header");
  HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  collect_timing(d);
  gp::DevHeader hdr = *d->h_hdr;
  out.t_ready = std::chrono::steady_clock::now();
  // at most three more compiles: a sort tile that gave up waiting for its
  // predecessor (never expected) runs the same compile once more; a bucket
  // too large for LDS redoes the grouping with the full radix sort; two
  // signatures under one key redo it keyed on both hashes (which always takes
  // the full sort)
  bool lookback_redone = false;
  for (int attempt = 0; attempt < 3 && !(hdr.flags & gp::FLAG_GAUGE); attempt++) {
    if (hdr.flags & gp::FLAG_LOOKBACK) {
      if (lookback_redone) break;
      lookback_redone = true;
      d->lookback_retries++;
    } else if (hdr.flags & gp::FLAG_BUCKET) {
      d->bucket_retries++;
      d->st.sort_mode = gp::SORT_FULL;
    } else if ((hdr.flags & gp::FLAG_COLLISION) && d->st.key_mode == 0) {
      d->collision_retries++;
      d->st.key_mode = 1;
    } else {
      break;
    }
    gp::LaunchHook none;
    hipError_t e = gp::enqueue_compile(d->st, d->stream, none);
    if (e != hipSuccess) {
      d->st.key_mode = 0;
      d->st.sort_mode = d->sort_mode;
      return hip_fail(e, "kernel launch");
    }
    HIP_TRY(hipMemcpyAsync(d->h_hdr, d->st.hdr, sizeof(gp::DevHeader), hipMemcpyDeviceToHost, d->stream),
            "download header");
    HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
    hdr = *d->h_hdr;
  }
  d->st.key_mode = 0;
  d->st.sort_mode = d->sort_mode;
  if (hdr.flags & gp::FLAG_LOOKBACK)
    return fail(GP_E_HIP, "a radix-sort tile gave up waiting for its predecessor, again after a re-run "
                          "(the grouping was abandoned; no result)");
  if (hdr.flags & gp::FLAG_BUCKET) return fail(GP_E_HIP, "bucket grouping overflow after the full-sort retry");
  if (hdr.flags & gp::FLAG_GAUGE)
    return fail(GP_E_NONDETERMINISTIC,
                "a detector or observable is sensitive to an error right after a reset or measurement "
                "(or at the start), so it is not deterministic");
  if (hdr.flags & gp::FLAG_COLLISION)
    return fail(GP_E_COLLISION, "two different signatures share both 64-bit hashes");
  if ((hdr.flags & gp::FLAG_OVERFLOW) || hdr.n_bits > d->bits_cap)
    return fail(GP_E_BOUNDS, "hyperedge signature bits exceed the driver's output capacity");
  const uint64_t U = hdr.n_edges;
  const uint64_t nb = hdr.n_bits;
  char* h = static_cast<char*>(d->h_out);
  const size_t o_off = 0, o_bits = align_up((U + 1) * 4), o_q = o_bits + align_up(nb * 4);
  const size_t o_c = o_q + align_up(U * 8);
  const size_t B = d->lw.branches.size();
  if (o_c + (B + 1) * 4 > d->h_out_cap) return fail(GP_E_BOUNDS, "result exceeds the download staging buffer");
  HIP_TRY(hipMemcpyAsync(h + o_off, d->st.edge_off32, (U + 1) * 4, hipMemcpyDeviceToHost, d->stream), "download");
  if (nb) HIP_TRY(hipMemcpyAsync(h + o_bits, d->st.edge_bits, nb * 4, hipMemcpyDeviceToHost, d->stream), "download");
  if (U) HIP_TRY(hipMemcpyAsync(h + o_q, d->st.edge_q, U * 8, hipMemcpyDeviceToHost, d->stream), "download");
  HIP_TRY(hipMemcpyAsync(h + o_c, d->st.circ_eoff, (B + 1) * 4, hipMemcpyDeviceToHost, d->stream), "download");
  HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  out.t_loaded = std::chrono::steady_clock::now();
  out.U = U;
  out.nb = nb;
  out.off32 = reinterpret_cast<const uint32_t*>(h + o_off);
  out.bits32 = reinterpret_cast<const uint32_t*>(h + o_bits);
  out.q64 = reinterpret_cast<const double*>(h + o_q);
  out.c_eoff = reinterpret_cast<const uint32_t*>(h + o_c);
  out.n_circuits = B;
  // the hyperedges are listed circuit by circuit: the offsets must rise to U
  if (out.c_eoff[0] != 0 || out.c_eoff[B] != U)
    return fail(GP_E_HIP, "the per-circuit hyperedge offsets do not cover the result");
  for (size_t k = 0; k < B; k++)
    if (out.c_eoff[k + 1] < out.c_eoff[k]) return fail(GP_E_HIP, "the per-circuit hyperedge offsets decrease");
  return GP_OK;
}

static int gp_fetch_sizes_impl(gp_driver* d, uint64_t* n_edges, uint64_t* n_bits, uint32_t* n_det, uint32_t* n_obs) {
  if (!d || !n_edges || !n_bits) return fail(GP_E_ARG, "null argument");
  d->staged_ok = false;
  Staged sg;
  int rc = fetch_staged(d, sg);
  if (rc) return rc;
  d->staged_U = sg.U;
  d->staged_nb = sg.nb;
  d->staged_off = sg.off32;
  d->staged_bits = sg.bits32;
  d->staged_q = sg.q64;
  d->staged_ceoff = sg.c_eoff;
  d->staged_ok = true;
  d->structured = true;
  d->struct_edges = sg.U;
  d->struct_id++;
  *n_edges = sg.U;
  *n_bits = sg.nb;
  if (n_det) *n_det = d->lw.n_det;
  if (n_obs) *n_obs = d->lw.n_obs;
  return GP_OK;
}

static int gp_fetch_circuit_offsets_impl(gp_driver* d, uint64_t* circuit_offsets) {
  if (!d || !circuit_offsets) return fail(GP_E_ARG, "null argument");
  if (!d->staged_ok) return fail(GP_E_STATE, "gp_fetch_circuit_offsets without a current gp_fetch_sizes");
  const size_t B = d->lw.branches.size();
  for (size_t k = 0; k <= B; k++) circuit_offsets[k] = d->staged_ceoff[k];
  return GP_OK;
}

static int gp_fetch_copy_impl(gp_driver* d, uint64_t* offsets, uint32_t* bits, double* q) {
  if (!d || !offsets) return fail(GP_E_ARG, "null argument");
  if (!d->staged_ok) return fail(GP_E_STATE, "gp_fetch_copy without a current gp_fetch_sizes");
  if ((!bits && d->staged_nb) || (!q && d->staged_U)) return fail(GP_E_ARG, "null argument");
  const uint64_t U = d->staged_U, nb = d->staged_nb;
  const size_t T = split_threads(U + nb / 2);
  run_threads(T, [&](size_t t) {
    for (uint64_t i = (U + 1) * t / T; i < (U + 1) * (t + 1) / T; i++) offsets[i] = d->staged_off[i];
    const uint64_t b0 = nb * t / T, b1 = nb * (t + 1) / T;
    if (b1 > b0) std::memcpy(bits + b0, d->staged_bits + b0, size_t(b1 - b0) * 4);
    const uint64_t q0 = U * t / T, q1 = U * (t + 1) / T;
    if (q1 > q0) std::memcpy(q + q0, d->staged_q + q0, size_t(q1 - q0) * 8);
  });
  return GP_OK;
}

static int gp_fetch_impl(gp_driver* d, gp_edges** out) {
  if (!d || !out) return fail(GP_E_ARG, "null argument");
  *out = nullptr;
  d->staged_ok = false;
  Staged sg;
  int rc = fetch_staged(d, sg);
  if (rc) return rc;
  const uint64_t U = sg.U, nb = sg.nb;
  const uint32_t* off32 = sg.off32;
  const uint32_t* bits32 = sg.bits32;
  const double* q64 = sg.q64;
  gp_edges* e = new gp_edges();
  e->n_det = d->lw.n_det;
  e->n_obs = d->lw.n_obs;
  const size_t B = d->lw.branches.size();
  for (const gp::BranchDesc& bd : d->lw.branches) {
    e->c_det.push_back(bd.n_det);
    e->c_obs.push_back(bd.n_obs);
  }
  // the device lists the hyperedges circuit by circuit (representative
  // position order): copied as they are, on host threads
  e->c_off.resize(B + 1);
  for (size_t k = 0; k <= B; k++) e->c_off[k] = sg.c_eoff[k];
  e->off.resize(U + 1);
  e->bits.resize(nb);
  e->q.resize(U);
  e->circuit.resize(U);
  const size_t T = split_threads(U + nb / 2);
  run_threads(T, [&](size_t t) {
    for (uint64_t i = (U + 1) * t / T; i < (U + 1) * (t + 1) / T; i++) e->off[i] = off32[i];
    const uint64_t b0 = nb * t / T, b1 = nb * (t + 1) / T;
    if (b1 > b0) std::memcpy(e->bits.data() + b0, bits32 + b0, size_t(b1 - b0) * 4);
    const uint64_t q0 = U * t / T, q1 = U * (t + 1) / T;
    if (q1 > q0) std::memcpy(e->q.data() + q0, q64 + q0, size_t(q1 - q0) * 8);
    for (size_t k = 0; k < B; k++) {
      const uint64_t a = std::max<uint64_t>(e->c_off[k], q0), z = std::min<uint64_t>(e->c_off[k + 1], q1);
      if (z > a) std::fill(e->circuit.begin() + a, e->circuit.begin() + z, uint32_t(k));
    }
  });
  *out = e;
  d->structured = true;
  d->struct_edges = U;
  d->struct_id++;
  return GP_OK;
}

static int gp_refresh_rates_impl(gp_driver* d, const double* rates, size_t n_rates) {
  if (!d || !rates) return fail(GP_E_ARG, "null argument");
  if (!d->structured) return fail(GP_E_STATE, "gp_refresh_rates before a fetched compile of this circuit");
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  // the pinned table buffer may still be read by an earlier upload
  HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  gp::Lowered& lw = d->lw;
  const std::vector<double> old = lw.chan_rate;
  gp::LowerError err{};
  int rc = gp::apply_rates(lw, rates, n_rates, err);
  if (rc) {
    lw.chan_rate = old;
    return fail(rc, err.msg);
  }
  TableLayout tl = layout_for(sizes_of(lw));
  const size_t bytes = lw.chan_rate.size() * 8;
  if (bytes) {
    std::memcpy(d->h_tables + tl.chan_rate, lw.chan_rate.data(), bytes);
    HIP_TRY(hipMemcpyAsync(d->d_tables + tl.chan_rate, d->h_tables + tl.chan_rate, bytes, hipMemcpyHostToDevice,
                           d->stream),
            "upload rates");
  }
  HIP_TRY(gp::enqueue_refresh(d->st, uint32_t(d->struct_edges), d->stream), "kernel launch");
  return GP_OK;
}

static int gp_rates_gradient_impl(gp_driver* d, const double* dl_dq, size_t n_edges, double* dl_dr, size_t n_rates) {
  if (!d || (!dl_dq && n_edges) || (!dl_dr && n_rates)) return fail(GP_E_ARG, "null argument");
  if (!d->structured) return fail(GP_E_STATE, "gp_rates_gradient before a fetched compile of this circuit");
  if (n_edges != d->struct_edges) return fail(GP_E_ARG, "dl_dq length differs from the hyperedge count");
  const gp::Lowered& lw = d->lw;
  const size_t C = lw.chan_kind.size();
  if (n_rates != C) return fail(GP_E_ARG, "dl_dr length differs from the channel count");
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  if (n_edges)
    HIP_TRY(hipMemcpyAsync(d->st.gq, dl_dq, n_edges * 8, hipMemcpyHostToDevice, d->stream), "upload dL/dq");
  HIP_TRY(gp::enqueue_rates_gradient(d->st, uint32_t(n_edges), d->stream), "kernel launch");
  std::vector<double> g(C);
  if (C) HIP_TRY(hipMemcpyAsync(g.data(), d->st.gr, C * 8, hipMemcpyDeviceToHost, d->stream), "download dL/dr");
  HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  // lowered channel order -> program order
  for (size_t c = 0; c < C; c++) dl_dr[lw.chan_src[c]] = g[c];
  return GP_OK;
}

// Runs `enqueue(stream)` on the caller's stream (NULL: the driver's), ordered
// after everything already enqueued on the driver's stream and before
// everything enqueued there later.
extern "C++" template <typename Enqueue>
static int on_caller_stream(gp_driver* d, void* stream, Enqueue&& enqueue) {
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : d->stream;
  if (s != d->stream) {
    HIP_TRY(hipEventRecord(d->ev_drv, d->stream), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(s, d->ev_drv, 0), "hipStreamWaitEvent");
  }
  HIP_TRY(enqueue(s), "kernel launch");
  if (s != d->stream) {
    HIP_TRY(hipEventRecord(d->ev_user, s), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(d->stream, d->ev_user, 0), "hipStreamWaitEvent");
  }
  return GP_OK;
}

static int gp_aggregate_impl(gp_driver* d, const double* d_rates, size_t n_rates, double* d_q, size_t n_edges,
                             void* stream) {
  if (!d || (!d_rates && n_rates) || (!d_q && n_edges)) return fail(GP_E_ARG, "null argument");
  if (!d->structured) return fail(GP_E_STATE, "gp_aggregate before a fetched compile");
  if (n_edges != d->struct_edges) return fail(GP_E_ARG, "q length differs from the hyperedge count");
  if (n_rates != d->lw.chan_kind.size()) return fail(GP_E_ARG, "rate array length differs from the channel count");
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  return on_caller_stream(d, stream, [&](hipStream_t s) {
    return gp::enqueue_aggregate(d->st, uint32_t(n_edges), d_rates, d_q, s);
  });
}

static int gp_aggregate_backward_impl(gp_driver* d, const double* d_rates, size_t n_rates, const double* d_gq,
                                      size_t n_edges, double* d_grates, void* stream) {
  if (!d || (!d_rates && n_rates) || (!d_gq && n_edges) || (!d_grates && n_rates))
    return fail(GP_E_ARG, "null argument");
  if (!d->structured) return fail(GP_E_STATE, "gp_aggregate_backward before a fetched compile");
  if (n_edges != d->struct_edges) return fail(GP_E_ARG, "dL/dq length differs from the hyperedge count");
  if (n_rates != d->lw.chan_kind.size()) return fail(GP_E_ARG, "rate array length differs from the channel count");
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  return on_caller_stream(d, stream, [&](hipStream_t s) {
    return gp::enqueue_aggregate_backward(d->st, uint32_t(n_edges), d_rates, d_gq, d_grates, nullptr, s);
  });
}

// gp_aggregate_backward with its per-fault dL/dp in the library's static
// device scratch instead of the driver's buffer; nothing is allocated.
static int gp_aggregate_backward_noalloc_impl(gp_driver* d, const double* d_rates, size_t n_rates,
                                              const double* d_gq, size_t n_edges, double* d_grates, void* stream) {
  if (!d || (!d_rates && n_rates) || (!d_gq && n_edges) || (!d_grates && n_rates))
    return fail(GP_E_ARG, "null argument");
  if (!d->structured) return fail(GP_E_STATE, "gp_aggregate_backward_noalloc before a fetched compile");
  if (n_edges != d->struct_edges) return fail(GP_E_ARG, "dL/dq length differs from the hyperedge count");
  if (n_rates != d->lw.chan_kind.size()) return fail(GP_E_ARG, "rate array length differs from the channel count");
  if (d->st.n_faults > gp::kScratchFaults)
    return fail(GP_E_BOUNDS, "the compile has " + std::to_string(d->st.n_faults) +
                                 " faults; the allocation-free adjoint holds at most " +
                                 std::to_string(gp::kScratchFaults));
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  double* scratch = gp::scratch_for(d->device);
  if (!scratch) return fail(GP_E_STATE, "the static scratch of this device has no address");
  return on_caller_stream(d, stream, [&](hipStream_t s) {
    return gp::enqueue_aggregate_backward(d->st, uint32_t(n_edges), d_rates, d_gq, d_grates, scratch, s);
  });
}

static int check_level(int level) {
  return (level < -1 || level > 2) ? fail(GP_E_ARG, "correlation level must be -1 (the driver's), 0, 1 or 2")
                                   : GP_OK;
}

static int gp_compile_hypergraph_impl(gp_driver* d, const char* text, size_t len, const double* rates, size_t n_rates,
                                      int level, gp_edges** out) {
  if (!d || !out) return fail(GP_E_ARG, "null argument");
  int rc = check_level(level);
  if (rc) return rc;
  if ((rc = lower_text_at(d, text, len, rates, n_rates, level < 0 ? d->level : uint32_t(level)))) return rc;
  if ((rc = gp_run(d))) return rc;
  return gp_fetch(d, out);
}

static int gp_compile_ir_impl(gp_driver* d, const gp_circuit_ir* ir, const double* rates, size_t n_rates, int level,
                              gp_edges** out) {
  if (!d || !out) return fail(GP_E_ARG, "null argument");
  int rc = check_level(level);
  if (rc) return rc;
  if ((rc = lower_ir_at(d, ir, rates, n_rates, level < 0 ? d->level : uint32_t(level)))) return rc;
  if ((rc = gp_run(d))) return rc;
  return gp_fetch(d, out);
}

void* gp_driver_stream(gp_driver* d) { return d ? static_cast<void*>(d->stream) : nullptr; }

int gp_circuit_info_get(const gp_driver* d, gp_circuit_info* out) {
  if (!d || !out) return fail(GP_E_ARG, "null argument");
  gp_circuit_info i{};
  const gp::Lowered& lw = d->lw;
  i.n_qubits = lw.n_qubits;
  i.n_layers = lw.n_layers;
  i.n_measurements = lw.n_meas;
  i.n_detectors = lw.n_det;
  i.n_observables = lw.n_obs;
  i.n_words = lw.w;
  i.n_channels = lw.chan_kind.size();
  i.n_faults = lw.n_faults;
  i.n_ops = lw.ops.size();
  i.n_items = lw.item_col.size();
  i.slab_words = lw.slab_words;
  i.n_circuits = uint32_t(lw.branches.size());
  if (d->h_hdr) {
    i.n_classes = d->h_hdr->n_seg;
    i.n_edges = d->h_hdr->n_edges;
    i.n_edge_bits = d->h_hdr->n_bits;
    i.n_live_words = d->h_hdr->n_words;
    i.n_live_faults = d->h_hdr->n_live;
    i.n_nonzero_words = d->h_hdr->n_nz_words;
  }
  *out = i;
  return GP_OK;
}

int gp_circuit_shape(const gp_driver* d, uint32_t circuit, uint32_t* n_det, uint32_t* n_obs) {
  if (!d || !n_det || !n_obs) return fail(GP_E_ARG, "null argument");
  if (circuit >= d->lw.branches.size()) return fail(GP_E_ARG, "circuit index out of range");
  *n_det = d->lw.branches[circuit].n_det;
  *n_obs = d->lw.branches[circuit].n_obs;
  return GP_OK;
}

int gp_set_timing(gp_driver* d, int enable) {
  if (!d) return fail(GP_E_ARG, "null driver");
  d->timing = enable != 0;
  return GP_OK;
}

int gp_reset_timing(gp_driver* d) {
  if (!d) return fail(GP_E_ARG, "null driver");
  for (int k = 0; k < gp::K_COUNT; k++) {
    d->total_ms[k] = 0;
    d->launches[k] = 0;
  }
  return GP_OK;
}

int gp_timing_count(const gp_driver*) { return gp::K_COUNT; }

int gp_debug_set_key_bits(gp_driver* d, int bits) {
  if (!d || bits < 1 || bits > 64) return fail(GP_E_ARG, "key bits must be in [1, 64]");
  d->key_bits = uint32_t(bits);
  return GP_OK;
}

uint64_t gp_debug_collision_retries(const gp_driver* d) { return d ? d->collision_retries : 0; }

int gp_debug_retry_counts(const gp_driver* d, uint64_t* lookback, uint64_t* bucket, uint64_t* collision) {
  if (!d) return fail(GP_E_ARG, "null driver");
  if (lookback) *lookback = d->lookback_retries;
  if (bucket) *bucket = d->bucket_retries;
  if (collision) *collision = d->collision_retries;
  return GP_OK;
}

int gp_debug_set_spin_limit(gp_driver* d, uint32_t limit) {
  if (!d) return fail(GP_E_ARG, "null driver");
  d->spin_limit = limit;
  return GP_OK;
}

static int gp_debug_device_flags_impl(gp_driver* d, uint32_t* flags, uint32_t* flags_seen, int clear_seen) {
  if (!d) return fail(GP_E_ARG, "null driver");
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  HIP_TRY(hipMemcpyAsync(d->h_hdr, d->st.hdr, sizeof(gp::DevHeader), hipMemcpyDeviceToHost, d->stream),
          "download header");
  HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  collect_timing(d);
  if (flags) *flags = d->h_hdr->flags;
  if (flags_seen) *flags_seen = d->h_hdr->flags_seen;
  if (clear_seen) {
    HIP_TRY(hipMemsetAsync(&d->st.hdr->flags_seen, 0, sizeof(uint32_t), d->stream), "clear flags");
    HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  }
  return GP_OK;
}

int gp_set_correlation_level(gp_driver* d, int level) {
  if (!d) return fail(GP_E_ARG, "null driver");
  if (level < 0 || level > 2) return fail(GP_E_ARG, "correlation level must be 0, 1 or 2");
  d->level = uint32_t(level);
  return GP_OK;
}

int gp_debug_set_sort_mode(gp_driver* d, int mode) {
  if (!d) return fail(GP_E_ARG, "null driver");
  if (mode != int(gp::SORT_AUTO) && mode != int(gp::SORT_FULL) && mode != int(gp::SORT_BUCKET16))
    return fail(GP_E_ARG, "sort mode must be 0, 1 or 2");
  d->sort_mode = uint32_t(mode);
  return GP_OK;
}

int gp_debug_capture_keys(gp_driver* d, int enable) {
  if (!d) return fail(GP_E_ARG, "null driver");
  if (enable && !d->key_copy) {
    HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
    if (int rc = dev_alloc(d, &d->key_copy, d->bounds.max_faults, "captured class keys")) return rc;
  }
  d->capture_keys = enable != 0;
  d->captured_faults = 0;
  return GP_OK;
}

int gp_debug_class_keys(gp_driver* d, uint64_t* out, uint64_t cap, uint64_t* n_faults, uint32_t* key_bits) {
  if (!d || !n_faults || (cap && !out)) return fail(GP_E_ARG, "null argument");
  if (!d->capture_keys || !d->ran) return fail(GP_E_STATE, "no compile has run with key capture on");
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  *n_faults = d->captured_faults;
  if (key_bits) *key_bits = d->captured_key_bits;
  const uint64_t m = std::min<uint64_t>(cap, d->captured_faults);
  if (m) HIP_TRY(hipMemcpy(out, d->key_copy, m * 8, hipMemcpyDeviceToHost), "download class keys");
  return GP_OK;
}

int gp_debug_sweep_times(gp_driver* d, uint64_t* out, uint64_t cap, uint64_t* n_items, double* clock_hz) {
  if (!d || !out || !n_items) return fail(GP_E_ARG, "null argument");
  if (!d->ran) return fail(GP_E_STATE, "no compile has run");
  HIP_TRY(hipSetDevice(d->device), "hipSetDevice");
  HIP_TRY(hipStreamSynchronize(d->stream), "hipStreamSynchronize");
  const uint64_t n = d->lw.item_col.size();
  *n_items = n;
  const uint64_t m = std::min<uint64_t>(cap, 2 * n);
  if (m) HIP_TRY(hipMemcpy(out, d->st.item_clock, m * 8, hipMemcpyDeviceToHost), "download item clocks");
  if (clock_hz) {
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, d->device), "clock rate");
    *clock_hz = double(khz) * 1e3;
  }
  return GP_OK;
}

int gp_timing_entry(const gp_driver* d, int index, const char** name, double* total_ms, uint64_t* launches) {
  if (!d || index < 0 || index >= gp::K_COUNT) return fail(GP_E_ARG, "bad timing index");
  if (name) *name = gp::kernel_name(index);
  if (total_ms) *total_ms = d->total_ms[index];
  if (launches) *launches = d->launches[index];
  return GP_OK;
}

// Words per packed signature: enough for the detectors and observables of the
// widest circuit of the result (bit b of a signature: detector b below the
// circuit's detector count D, else observable b - D).
static uint32_t packed_words(const gp_edges* e) {
  uint64_t most = uint64_t(e->n_det) + e->n_obs;
  for (size_t k = 0; k < e->c_det.size(); k++) most = std::max<uint64_t>(most, uint64_t(e->c_det[k]) + e->c_obs[k]);
  return uint32_t((most + 63) / 64);
}

uint32_t gp_edges_words(const gp_edges* e) { return e ? packed_words(e) : 0; }

const uint64_t* gp_edges_signatures(const gp_edges* e) {
  if (!e) {
    fail(GP_E_ARG, "null argument");
    return nullptr;
  }
  gp_edges* m = const_cast<gp_edges*>(e);
  std::call_once(m->words_once, [m] {
    m->words_rc = gp::guarded([m] {
      const uint32_t W = packed_words(m);
      const uint64_t U = m->q.size();
      m->n_words = W;
      m->words.assign(std::max<uint64_t>(U * W, 1), 0ull);
      for (uint64_t k = 0; k < U; k++)
        for (uint64_t i = m->off[k]; i < m->off[k + 1]; i++) {
          const uint32_t b = m->bits[i];
          m->words[k * W + b / 64] |= 1ull << (b % 64);
        }
      return GP_OK;
    });
  });
  if (m->words_rc) {
    fail(m->words_rc, "could not build the packed signatures");
    return nullptr;
  }
  return m->words.data();
}

uint64_t gp_edges_count(const gp_edges* e) { return e ? e->q.size() : 0; }
uint32_t gp_edges_detectors(const gp_edges* e) { return e ? e->n_det : 0; }
uint32_t gp_edges_observables(const gp_edges* e) { return e ? e->n_obs : 0; }
const uint64_t* gp_edges_offsets(const gp_edges* e) { return e ? e->off.data() : nullptr; }
const uint32_t* gp_edges_bits(const gp_edges* e) { return e ? e->bits.data() : nullptr; }
const double* gp_edges_probabilities(const gp_edges* e) { return e ? e->q.data() : nullptr; }
uint32_t gp_edges_circuits(const gp_edges* e) { return e ? uint32_t(e->c_det.size()) : 0; }
const uint32_t* gp_edges_circuit_ids(const gp_edges* e) { return e ? e->circuit.data() : nullptr; }
const uint64_t* gp_edges_circuit_offsets(const gp_edges* e) { return e ? e->c_off.data() : nullptr; }

int gp_edges_circuit_shape(const gp_edges* e, uint32_t k, uint32_t* n_det, uint32_t* n_obs) {
  if (!e) return fail(GP_E_ARG, "null argument");
  if (k >= e->c_det.size()) return fail(GP_E_ARG, "circuit index out of range");
  if (n_det) *n_det = e->c_det[k];
  if (n_obs) *n_obs = e->c_obs[k];
  return GP_OK;
}

static int gp_edges_to_dem_text_impl(const gp_edges* e, char** text, size_t* len) {
  if (!e || !text) return fail(GP_E_ARG, "null argument");
  if (e->c_det.size() > 1) return fail(GP_E_STATE, "a batch result: use gp_edges_circuit_dem_text");
  return gp_edges_circuit_dem_text(e, 0, text, len);
}

static int gp_edges_circuit_dem_text_impl(const gp_edges* e, uint32_t circuit, char** text, size_t* len) {
  if (!e || !text) return fail(GP_E_ARG, "null argument");
  if (circuit >= std::max<size_t>(e->c_det.size(), 1)) return fail(GP_E_ARG, "circuit index out of range");
  const uint32_t n_det = e->c_det.empty() ? e->n_det : e->c_det[circuit];
  std::string s;
  s.reserve(e->q.size() * 32);
  char buf[64];
  for (size_t k = 0; k < e->q.size(); k++) {
    if (e->circuit[k] != circuit) continue;
    std::snprintf(buf, sizeof buf, "error(%.17g)", e->q[k]);
    s += buf;
    for (uint64_t i = e->off[k]; i < e->off[k + 1]; i++) {
      uint32_t b = e->bits[i];
      if (b < n_det)
        std::snprintf(buf, sizeof buf, " D%u", b);
      else
        std::snprintf(buf, sizeof buf, " L%u", b - n_det);
      s += buf;
    }
    s += '\n';
  }
  char* out = static_cast<char*>(std::malloc(s.size() + 1));
  if (!out) return fail(GP_E_OOM, "out of memory");
  std::memcpy(out, s.data(), s.size() + 1);
  *text = out;
  if (len) *len = s.size();
  return GP_OK;
}

void gp_edges_free(gp_edges* e) { delete e; }
void gp_free(void* p) { std::free(p); }

// ---- exported entry points: the bodies above run under gp::guarded, so no
// C++ exception (an allocation failure while lowering, splitting or copying a
// result) crosses the C ABI

#define GP_GUARD(call) gp::guarded([&] { return call; })

int gp_bounds_from_circuit(const char* text, size_t len, gp_bounds* out) {
  return GP_GUARD(gp_bounds_from_circuit_impl(text, len, out));
}
int gp_driver_create(const gp_bounds* bounds, int device, gp_driver** out) {
  return GP_GUARD(gp_driver_create_impl(bounds, device, out));
}
int gp_driver_create_from_circuit(const char* text, size_t len, int device, gp_driver** out) {
  return GP_GUARD(gp_driver_create_from_circuit_impl(text, len, device, out));
}
int gp_bounds_from_batch(const char* const* texts, const size_t* lens, size_t n, gp_bounds* out) {
  return GP_GUARD(gp_bounds_from_batch_impl(texts, lens, n, out));
}
int gp_driver_create_from_batch(const char* const* texts, const size_t* lens, size_t n, int device,
                                gp_driver** out) {
  return GP_GUARD(gp_driver_create_from_batch_impl(texts, lens, n, device, out));
}
int gp_lower(gp_driver* d, const char* text, size_t len, const double* rates, size_t n_rates) {
  return GP_GUARD(gp_lower_impl(d, text, len, rates, n_rates));
}
int gp_lower_batch(gp_driver* d, const char* const* texts, const size_t* lens, const double* const* rates,
                   const size_t* n_rates, size_t n) {
  return GP_GUARD(gp_lower_batch_impl(d, texts, lens, rates, n_rates, n));
}
int gp_run(gp_driver* d) { return GP_GUARD(gp_run_impl(d)); }
int gp_autotune(gp_driver* d, const char* text, size_t len, int iters, gp_tuning* out) {
  return GP_GUARD(gp_autotune_impl(d, text, len, iters, out));
}
int gp_autotune_batch(gp_driver* d, const char* const* texts, const size_t* lens, size_t n, int iters,
                      gp_tuning* out) {
  return GP_GUARD(gp_autotune_batch_impl(d, texts, lens, n, iters, out));
}
int gp_tuning_cache_put(const gp_tuning* t) { return GP_GUARD(gp_tuning_cache_put_impl(t)); }
int gp_sync(gp_driver* d) { return GP_GUARD(gp_sync_impl(d)); }
int gp_fetch_sizes(gp_driver* d, uint64_t* n_edges, uint64_t* n_bits, uint32_t* n_det, uint32_t* n_obs) {
  return GP_GUARD(gp_fetch_sizes_impl(d, n_edges, n_bits, n_det, n_obs));
}
int gp_fetch_circuit_offsets(gp_driver* d, uint64_t* circuit_offsets) {
  return GP_GUARD(gp_fetch_circuit_offsets_impl(d, circuit_offsets));
}
int gp_fetch_copy(gp_driver* d, uint64_t* offsets, uint32_t* bits, double* q) {
  return GP_GUARD(gp_fetch_copy_impl(d, offsets, bits, q));
}
int gp_fetch(gp_driver* d, gp_edges** out) { return GP_GUARD(gp_fetch_impl(d, out)); }
int gp_refresh_rates(gp_driver* d, const double* rates, size_t n_rates) {
  return GP_GUARD(gp_refresh_rates_impl(d, rates, n_rates));
}
int gp_rates_gradient(gp_driver* d, const double* dl_dq, size_t n_edges, double* dl_dr, size_t n_rates) {
  return GP_GUARD(gp_rates_gradient_impl(d, dl_dq, n_edges, dl_dr, n_rates));
}
int gp_compile_hypergraph(gp_driver* d, const char* text, size_t len, const double* rates, size_t n_rates,
                          int level, gp_edges** out) {
  return GP_GUARD(gp_compile_hypergraph_impl(d, text, len, rates, n_rates, level, out));
}
int gp_compile_ir(gp_driver* d, const gp_circuit_ir* ir, const double* rates, size_t n_rates, int level,
                  gp_edges** out) {
  return GP_GUARD(gp_compile_ir_impl(d, ir, rates, n_rates, level, out));
}
int gp_bounds_from_ir(const gp_circuit_ir* ir, gp_bounds* out) { return GP_GUARD(gp_bounds_from_ir_impl(ir, out)); }
int gp_bounds_from_batch_ir(const gp_circuit_ir* irs, size_t n, gp_bounds* out) {
  return GP_GUARD(gp_bounds_from_batch_ir_impl(irs, n, out));
}
int gp_lower_ir(gp_driver* d, const gp_circuit_ir* ir, const double* rates, size_t n_rates) {
  return GP_GUARD(gp_lower_ir_impl(d, ir, rates, n_rates));
}
int gp_lower_batch_ir(gp_driver* d, const gp_circuit_ir* irs, size_t n, const double* const* rates,
                      const size_t* n_rates) {
  return GP_GUARD(gp_lower_batch_ir_impl(d, irs, n, rates, n_rates));
}
int gp_edges_to_dem_text(const gp_edges* e, char** text, size_t* len) {
  return GP_GUARD(gp_edges_to_dem_text_impl(e, text, len));
}
int gp_edges_circuit_dem_text(const gp_edges* e, uint32_t circuit, char** text, size_t* len) {
  return GP_GUARD(gp_edges_circuit_dem_text_impl(e, circuit, text, len));
}
int gp_debug_device_flags(gp_driver* d, uint32_t* flags, uint32_t* flags_seen, int clear_seen) {
  return GP_GUARD(gp_debug_device_flags_impl(d, flags, flags_seen, clear_seen));
}
int gp_aggregate(gp_driver* d, const double* d_rates, size_t n_rates, double* d_q, size_t n_edges, void* stream) {
  return GP_GUARD(gp_aggregate_impl(d, d_rates, n_rates, d_q, n_edges, stream));
}
int gp_aggregate_backward(gp_driver* d, const double* d_rates, size_t n_rates, const double* d_gq, size_t n_edges,
                          double* d_grates, void* stream) {
  return GP_GUARD(gp_aggregate_backward_impl(d, d_rates, n_rates, d_gq, n_edges, d_grates, stream));
}
int gp_aggregate_backward_noalloc(gp_driver* d, const double* d_rates, size_t n_rates, const double* d_gq,
                                  size_t n_edges, double* d_grates, void* stream) {
  return GP_GUARD(gp_aggregate_backward_noalloc_impl(d, d_rates, n_rates, d_gq, n_edges, d_grates, stream));
}
uint64_t gp_structure_id(const gp_driver* d) { return d && d->structured ? d->struct_id : 0; }

#undef GP_GUARD

}  // extern "C"

namespace gp {

int driver_upload_parts(gp_driver* d, const std::vector<const Lowered*>& parts) {
  if (!d || parts.empty()) return fail(GP_E_ARG, "a batch needs a driver and at least one circuit");
  d->lowered = false;
  d->ran = false;
  d->structured = false;
  return guarded([&] {
    merge_branches(parts, d->lw);
    return upload_lowered(d);
  });
}

uint32_t driver_level(const gp_driver* d) { return d ? d->level : 2u; }

static int driver_fetch_split_impl(gp_driver* d, std::vector<gp_edges*>& out, uint64_t* wait_ns);

int driver_fetch_split(gp_driver* d, std::vector<gp_edges*>& out, uint64_t* wait_ns) {
  const int rc = guarded([&] { return driver_fetch_split_impl(d, out, wait_ns); });
  if (rc) {
    // a failure part way through frees the results made so far
    for (gp_edges* e : out) delete e;
    out.clear();
  }
  return rc;
}

static int driver_fetch_split_impl(gp_driver* d, std::vector<gp_edges*>& out, uint64_t* wait_ns) {
  out.clear();
  if (!d) return fail(GP_E_ARG, "null driver");
  const auto t0 = std::chrono::steady_clock::now();
  Staged sg;
  sg.t_ready = sg.t_loaded = t0;
  d->staged_ok = false;
  int rc = fetch_staged(d, sg);
  if (wait_ns) {
    wait_ns[0] = uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(sg.t_ready - t0).count());
    wait_ns[1] = uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(sg.t_loaded - sg.t_ready).count());
  }
  if (rc) return rc;
  // the results leave with the requests: no refresh or adjoint on this compile
  d->structured = false;
  const size_t B = d->lw.branches.size();
  if (sg.n_circuits != B) return fail(GP_E_INTERNAL, "circuit count of the staged result");
  // the device lists the hyperedges circuit by circuit: each circuit's are a
  // contiguous range, copied into its own result (on host threads, which
  // also allocate and first touch the results)
  out.resize(B);
  const size_t T = std::min<size_t>(split_threads(sg.U + sg.nb / 2), std::max<size_t>(B, 1));
  std::vector<int> oom(T, 0);
  run_threads(T, [&](size_t t) {
    for (size_t k = t; k < B; k += T) {
      const uint64_t e0 = sg.c_eoff[k], e1 = sg.c_eoff[k + 1];
      const uint64_t b0 = sg.off32[e0], b1 = sg.off32[e1];
      gp_edges* e = nullptr;
      try {
        e = new gp_edges();
        e->n_det = d->lw.branches[k].n_det;
        e->n_obs = d->lw.branches[k].n_obs;
        e->off.resize(e1 - e0 + 1);
        for (uint64_t i = e0; i <= e1; i++) e->off[i - e0] = sg.off32[i] - b0;
        e->bits.assign(sg.bits32 + b0, sg.bits32 + b1);
        e->q.assign(sg.q64 + e0, sg.q64 + e1);
        e->circuit.assign(e1 - e0, 0u);
        e->c_det.assign(1, e->n_det);
        e->c_obs.assign(1, e->n_obs);
        e->c_off = {0, e1 - e0};
      } catch (const std::bad_alloc&) {
        delete e;
        e = nullptr;
        oom[t] = 1;
      }
      out[k] = e;
    }
  });
  for (int v : oom)
    if (v) return fail(GP_E_OOM, "host allocation of a split result failed");
  return GP_OK;
}

int set_last_error(int code, const char* msg) noexcept { return fail(code, msg); }

}  // namespace gp
