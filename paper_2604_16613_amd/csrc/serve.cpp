// Request server: continuous batching over two drivers (C ABI in gp.h).
//
// Submitted circuits are lowered at once by a pool of host threads. A worker
// thread owns two drivers of identical bounds, each with its own HIP stream.
// Every pass it takes the lowered requests (up to the batch size the bounds
// allow), uploads them as one batch to the free driver and launches both
// stages there; while that batch runs on the device it downloads the other
// driver's finished batch and completes its requests, each with its own
// circuit's hyperedges.
// Requests never share a hyperedge (a batch groups every circuit on its own),
// so a request's result does not depend on what it was batched with.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "driver_internal.h"
#include "gp.h"
#include "lower.h"

namespace {

uint64_t now_ns() {
  return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                      std::chrono::steady_clock::now().time_since_epoch()).count());
}

struct Request {
  uint64_t ticket = 0;
  std::string text;
  // a circuit submitted in binary form: its arrays, copied
  bool is_ir = false;
  uint64_t ir_n_ops = 0;
  std::vector<uint8_t> ir_code;
  std::vector<uint32_t> ir_q0, ir_q1, ir_rec;
  std::vector<double> ir_rate;
  std::vector<double> rates;
  bool has_rates = false;
  uint64_t t_submit = 0, t_done = 0;
  bool lowered = false;
  bool solo = false;  // failed inside a batch: runs alone next, to find whose error it was
  gp::Lowered lw;
  bool done = false;
  int rc = GP_OK;
  std::string msg;
  gp_edges* edges = nullptr;
  uint64_t held = 0;  // host bytes counted against the admission limit
};

using ReqPtr = std::shared_ptr<Request>;

}  // namespace

struct gp_server {
  gp_bounds bounds{};
  gp_driver* drv[2] = {nullptr, nullptr};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ReqPtr> to_lower;  // submitted, waiting for a lowering thread
  std::condition_variable cv_lower;
  std::vector<std::thread> lowerers;
  bool lowerers_done = false;
  std::deque<ReqPtr> pending;   // lowered, waiting for a batch
  std::unordered_map<uint64_t, ReqPtr> live;  // submitted and not yet collected
  uint64_t max_live = 4096, max_bytes = uint64_t(4) << 30;  // admission limits
  uint64_t live_bytes = 0;                                    // host bytes of the live requests
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  uint64_t n_batches = 0, n_requests = 0, max_batch = 0;
  uint64_t ns_lower = 0, ns_upload = 0, ns_fetch = 0, ns_wait = 0, ns_download = 0;  // worker time per phase
};

namespace {

void complete(gp_server* s, const ReqPtr& r, int rc, const std::string& msg, gp_edges* e) {
  std::lock_guard<std::mutex> lk(s->mu);
  r->rc = rc;
  try {
    r->msg = msg;
  } catch (...) {
    // no memory for the message: the status alone reports the failure
  }
  r->edges = e;
  r->t_done = now_ns();
  r->done = true;
  // the result counts against the byte limit until it is collected
  uint64_t rb = msg.size();
  if (e) {
    const uint64_t U = gp_edges_count(e);
    rb += U * (8 + 8 + 4) + (U ? gp_edges_offsets(e)[U] * 4 : 0);
  }
  r->held += rb;
  s->live_bytes += rb;
  r->lw = gp::Lowered();  // the tables are no longer needed
  s->cv_done.notify_all();
}

// A lowering thread: lowers submitted requests one at a time and hands them
// to the worker.
void lower_loop(gp_server* s, uint32_t level) {
  // sweep slots per circuit: batches under load hold a few circuits
  const uint32_t slots = std::max<uint32_t>(1, gp::kSweepSlots / 4);
  for (;;) {
    ReqPtr r;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_lower.wait(lk, [&] { return s->stop || !s->to_lower.empty(); });
      if (s->to_lower.empty()) return;  // stopping, and nothing left
      r = s->to_lower.front();
      s->to_lower.pop_front();
    }
    const uint64_t t0 = now_ns();
    gp::LowerError err{};
    int rc;
    try {
      const double* rates = r->has_rates ? r->rates.data() : nullptr;
      const size_t n_rates = r->has_rates ? r->rates.size() : 0;
      if (r->is_ir) {
        gp_circuit_ir ir{};
        ir.n_ops = r->ir_n_ops;
        ir.code = r->ir_code.empty() ? nullptr : r->ir_code.data();
        ir.q0 = r->ir_q0.empty() ? nullptr : r->ir_q0.data();
        ir.q1 = r->ir_q1.empty() ? nullptr : r->ir_q1.data();
        ir.rate = r->ir_rate.empty() ? nullptr : r->ir_rate.data();
        ir.n_rec = r->ir_rec.size();
        ir.rec = r->ir_rec.empty() ? nullptr : r->ir_rec.data();
        rc = gp::lower_ir(ir, rates, n_rates, slots, r->lw, err, level);
      } else {
        rc = gp::lower_circuit(r->text.data(), r->text.size(), rates, n_rates, slots, r->lw, err, level);
      }
    } catch (...) {
      // nothing may leave this thread: the request fails on its own
      r->lw = gp::Lowered();
      rc = GP_E_OOM;
      err.msg.clear();
    }
    r->lowered = true;
    if (rc) {
      complete(s, r, rc, rc == GP_E_OOM && err.msg.empty() ? "host memory allocation failed while lowering" : err.msg,
               nullptr);
    } else {
      bool queued = false;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        try {
          s->pending.push_back(r);
          queued = true;
        } catch (...) {
        }
      }
      if (!queued) complete(s, r, GP_E_OOM, "host memory allocation failed while queueing", nullptr);
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->ns_lower += now_ns() - t0;
    }
    s->cv_work.notify_one();
  }
}

// Download a driver's finished batch and complete its requests.
void finish(gp_server* s, int slot, std::vector<ReqPtr>& batch) {
  if (batch.empty()) return;
  const uint64_t t0 = now_ns();
  std::vector<gp_edges*> parts;
  uint64_t wait[2] = {0, 0};
  int rc = gp::driver_fetch_split(s->drv[slot], parts, wait);
  if (rc && batch.size() > 1) {
    // a device-side error (e.g. a non-deterministic detector) names no
    // circuit: every request of the batch runs again on its own
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t k = batch.size(); k-- > 0;) {
      batch[k]->solo = true;
      s->pending.push_front(batch[k]);
    }
  } else if (rc) {
    const std::string msg = gp_last_error();
    for (const ReqPtr& r : batch) complete(s, r, rc, msg, nullptr);
  } else {
    for (size_t k = 0; k < batch.size(); k++) {
      if (k < parts.size())
        complete(s, batch[k], GP_OK, "", parts[k]);
      else
        complete(s, batch[k], GP_E_STATE, "result missing for a circuit of the batch", nullptr);
    }
    for (size_t k = batch.size(); k < parts.size(); k++) gp_edges_free(parts[k]);
  }
  batch.clear();
  std::lock_guard<std::mutex> lk(s->mu);
  s->ns_fetch += now_ns() - t0;
  s->ns_wait += wait[0];
  s->ns_download += wait[1];
}

void worker_pass_loop(gp_server* s, std::vector<ReqPtr>* inflight, int& cur, std::vector<ReqPtr>& take,
                      std::vector<ReqPtr>& batch);

// The worker: passes of worker_pass_loop; an exception in a pass (host
// allocation) fails the requests that pass held and the loop goes on.
void worker_loop(gp_server* s) {
  std::vector<ReqPtr> inflight[2];
  int cur = 0;
  for (;;) {
    std::vector<ReqPtr> take, batch;
    try {
      worker_pass_loop(s, inflight, cur, take, batch);
      break;  // the loop ended normally: the server stops
    } catch (...) {
      try {
        for (std::vector<ReqPtr>* v : {&take, &batch})
          for (const ReqPtr& r : *v) {
            bool done;
            {
              std::lock_guard<std::mutex> lk(s->mu);
              done = r->done;
            }
            if (!done) complete(s, r, GP_E_OOM, "host memory allocation failed in the server", nullptr);
          }
      } catch (...) {
        // no memory even for the failure message: the requests stay pending
      }
    }
  }
  finish(s, 0, inflight[0]);
  finish(s, 1, inflight[1]);
}

void worker_pass_loop(gp_server* s, std::vector<ReqPtr>* inflight, int& cur, std::vector<ReqPtr>& take,
                      std::vector<ReqPtr>& batch) {
  const size_t max_batch = std::max<uint32_t>(s->bounds.max_branches, 1);
  for (;;) {
    take.clear();
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(s->mu);
      const bool busy = !inflight[0].empty() || !inflight[1].empty();
      if (!busy) s->cv_work.wait(lk, [&] { return s->lowerers_done || !s->pending.empty(); });
      if (s->pending.empty() && !busy && s->lowerers_done) break;
      while (!s->pending.empty() && take.size() < max_batch) {
        const bool solo = s->pending.front()->solo;
        if (solo && !take.empty()) break;
        take.push_back(s->pending.front());
        s->pending.pop_front();
        if (solo) break;
      }
    }
    batch.swap(take);
    // upload the largest prefix that fits the bounds; the rest waits
    while (!batch.empty()) {
      if (!inflight[cur].empty()) finish(s, cur, inflight[cur]);
      std::vector<const gp::Lowered*> parts;
      for (const ReqPtr& r : batch) parts.push_back(&r->lw);
      const uint64_t u0 = now_ns();
      int rc = gp::driver_upload_parts(s->drv[cur], parts);
      if (rc == GP_OK) rc = gp_run(s->drv[cur]);
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->ns_upload += now_ns() - u0;
      }
      if (rc == GP_OK) break;
      const std::string msg = gp_last_error();
      if (rc != GP_E_BOUNDS || batch.size() == 1) {
        for (const ReqPtr& r : batch) complete(s, r, rc, msg, nullptr);
        batch.clear();
        break;
      }
      const size_t keep = batch.size() / 2;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (size_t k = batch.size(); k-- > keep;) s->pending.push_front(batch[k]);
      }
      batch.resize(keep);
    }
    if (!batch.empty()) {
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->n_batches++;
        s->n_requests += batch.size();
        s->max_batch = std::max<uint64_t>(s->max_batch, batch.size());
      }
      inflight[cur] = std::move(batch);
      // the new batch runs while the older one is downloaded
      finish(s, cur ^ 1, inflight[cur ^ 1]);
      cur ^= 1;
    } else {
      finish(s, cur ^ 1, inflight[cur ^ 1]);
      finish(s, cur, inflight[cur]);
    }
  }
}

}  // namespace

extern "C" {

static int gp_server_create_impl(const gp_bounds* bounds, int device, gp_server** out);
static int gp_server_submit_impl(gp_server* s, const char* text, size_t len, const double* rates, size_t n_rates,
                                 uint64_t* ticket);
static int gp_server_submit_ir_impl(gp_server* s, const gp_circuit_ir* ir, const double* rates, size_t n_rates,
                                    uint64_t* ticket);

int gp_server_submit_ir(gp_server* s, const gp_circuit_ir* ir, const double* rates, size_t n_rates,
                        uint64_t* ticket) {
  return gp::guarded([&] { return gp_server_submit_ir_impl(s, ir, rates, n_rates, ticket); });
}

int gp_server_create(const gp_bounds* bounds, int device, gp_server** out) {
  return gp::guarded([&] { return gp_server_create_impl(bounds, device, out); });
}

int gp_server_submit(gp_server* s, const char* text, size_t len, const double* rates, size_t n_rates,
                     uint64_t* ticket) {
  return gp::guarded([&] { return gp_server_submit_impl(s, text, len, rates, n_rates, ticket); });
}

static int gp_server_create_impl(const gp_bounds* bounds, int device, gp_server** out) {
  if (!bounds || !out) return gp::set_last_error(GP_E_ARG, "null argument");
  *out = nullptr;
  gp_server* s = new gp_server();
  s->bounds = *bounds;
  for (int k = 0; k < 2; k++) {
    int rc = gp_driver_create(bounds, device, &s->drv[k]);
    if (rc) {
      const std::string msg = gp_last_error();
      if (s->drv[0]) gp_driver_destroy(s->drv[0]);
      delete s;
      return gp::set_last_error(rc, msg);
    }
  }
  const uint32_t level = gp::driver_level(s->drv[0]);
  const size_t n_lower = std::min<size_t>(8, std::max<size_t>(1, std::thread::hardware_concurrency()));
  try {
    for (size_t k = 0; k < n_lower; k++) s->lowerers.emplace_back(lower_loop, s, level);
    s->worker = std::thread(worker_loop, s);
  } catch (...) {
    gp_server_destroy(s);  // stops and joins the threads that did start, frees the drivers
    return gp::set_last_error(GP_E_OOM, "could not start the server's threads");
  }
  *out = s;
  return GP_OK;
}

// Admit a request (or refuse it past the limits) and queue it for lowering.
static int enqueue(gp_server* s, const ReqPtr& r, uint64_t* ticket) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return gp::set_last_error(GP_E_STATE, "the server is shutting down");
    if (!s->live.empty() && (s->live.size() >= s->max_live || s->live_bytes + r->held > s->max_bytes))
      return gp::set_last_error(GP_E_BUSY, "admission refused: the server holds its limit of live requests or "
                                           "bytes (collect results with gp_server_wait, then retry)");
    s->live_bytes += r->held;
    r->ticket = s->next_ticket++;
    r->t_submit = now_ns();
    s->to_lower.push_back(r);
    s->live[r->ticket] = r;
  }
  s->cv_lower.notify_one();
  *ticket = r->ticket;
  return GP_OK;
}

static int gp_server_submit_impl(gp_server* s, const char* text, size_t len, const double* rates, size_t n_rates,
                                 uint64_t* ticket) {
  if (!s || !text || !ticket || (!rates && n_rates)) return gp::set_last_error(GP_E_ARG, "null argument");
  ReqPtr r = std::make_shared<Request>();
  r->text.assign(text, len);
  if (rates) {
    r->rates.assign(rates, rates + n_rates);
    r->has_rates = true;
  }
  r->held = len + uint64_t(n_rates) * sizeof(double);
  return enqueue(s, r, ticket);
}

static int gp_server_submit_ir_impl(gp_server* s, const gp_circuit_ir* ir, const double* rates, size_t n_rates,
                                    uint64_t* ticket) {
  if (!s || !ir || !ticket || (!rates && n_rates)) return gp::set_last_error(GP_E_ARG, "null argument");
  if ((ir->n_ops && !ir->code) || (ir->n_rec && !ir->rec))
    return gp::set_last_error(GP_E_ARG, "binary circuit without its operation codes or records");
  ReqPtr r = std::make_shared<Request>();
  r->is_ir = true;
  const size_t n = size_t(ir->n_ops);
  r->ir_n_ops = ir->n_ops;
  if (n) {
    r->ir_code.assign(ir->code, ir->code + n);
    if (ir->q0) r->ir_q0.assign(ir->q0, ir->q0 + n);
    if (ir->q1) r->ir_q1.assign(ir->q1, ir->q1 + n);
    if (ir->rate) r->ir_rate.assign(ir->rate, ir->rate + n);
  }
  if (ir->n_rec) r->ir_rec.assign(ir->rec, ir->rec + ir->n_rec);
  if (rates) {
    r->rates.assign(rates, rates + n_rates);
    r->has_rates = true;
  }
  r->held = n * (1 + 4 + 4 + 8) + ir->n_rec * 4 + uint64_t(n_rates) * sizeof(double);
  return enqueue(s, r, ticket);
}

int gp_server_set_admission(gp_server* s, uint64_t max_requests, uint64_t max_bytes) {
  if (!s) return gp::set_last_error(GP_E_ARG, "null server");
  if (!max_requests || !max_bytes) return gp::set_last_error(GP_E_ARG, "admission limits must be positive");
  std::lock_guard<std::mutex> lk(s->mu);
  s->max_live = max_requests;
  s->max_bytes = max_bytes;
  return GP_OK;
}

int gp_server_wait(gp_server* s, uint64_t ticket, int64_t timeout_us, gp_edges** out, uint64_t* latency_ns) {
  if (!s || !out) return gp::set_last_error(GP_E_ARG, "null argument");
  *out = nullptr;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->live.find(ticket);
  if (it == s->live.end()) return gp::set_last_error(GP_E_ARG, "unknown ticket (never issued or already collected)");
  ReqPtr r = it->second;
  if (timeout_us < 0) {
    s->cv_done.wait(lk, [&] { return r->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->done; })) {
    return gp::set_last_error(GP_E_STATE, "the request has not finished yet");
  }
  s->live.erase(ticket);
  s->live_bytes -= r->held;
  if (latency_ns) *latency_ns = r->t_done - r->t_submit;
  if (r->rc) return gp::set_last_error(r->rc, r->msg);
  *out = r->edges;
  r->edges = nullptr;
  return GP_OK;
}

int gp_server_stats(const gp_server* s, uint64_t* batches, uint64_t* requests, uint64_t* max_batch) {
  if (!s) return gp::set_last_error(GP_E_ARG, "null server");
  gp_server* m = const_cast<gp_server*>(s);
  std::lock_guard<std::mutex> lk(m->mu);
  if (batches) *batches = s->n_batches;
  if (requests) *requests = s->n_requests;
  if (max_batch) *max_batch = s->max_batch;
  return GP_OK;
}

int gp_server_timing(const gp_server* s, double* lower_ms, double* upload_ms, double* fetch_ms, double* wait_ms,
                     double* download_ms) {
  if (!s) return gp::set_last_error(GP_E_ARG, "null server");
  gp_server* m = const_cast<gp_server*>(s);
  std::lock_guard<std::mutex> lk(m->mu);
  if (lower_ms) *lower_ms = s->ns_lower * 1e-6;
  if (upload_ms) *upload_ms = s->ns_upload * 1e-6;
  if (fetch_ms) *fetch_ms = s->ns_fetch * 1e-6;
  if (wait_ms) *wait_ms = s->ns_wait * 1e-6;
  if (download_ms) *download_ms = s->ns_download * 1e-6;
  return GP_OK;
}

void gp_server_destroy(gp_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_lower.notify_all();
  for (std::thread& th : s->lowerers) th.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->lowerers_done = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->live)
    if (kv.second->edges) gp_edges_free(kv.second->edges);
  for (gp_driver* d : s->drv)
    if (d) gp_driver_destroy(d);
  delete s;
}

}  // extern "C"
