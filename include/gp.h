/*
 * gp.h -- C ABI of the MI355X just-in-time compiler for decoding hypergraphs.
 *
 * The library compiles one realised, fully unrolled Clifford circuit with
 * Pauli noise channels into its decoding hypergraph (the detector error model
 * of paper Sec. 2.1.4): one hyperedge per equivalence class of faults, carrying
 * the exact set of detectors and logical observables the class flips and the
 * merged probability of its faults (Eq. 3). The pipeline is the paper's
 * two-stage method (Sec. 3): lowering to the space-time error propagation graph
 * (Sec. 2.3.1), stage 1 error-equivalence-class generation by a backward XOR
 * sweep (Alg. 1, Eq. 1, Eq. 2), stage 2 probability aggregation by hash, sort
 * and segmented reduction (Sec. 3.2, Eq. 3). Lowering runs on the host; both
 * stages run in HIP kernels on one gfx950 device.
 *
 * Conventions for every function:
 *   - the return value is a status: GP_OK (0) or a negative GP_E_* code; on a
 *     non-zero status gp_last_error() returns a thread-local message and no
 *     output argument is written;
 *   - pointers named text/rates are host pointers owned by the caller and only
 *     read during the call;
 *   - objects returned through an out-pointer are owned by the caller and are
 *     released with the matching *_destroy / *_free function;
 *   - a driver is not thread-safe: use one driver per host thread.
 *
 * Circuit language: a subset of the Stim text format. Gates R RZ RX M MZ MX MR
 * MRZ MRX H H_XZ S S_DAG SQRT_Z SQRT_Z_DAG SQRT_X SQRT_X_DAG I X Y Z CX CNOT
 * ZCX CZ ZCZ SWAP; noise X_ERROR Y_ERROR Z_ERROR DEPOLARIZE1 DEPOLARIZE2 (one
 * probability argument); annotations DETECTOR OBSERVABLE_INCLUDE(k) with
 * rec[-k] targets; TICK QUBIT_COORDS SHIFT_COORDS are accepted and ignored.
 * REPEAT blocks, measurement-flip arguments and inverted targets are rejected
 * with GP_E_UNSUPPORTED. Every qubit starts in |0>.
 *
 * Channels are numbered in program order and, inside one noise instruction,
 * in target-group order (one qubit; one pair for DEPOLARIZE2). A rate array
 * passed to the compile functions is indexed by that channel number.
 *
 * Per-fault probabilities (the paper does not state them): X/Y/Z_ERROR(r)
 * give one fault with p = r; DEPOLARIZE1(r) gives X, Y and Z each with the p
 * for which (1-2p)^2 = 1 - 4r/3, DEPOLARIZE2(r) the fifteen non-identity
 * two-qubit Paulis each with (1-2p)^8 = 1 - 16r/15 (independent channels with
 * the same Pauli transfer eigenvalues as the depolarising channel).
 */
#ifndef GP_H
#define GP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  GP_OK = 0,
  GP_E_ARG = -1,              /* null pointer, bad size, bad handle */
  GP_E_PARSE = -2,            /* malformed circuit text */
  GP_E_UNSUPPORTED = -3,      /* instruction or target outside the subset, REPEAT */
  GP_E_BOUNDS = -4,           /* circuit exceeds the driver's bounds (no silent re-allocation) */
  GP_E_NONDETERMINISTIC = -5, /* a detector or observable is not deterministic */
  GP_E_NOISE = -6,            /* rate outside its domain, or wrong rate-array length */
  GP_E_HIP = -7,              /* HIP runtime error, or no usable gfx950 device */
  GP_E_OOM = -8,              /* host or device allocation failed */
  GP_E_COLLISION = -9,        /* two different signatures share both 64-bit hashes */
  GP_E_STATE = -10,           /* call out of order (e.g. gp_run before gp_lower) */
  GP_E_BUSY = -11,            /* the server holds its limit of requests or bytes: collect results, retry */
  GP_E_INTERNAL = -12         /* an unexpected internal failure (no result; the driver stays usable) */
};

typedef struct gp_driver gp_driver;
typedef struct gp_edges gp_edges;
typedef struct gp_server gp_server;

/* Size bounds of a driver; every device buffer is allocated once from these
 * (paper Sec. 3.4, buffer reuse). Circuits within the bounds reuse the buffers.
 * For a batch (gp_lower_batch), qubits, layers, detectors and observables
 * bound each circuit; every other field bounds the sum over the batch. */
typedef struct gp_bounds {
  uint32_t max_qubits;
  uint32_t max_layers;        /* gate layers after as-soon-as-possible scheduling */
  uint32_t max_measurements;
  uint32_t max_detectors;
  uint32_t max_observables;
  uint32_t max_channels;
  uint64_t max_faults;        /* at most 2^30 - 1 */
  uint64_t max_ops;           /* elementary gate/measurement/reset operations */
  uint64_t max_leaf_bits;     /* total (measurement, detector-or-observable) memberships */
  uint64_t max_slab_words;    /* 64-bit words of stage-1 signature storage (0: max_faults words per column) */
  uint64_t max_items;         /* stage-1 sweep work items (0: enough for any circuit within the bounds) */
  uint32_t max_branches;      /* circuits one batch may hold (0 means 1) */
} gp_bounds;

/* Sizes of the most recently lowered circuit (and, after a fetch, its result). */
typedef struct gp_circuit_info {
  uint32_t n_qubits, n_layers, n_measurements, n_detectors, n_observables;
  uint32_t n_words;           /* 64-bit signature words: ceil(D/64) + ceil(O/64) */
  uint64_t n_channels, n_faults, n_ops, n_items, slab_words;
  uint64_t n_classes;         /* equivalence classes incl. the empty one (valid after fetch) */
  uint64_t n_edges;           /* hyperedges = non-empty classes (valid after fetch) */
  uint64_t n_edge_bits;       /* total signature bits over all hyperedges (valid after fetch) */
  uint64_t n_live_words;      /* stage-1 signature words in the swept windows (valid after fetch) */
  uint64_t n_live_faults;     /* faults with a non-empty signature (valid after fetch) */
  uint64_t n_nonzero_words;   /* non-zero stage-1 signature words stored (valid after fetch) */
  uint32_t n_circuits;        /* circuits lowered together (1 after gp_lower) */
} gp_circuit_info;

/* Binary form of a realised circuit (the input a simulator that realises
 * adaptive branches produces, Sec. 3.4 and Sec. 5.2.1: no text to print or
 * parse). One entry per elementary operation, in program order, as parallel
 * arrays of n_ops entries:
 *   code[k]  GP_IR_* below;
 *   q0[k]    the qubit (the control of CX); for GP_IR_OBSERVABLE the
 *            observable index (at most 65535); unused for GP_IR_DETECTOR;
 *   q1[k]    the second qubit of CX / CZ / SWAP / DEPOLARIZE2 (different from
 *            q0); for GP_IR_DETECTOR and GP_IR_OBSERVABLE the number of
 *            records the operation takes from `rec`; unused otherwise;
 *   rate[k]  the rate of a noise operation (X/Y/Z_ERROR at most 1/2,
 *            DEPOLARIZE1 at most 3/4, DEPOLARIZE2 at most 15/16); unused
 *            otherwise.
 * rec holds the records of the annotations, concatenated in program order
 * (n_rec entries, all used): absolute measurement indices, the first
 * measurement of the circuit being 0, each naming a measurement made before
 * the annotation. A measurement listed twice by one detector or observable
 * cancels (XOR), and GP_IR_OBSERVABLE accumulates over operations, as in the
 * text form. Each noise operation is one channel (a DEPOLARIZE2 one pair), so
 * channels are numbered by their position among the noise operations. An
 * array no operation reads may be NULL. The arrays are host memory owned by
 * the caller and only read during the call. Qubit indices are below 2^28.
 * The semantics are those of the same operations in the text form; GP_IR_PAULI
 * (I, X, Y or Z) only makes its qubit part of the circuit. */
enum {
  GP_IR_PAULI = 0, GP_IR_H = 1, GP_IR_S = 2, GP_IR_SQRT_X = 3, GP_IR_CX = 4, GP_IR_CZ = 5, GP_IR_SWAP = 6,
  GP_IR_R = 7, GP_IR_RX = 8, GP_IR_M = 9, GP_IR_MX = 10, GP_IR_MR = 11, GP_IR_MRX = 12,
  GP_IR_X_ERROR = 16, GP_IR_Y_ERROR = 17, GP_IR_Z_ERROR = 18, GP_IR_DEPOLARIZE1 = 19, GP_IR_DEPOLARIZE2 = 20,
  GP_IR_DETECTOR = 32, GP_IR_OBSERVABLE = 33
};
typedef struct gp_circuit_ir {
  uint64_t n_ops;
  const uint8_t* code;
  const uint32_t* q0;
  const uint32_t* q1;
  const double* rate;
  uint64_t n_rec;
  const uint32_t* rec;
} gp_circuit_ir;

/* Thread-local description of the last non-zero status. Never NULL. */
const char* gp_last_error(void);

/* Lower `text` on the host only and report the bounds it needs. No GPU use. */
int gp_bounds_from_circuit(const char* text, size_t len, gp_bounds* out);

/* Create a driver on HIP device `device`: allocates every device buffer from
 * `bounds` and a HIP stream of default priority. Fails with GP_E_HIP when the
 * device is missing or is not gfx950. */
int gp_driver_create(const gp_bounds* bounds, int device, gp_driver** out);

/* Listing 1 of the paper: a driver whose bounds are those of a maximum circuit. */
int gp_driver_create_from_circuit(const char* text, size_t len, int device, gp_driver** out);

/* Batch forms (Sec. 3.4 compiles many circuit instances; here several are
 * compiled by one launch of each stage). `texts[k]`, `lens[k]`: host circuit
 * texts, k < n. gp_bounds_from_batch reports the bounds the batch needs (no
 * GPU use); gp_driver_create_from_batch creates a driver from them. */
int gp_bounds_from_batch(const char* const* texts, const size_t* lens, size_t n, gp_bounds* out);
int gp_driver_create_from_batch(const char* const* texts, const size_t* lens, size_t n, int device,
                                gp_driver** out);

/* Waits for outstanding work, frees device and host buffers. NULL is ignored. */
void gp_driver_destroy(gp_driver* drv);

/* Whole path, blocking: lower, run both stages, copy the hypergraph to the
 * host (paper Listing 1, compile_detector_error_model). `rates` (NULL = rates
 * written in the text) must hold exactly one rate per channel. `level` is the
 * correlation level of Table 1 for this compile (0, 1, 2 = every Pauli; -1 =
 * the driver's, see gp_set_correlation_level). On success *out owns the
 * result. */
int gp_compile_hypergraph(gp_driver* drv, const char* text, size_t len,
                          const double* rates, size_t n_rates, int level, gp_edges** out);

/* The same for a circuit in binary form (gp_circuit_ir above): lowering it
 * gives the same tables as lowering the equivalent text, with no parsing. Its
 * split forms, batch form and bounds (same status codes as the text forms,
 * errors naming the operation index instead of a line): */
int gp_compile_ir(gp_driver* drv, const gp_circuit_ir* ir, const double* rates, size_t n_rates, int level,
                  gp_edges** out);
int gp_lower_ir(gp_driver* drv, const gp_circuit_ir* ir, const double* rates, size_t n_rates);
int gp_lower_batch_ir(gp_driver* drv, const gp_circuit_ir* irs, size_t n, const double* const* rates,
                      const size_t* n_rates);
int gp_bounds_from_ir(const gp_circuit_ir* ir, gp_bounds* out);
int gp_bounds_from_batch_ir(const gp_circuit_ir* irs, size_t n, gp_bounds* out);

/* Split form of gp_compile_hypergraph, for callers that keep state on the
 * device and time the device stages alone:
 *   gp_lower  -- host lowering + asynchronous upload of the tables to the
 *                driver's buffers (the upload is ordered on the driver's stream);
 *   gp_run    -- enqueue stage 1 and stage 2 on the driver's stream; returns
 *                without waiting; may be called repeatedly on one lowering;
 *   gp_fetch  -- wait for the stream, check device-side error flags
 *                (GP_E_NONDETERMINISTIC, GP_E_COLLISION, GP_E_BOUNDS; GP_E_HIP
 *                when a radix-sort tile gave up waiting for its predecessor
 *                twice), redoing the compile where a flag calls for it, and
 *                copy the hypergraph to a new host gp_edges. */
int gp_lower(gp_driver* drv, const char* text, size_t len, const double* rates, size_t n_rates);
int gp_run(gp_driver* drv);
int gp_fetch(gp_driver* drv, gp_edges** out);

/* Fetch of a result into caller-owned host arrays, with one host copy.
 * gp_fetch_sizes does what gp_fetch does up to the download (wait, error
 * flags, retries; the same status codes) and returns the hyperedge and
 * signature-bit counts (n_det, n_obs: the detector and observable counts, of
 * a batch the largest of any circuit; may be NULL). gp_fetch_copy then fills
 * offsets (n_edges + 1 entries, edge e's bits are bits[offsets[e] ..
 * offsets[e+1])), bits (n_bits) and q (n_edges), laid out as
 * gp_edges_offsets/bits/probabilities; a batch's hyperedges are listed circuit
 * by circuit, and gp_fetch_circuit_offsets fills the circuits + 1 offsets
 * (circuit k owns hyperedges circuit_offsets[k] .. circuit_offsets[k+1]-1, its
 * bits numbered as in gp_edges_circuit_shape). Both may be called again until
 * the next gp_lower, gp_run or fetch; GP_E_STATE without a current
 * gp_fetch_sizes. Rate refreshes and the adjoint work after it as after
 * gp_fetch. */
int gp_fetch_sizes(gp_driver* drv, uint64_t* n_edges, uint64_t* n_bits, uint32_t* n_det, uint32_t* n_obs);
int gp_fetch_copy(gp_driver* drv, uint64_t* offsets, uint32_t* bits, double* q);
int gp_fetch_circuit_offsets(gp_driver* drv, uint64_t* circuit_offsets);

/* Lower n independent circuits as one batch; gp_run then compiles them all in
 * one pass of each stage and gp_fetch returns every circuit's hyperedges in
 * one gp_edges, tagged by circuit (gp_edges_circuit_ids). Each circuit is
 * grouped on its own: a hyperedge never merges faults of two circuits, and
 * circuit k's hyperedges are those a compile of circuit k alone gives, in the
 * same order (same bits; the same probabilities, bitwise when both compiles
 * take the same stage-2 grouping). `rates` (host,
 * may be NULL) holds one rate array per circuit (rates[k] NULL = the rates in
 * texts[k]) of n_rates[k] entries. For gp_refresh_rates and gp_rates_gradient
 * the channels of a batch are numbered circuit by circuit: circuit 0's in
 * program order, then circuit 1's, and so on. A failing circuit reports its
 * index in gp_last_error. */
int gp_lower_batch(gp_driver* drv, const char* const* texts, const size_t* lens, const double* const* rates,
                   const size_t* n_rates, size_t n);

/* Autotuner for stage 1 and the stage-2 grouping. An observable column stays live over the whole
 * circuit, so it is cut into boundary ranges swept by separate work items;
 * the cut balances estimated item times in which a layer costs 1 and emitting
 * a boundary 1 + fault_cost per fault there. The sweep runs one work-group of
 * 1024 threads per item, or of 256 threads with smaller LDS tables (two per
 * CU) when the circuit fits them. gp_autotune compiles `text` (gp_autotune_batch:
 * the batch, as gp_lower_batch with the rates in the texts) with each of a few
 * fault costs and each work-group size that fits, times `iters` device runs
 * of each (HIP events on the driver's stream) and keeps the fastest pair for
 * the following lowerings of this driver. For that pair it then times the
 * stage-2 groupings (the size's default, the full radix sort, the 65,536
 * buckets; one whose runs raise a device flag is not a candidate) and keeps
 * the fastest for the following runs. Results are cached per process by
 * the lowered shape (the key fields below): a shape already tuned is lowered
 * once to read its key and not timed again (cached = 1). *out (may be NULL)
 * receives the choice. The driver must be sized for the input. Afterwards no
 * lowering is current (gp_lower again). gp_set_fault_cost sets the cut
 * directly (0 < c < 1). Neither changes any signature or probability. */
typedef struct gp_tuning {
  double fault_cost; /* cost per fault of an observable range, relative to a layer */
  int32_t sweep_block; /* stage-1 work-group size: 1024 or 256 */
  int32_t cached;    /* 1: taken from the cache */
  double ms;         /* mean device time per run when it was tuned */
  /* the shape key: circuits, most qubits and layers of one circuit, faults,
   * most detectors and observables of one circuit, correlation level */
  uint32_t n_circuits, n_qubits, n_layers, n_det;
  uint64_t n_faults;
  uint32_t n_obs, level;
  int32_t grouping;  /* stage-2 grouping (as gp_debug_set_sort_mode): 0 the size's default, 1 the full
                      * radix sort, 2 the 65,536 buckets */
  int32_t reserved;  /* 0 */
} gp_tuning;
int gp_autotune(gp_driver* drv, const char* text, size_t len, int iters, gp_tuning* out);
int gp_autotune_batch(gp_driver* drv, const char* const* texts, const size_t* lens, size_t n, int iters,
                      gp_tuning* out);
/* The process-wide tuning cache, for saving and restoring it: the number of
 * entries, entry i (in key order; GP_E_ARG past the end), and inserting or
 * replacing an entry by its key (GP_E_ARG for a fault cost outside (0, 1), a
 * work-group size other than 256 or 1024, or a level above 2). */
size_t gp_tuning_cache_size(void);
int gp_tuning_cache_get(size_t i, gp_tuning* out);
int gp_tuning_cache_put(const gp_tuning* t);
int gp_set_fault_cost(gp_driver* drv, double fault_cost);

/* Correlation level (Table 1) for the following lowerings: which Paulis of
 * each noise channel become faults. 0: products of X's or of Z's (IX, IZ, XI,
 * XX, ZI, ZZ; one-qubit X, Z); 1 adds a Y next to the identity and mixed X/Z
 * pairs (IY, YI, XZ, ZX; one-qubit Y); 2 (default): every Pauli. A kept fault
 * keeps the probability it has at level 2. GP_E_ARG for other values. */
int gp_set_correlation_level(gp_driver* drv, int level);

/* Fixed structure, new rates (Eq. 3 over cached classes). After a gp_fetch,
 * the driver keeps each hyperedge's member faults (in fault order) on the
 * device. gp_refresh_rates replaces the channel rates (`rates`: host,
 * n_rates = channel count, program order, each within its channel's range)
 * and enqueues the per-fault probabilities and the merge of every hyperedge
 * again -- no stage-1 sweep, no grouping; the next gp_fetch returns the same
 * hyperedges in the same order with the new probabilities (bitwise what a full
 * compile gives, except classes of more than 65 faults compiled by the full
 * radix sort, which agree to rounding). GP_E_STATE if no fetched compile of
 * the lowered circuit exists; GP_E_NOISE for a bad rate array (the previous
 * rates stay). */
int gp_refresh_rates(gp_driver* drv, const double* rates, size_t n_rates);

/* Adjoint of stage 2 for the current rates (those of the last compile or
 * refresh). Input dl_dq: host, one dL/dq per hyperedge in the order of the
 * last gp_fetch. Output dl_dr: host, one dL/d(rate) per channel in program
 * order. With q_k = 1/2 (1 - prod_{i in k} (1 - 2 p_i)) (Eq. 3 unrolled),
 * dq_k/dp_i = prod_{j in k, j != i} (1 - 2 p_j); dp_i/dr is the derivative of
 * the per-fault split of the fault's channel; faults with an empty signature
 * contribute nothing. Synchronous. GP_E_STATE without a fetched compile,
 * GP_E_ARG for wrong lengths. */
int gp_rates_gradient(gp_driver* drv, const double* dl_dq, size_t n_edges, double* dl_dr, size_t n_rates);

/* Stage 2 over the cached structure with every operand in device memory, on
 * the caller's stream: the drift-recalibration refresh (Sec. 2.2) and its
 * adjoint, for callers (such as an autograd function) whose rates, q and
 * gradients already live on the GPU. After a fetched compile:
 *   gp_aggregate          d_rates -> d_q: the per-fault probabilities at the
 *                         rates and the Eq. 3 merge of every hyperedge, as
 *                         gp_refresh_rates computes them (bitwise the same);
 *   gp_aggregate_backward d_rates, d_gq -> d_grates: dL/d(rate) for dL/dq,
 *                         as gp_rates_gradient computes it, at d_rates (so it
 *                         does not depend on which rates were applied last).
 * d_rates: n_rates = channel count doubles, program order (a batch: circuit
 * by circuit), each within its channel's range (not checked on the device; an
 * out-of-range rate gives NaN); d_q, d_gq: n_edges = the fetched compile's
 * hyperedge count doubles, in the order of the last fetch; d_grates: n_rates
 * doubles. All device pointers on the driver's device, owned by the caller.
 * `stream` is a hipStream_t (NULL: the driver's stream); the work is enqueued
 * there without waiting, after everything already enqueued on the driver and
 * before anything enqueued on it later (the driver's per-fault buffers are
 * shared: do not overlap two of these calls on different streams). The first
 * call after a batch fetch uploads that fetch's hyperedge order once
 * (synchronously). GP_E_STATE without a fetched compile, GP_E_ARG for wrong
 * lengths. gp_structure_id returns an id that changes whenever a fetch
 * replaces the cached structure (0: none), so that a caller holding results
 * of an earlier structure can tell. */
int gp_aggregate(gp_driver* drv, const double* d_rates, size_t n_rates, double* d_q, size_t n_edges, void* stream);
int gp_aggregate_backward(gp_driver* drv, const double* d_rates, size_t n_rates, const double* d_gq, size_t n_edges,
                          double* d_grates, void* stream);
uint64_t gp_structure_id(const gp_driver* drv);

/* gp_aggregate_backward for callers that cannot allocate device memory in the
 * call: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation. Same arguments, checks, stream ordering and result
 * (bitwise) as gp_aggregate_backward, but the per-fault dL/dp it accumulates
 * lives in a static device array of the library (16 MiB: at most 2^21 =
 * 2,097,152 faults per compile) instead of the driver's buffer, and the call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * Each GPU the library runs on holds its own copy of that array from the first
 * driver created on it until the process ends. The array is cleared by a fill
 * kernel at the start of every call (it keeps the last call's contents
 * otherwise). Calls that overlap on one GPU (two drivers or two streams of
 * that device at once) share the array and race: serialise them.
 * GP_E_BOUNDS when the fetched compile has more faults than the array holds;
 * otherwise the errors of gp_aggregate_backward. */
int gp_aggregate_backward_noalloc(gp_driver* drv, const double* d_rates, size_t n_rates, const double* d_gq,
                                  size_t n_edges, double* d_grates, void* stream);

/* Request server (continuous batching). A worker thread owns two drivers
 * created with `batch_bounds` (the bounds of one batch: max_branches circuits
 * at most, totals summed over them), each on its own HIP stream of default
 * priority on `device`; a pool of host threads lowers every submitted circuit
 * as soon as it arrives. Every pass the worker takes the lowered requests,
 * uploads them as one batch to the free driver and launches both stages;
 * while that batch runs, it downloads the other driver's batch and completes
 * those requests. A batch that exceeds the
 * bounds is split; a request that exceeds them alone fails with GP_E_BOUNDS.
 * Each request gets exactly the hyperedges of its own circuit (a batch never
 * merges faults of two circuits), whatever it was batched with.
 *
 * gp_server_submit copies `text` and `rates` (host; rates NULL = the rates in
 * the text) and returns a ticket at once. gp_server_wait blocks until that
 * request is done (timeout_us < 0: no limit; otherwise GP_E_STATE when the
 * time runs out, and the ticket stays valid), then hands over its result
 * (*out, released with gp_edges_free) or returns the request's own error
 * status and message; latency_ns (may be NULL) receives the time from submit
 * to completion. A ticket is collected once; GP_E_ARG for unknown tickets.
 * gp_server_stats reports batches launched, requests batched and the largest
 * batch. gp_server_destroy finishes every submitted request, frees the
 * results nobody collected and the drivers. The functions may be called from
 * several host threads. */
int gp_server_create(const gp_bounds* batch_bounds, int device, gp_server** out);
int gp_server_submit(gp_server* srv, const char* text, size_t len, const double* rates, size_t n_rates,
                     uint64_t* ticket);
/* gp_server_submit for a circuit in binary form: its arrays are copied, so
 * the caller may reuse them as soon as the call returns. */
int gp_server_submit_ir(gp_server* srv, const gp_circuit_ir* ir, const double* rates, size_t n_rates,
                        uint64_t* ticket);
int gp_server_wait(gp_server* srv, uint64_t ticket, int64_t timeout_us, gp_edges** out, uint64_t* latency_ns);
int gp_server_stats(const gp_server* srv, uint64_t* batches, uint64_t* requests, uint64_t* max_batch);
/* Admission (backpressure): a server holds at most `max_requests` live
 * requests (submitted and not yet collected by gp_server_wait) and at most
 * `max_bytes` of host memory for them (circuit text and rates, then the
 * result until it is collected). gp_server_submit returns GP_E_BUSY at once,
 * without queueing, when admitting the request would pass either limit;
 * a request is always admitted when nothing is live. Defaults: 4096 requests,
 * 4 GiB. GP_E_ARG for a zero limit. Device memory needs no admission: each
 * driver is allocated once for the batch bounds. */
int gp_server_set_admission(gp_server* srv, uint64_t max_requests, uint64_t max_bytes);
/* Worker time so far (milliseconds) in host lowering, in merging +
 * uploading + launching, and in fetching results (waiting for the device,
 * downloading, splitting per request), with the waiting and the downloading
 * parts of the latter. Any output may be NULL. */
int gp_server_timing(const gp_server* srv, double* lower_ms, double* upload_ms, double* fetch_ms, double* wait_ms,
                     double* download_ms);
void gp_server_destroy(gp_server* srv);

/* Wait for every operation enqueued on the driver's stream. */
int gp_sync(gp_driver* drv);

/* The driver's hipStream_t, as an opaque pointer. */
void* gp_driver_stream(gp_driver* drv);

int gp_circuit_info_get(const gp_driver* drv, gp_circuit_info* out);
/* Detector and observable counts of circuit `circuit` of the current
 * lowering (0 after gp_lower); GP_E_ARG past the last circuit. */
int gp_circuit_shape(const gp_driver* drv, uint32_t circuit, uint32_t* n_det, uint32_t* n_obs);

/* Per-kernel timing with HIP events recorded on the driver's stream around
 * every launch while enabled. Totals accumulate over gp_run calls until reset;
 * they are read after gp_sync / gp_fetch. */
int gp_set_timing(gp_driver* drv, int enable);
int gp_reset_timing(gp_driver* drv);
int gp_timing_count(const gp_driver* drv);
int gp_timing_entry(const gp_driver* drv, int index, const char** name,
                    double* total_ms, uint64_t* launches);

/* Test hooks. gp_debug_set_key_bits keeps only the low `bits` bits of the
 * stage-2 class key (default 64), which forces key collisions; the result must
 * not change, because a collision found on the device makes gp_fetch compile
 * again keyed on both hashes. gp_debug_collision_retries counts such re-runs. */
int gp_debug_set_key_bits(gp_driver* drv, int bits);
uint64_t gp_debug_collision_retries(const gp_driver* drv);

/* Re-runs made by fetches so far, by cause: a radix-sort tile that gave up
 * waiting for the tile before it (the same compile runs once more; a second
 * give-up fails the fetch with GP_E_HIP and no result), a 256-bucket group too
 * large for LDS (redone with the full sort), a key collision (redone keyed on
 * both hashes). Any output may be NULL. */
int gp_debug_retry_counts(const gp_driver* drv, uint64_t* lookback, uint64_t* bucket, uint64_t* collision);

/* Test hook: look-back rounds a radix-sort tile waits for the tiles before it
 * (each round reads up to 16 of them, then sleeps briefly) before giving up;
 * default 2^22. With 0 every tile after the first gives up at once, so the
 * fetch after a gp_run fails with GP_E_HIP; every kernel still ends normally
 * (a give-up stops the grouping kernels that follow it). */
int gp_debug_set_spin_limit(gp_driver* drv, uint32_t limit);

/* Waits for the driver's stream and reads the device status flags: those of
 * the last compile (*flags), and the union of those raised by every compile
 * since the last clear (*flags_seen, which catches a flag raised by a compile
 * whose result was never fetched, such as a timing loop of gp_run calls).
 * Bits: 1 non-deterministic detector, 2 key collision, 4 output capacity,
 * 8 sort look-back give-up, 16 bucket overflow. clear_seen != 0 clears the
 * union afterwards. */
int gp_debug_device_flags(gp_driver* drv, uint32_t* flags, uint32_t* flags_seen, int clear_seen);

/* Test hook: stage-2 grouping method for later gp_run calls. 0 (default):
 * up to 1,572,864 faults one stable radix pass on the top 8-bit key digit
 * splits the faults into 256 buckets, and from 12,000,000 to 67,108,864 faults
 * two passes on the top two digits split them into 65,536 buckets; each bucket
 * is sorted and merged in LDS (a bucket over its LDS capacity makes gp_fetch
 * redo the grouping with the full sort); otherwise the full LSD radix sort
 * over every key digit. 1: always the full sort. 2: the 65,536 buckets whenever
 * the key has at least three digits. All give the same hyperedges (same
 * classes, same merge order within a class; the edge order may differ).
 * GP_E_ARG for other values. */
int gp_debug_set_sort_mode(gp_driver* drv, int mode);

/* Test hook: stage-1 work-group shape for later gp_run calls. 0 (default):
 * automatic (work-groups of 256 threads with smaller LDS tables, several per
 * CU, when a compile has at least 512 sweep items of a circuit small enough;
 * otherwise one work-group of 1024 threads per item); 1: always 1024 threads;
 * 2: 256 threads wherever the circuit fits them. Same signatures either way.
 * GP_E_ARG for other values. */
int gp_debug_set_sweep_shape(gp_driver* drv, int shape);

/* Launch mode: with enable = 1, gp_run replays the compile's kernel launches as
 * one HIP graph, captured at the first gp_run after each lowering (and after a
 * change of the test modes above); 0 (default) launches every kernel on its
 * own. Worth it only when one lowering is run many times; runs with timing
 * enabled (gp_set_timing) are never captured. */
int gp_debug_set_graph(gp_driver* drv, int enable);

/* Test hook for the class key of Sec. 3.2. With enable = 1, every later gp_run
 * copies the per-position class keys (written by the hash kernel, before the
 * grouping passes reuse that buffer) into a buffer this call allocates once
 * (8 B per fault of the driver's bounds); runs with the hook on are never
 * replayed as a graph. gp_debug_class_keys synchronises the driver's stream
 * and copies min(cap, n) keys of the last gp_run to out (host memory, may be
 * NULL when cap is 0): position order (the lowered fault order), each key the
 * 64-bit FNV-1a of the fault's signature (the 8W little-endian octets of its W
 * signature words: detector words, then observable words) cut to its low
 * *key_bits bits; a circuit of a batch other than the first also has a
 * per-circuit salt in it. *n_faults gets n; key_bits may be NULL.
 * GP_E_STATE when no gp_run has run with the hook on. */
int gp_debug_capture_keys(gp_driver* drv, int enable);
int gp_debug_class_keys(gp_driver* drv, uint64_t* out, uint64_t cap, uint64_t* n_faults, uint32_t* key_bits);

/* Profiling hook: device wall-clock stamps of every stage-1 sweep item of the
 * last gp_run (start, end pairs; `cap` entries at most), the item count, and
 * the clock rate in Hz. Synchronises the driver's stream. */
int gp_debug_sweep_times(gp_driver* drv, uint64_t* out, uint64_t cap, uint64_t* n_items, double* clock_hz);

/* Result accessors. Hyperedge e has signature bits
 *   bits[offsets[e]] ... bits[offsets[e+1]-1]   (strictly increasing),
 * where bit b < n_detectors is detector b and bit n_detectors + k is
 * observable k, and probability probabilities[e]. Hyperedges are ordered by
 * their lowest fault (the class member with the lowest position in the
 * lowered fault order: channels by boundary, then program order), so the
 * order is deterministic for a given circuit and a batch is listed circuit by
 * circuit. Pointers stay valid until gp_edges_free.
 * A batch result lists the hyperedges circuit by circuit: circuit k owns
 * hyperedges circuit_offsets[k] .. circuit_offsets[k+1]-1 (n_circuits + 1
 * offsets; circuit_ids[e] names the circuit of each hyperedge); bits use
 * that circuit's numbering (its shape from gp_edges_circuit_shape), and
 * gp_edges_detectors / gp_edges_observables give the largest of any circuit. */
uint64_t gp_edges_count(const gp_edges* e);
uint32_t gp_edges_detectors(const gp_edges* e);
uint32_t gp_edges_observables(const gp_edges* e);
const uint64_t* gp_edges_offsets(const gp_edges* e);
const uint32_t* gp_edges_bits(const gp_edges* e);
const double* gp_edges_probabilities(const gp_edges* e);
uint32_t gp_edges_circuits(const gp_edges* e);            /* circuits in the compile (1 without a batch) */
const uint32_t* gp_edges_circuit_ids(const gp_edges* e);  /* per hyperedge: its circuit */
const uint64_t* gp_edges_circuit_offsets(const gp_edges* e);  /* first hyperedge of each circuit, and the count */
int gp_edges_circuit_shape(const gp_edges* e, uint32_t circuit, uint32_t* n_det, uint32_t* n_obs);
/* Detector error model text, one "error(q) D.. L.." line per hyperedge. The
 * caller releases *text with gp_free. GP_E_STATE for a batch result, whose
 * circuits each have their own text (gp_edges_circuit_dem_text). */
int gp_edges_to_dem_text(const gp_edges* e, char** text, size_t* len);
/* Signatures packed as 64-bit words (the layout of paper Sec. 3.1.2's class
 * bit vectors): gp_edges_words gives W, the words per signature (enough for
 * the detectors and observables of the widest circuit of the result), and
 * gp_edges_signatures the U x W row-major array in which bit b % 64 of word
 * b / 64 of row e is set when hyperedge e flips signature bit b (numbered as
 * in gp_edges_bits). The array is built on the first call (thread-safe) and
 * stays valid until gp_edges_free; NULL with gp_last_error set if it cannot
 * be allocated. */
uint32_t gp_edges_words(const gp_edges* e);
const uint64_t* gp_edges_signatures(const gp_edges* e);
int gp_edges_circuit_dem_text(const gp_edges* e, uint32_t circuit, char** text, size_t* len);
void gp_edges_free(gp_edges* e);
void gp_free(void* p);

#ifdef __cplusplus
}
#endif

#endif /* GP_H */
