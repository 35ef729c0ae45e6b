"""Python face of the compiler, shaped like the paper's Listing 1 (Sec. 3.4):
a driver built from a maximum circuit reuses its device buffers for every
circuit within those bounds.

    drv = get_driver(max_circuit_text)
    dem = drv.compile_detector_error_model(circuit_text)
    hg = drv.compile_hypergraph(circuit_text, rates)   # arrays of the edges
"""

from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _gp


@dataclasses.dataclass
class Hypergraph:
    """Hyperedge e: bits[offsets[e]:offsets[e+1]] (detector b < n_detectors,
    else observable b - n_detectors) with probability q[e]."""
    n_detectors: int
    n_observables: int
    offsets: np.ndarray
    bits: np.ndarray
    q: np.ndarray
    #: the signatures packed as 64-bit words (U x W, see gp_edges_signatures),
    #: when requested
    words: Optional[np.ndarray] = None

    def __len__(self) -> int:
        return len(self.q)

    def edges(self) -> Dict[Tuple[int, ...], float]:
        out = {}
        for e in range(len(self.q)):
            out[tuple(int(x) for x in self.bits[self.offsets[e]:self.offsets[e + 1]])] = float(self.q[e])
        return out


def _take(handle: int, words: bool = False) -> Hypergraph:
    try:
        return Hypergraph(
            n_detectors=_gp.gp_edges_detectors(handle),
            n_observables=_gp.gp_edges_observables(handle),
            offsets=_gp.gp_edges_offsets(handle),
            bits=_gp.gp_edges_bits(handle),
            q=_gp.gp_edges_probabilities(handle),
            words=_gp.gp_edges_signatures(handle) if words else None,
        )
    finally:
        _gp.gp_edges_free(handle)


def _take_batch(handle: int) -> List[Hypergraph]:
    """Split a batch result (listed circuit by circuit) into one Hypergraph per circuit."""
    try:
        off = _gp.gp_edges_offsets(handle)
        bits = _gp.gp_edges_bits(handle)
        q = _gp.gp_edges_probabilities(handle)
        cut = _gp.gp_edges_circuit_offsets(handle)
        shapes = [_gp.gp_edges_circuit_shape(handle, k) for k in range(len(cut) - 1)]
    finally:
        _gp.gp_edges_free(handle)
    out = []
    for k, (nd, no) in enumerate(shapes):
        a, b = int(cut[k]), int(cut[k + 1])
        o = off[a:b + 1]
        out.append(Hypergraph(n_detectors=nd, n_observables=no, offsets=o - o[0],
                              bits=bits[int(o[0]):int(o[-1])], q=q[a:b]))
    return out


class Driver:
    """Owns one gp_driver (device buffers + stream) on one HIP device."""

    def __init__(self, bounds: _gp.GpBounds, device: int = 0):
        self.bounds = bounds
        self._batch = False  # the current lowering is a batch (fetched with gp_fetch)
        self.handle = _gp.gp_driver_create(bounds, device)

    @classmethod
    def from_circuit(cls, max_circuit: str, device: int = 0) -> "Driver":
        return cls(_gp.gp_bounds_from_circuit(max_circuit), device)

    @classmethod
    def from_batch(cls, circuits: Sequence[str], device: int = 0) -> "Driver":
        """A driver sized for compiling `circuits` together as one batch."""
        return cls(_gp.gp_bounds_from_batch(circuits), device)

    @classmethod
    def from_ir(cls, max_ir: dict, device: int = 0) -> "Driver":
        """A driver sized for a circuit in binary form (see gp_circuit_ir)."""
        return cls(_gp.gp_bounds_from_ir(max_ir), device)

    @classmethod
    def from_batch_ir(cls, irs: Sequence[dict], device: int = 0) -> "Driver":
        return cls(_gp.gp_bounds_from_batch_ir(irs), device)

    def close(self) -> None:
        if self.handle:
            _gp.gp_driver_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # whole path
    def compile_hypergraph(self, circuit: str, rates: Optional[Sequence[float]] = None,
                           level: Optional[int] = None, words: bool = False) -> Hypergraph:
        """`level`: Table 1 correlation level for this compile (None: the
        driver's); `words`: also return the packed signatures."""
        if level is None and not words:
            self.lower(circuit, rates)
            self.run()
            return self.fetch()
        self._batch = False
        return _take(_gp.gp_compile_hypergraph(self.handle, circuit, rates, -1 if level is None else level), words)

    def compile_ir(self, ir: dict, rates: Optional[Sequence[float]] = None, level: Optional[int] = None,
                   words: bool = False) -> Hypergraph:
        """The same for a circuit in binary form (dict of arrays, see
        workloads' Circuit.ir and gp_circuit_ir)."""
        if level is None and not words:
            self.lower_ir(ir, rates)
            self.run()
            return self.fetch()
        self._batch = False
        return _take(_gp.gp_compile_ir(self.handle, ir, rates, -1 if level is None else level), words)

    def compile_detector_error_model(self, circuit: str, rates: Optional[Sequence[float]] = None) -> str:
        h = _gp.gp_compile_hypergraph(self.handle, circuit, rates)
        try:
            return _gp.gp_edges_to_dem_text(h)
        finally:
            _gp.gp_edges_free(h)

    def compile_batch(self, circuits: Sequence[str],
                      rates: Optional[Sequence[Optional[Sequence[float]]]] = None) -> List[Hypergraph]:
        """Compile several circuits in one pass of each stage; one Hypergraph
        per circuit, each equal to what compiling that circuit alone gives."""
        self.lower_batch(circuits, rates)
        self.run()
        return self.fetch_batch()

    # split path
    def lower(self, circuit: str, rates: Optional[Sequence[float]] = None) -> None:
        self._batch = False
        _gp.gp_lower(self.handle, circuit, rates)

    def lower_batch(self, circuits: Sequence[str],
                    rates: Optional[Sequence[Optional[Sequence[float]]]] = None) -> None:
        self._batch = True
        _gp.gp_lower_batch(self.handle, circuits, rates)

    def lower_ir(self, ir: dict, rates: Optional[Sequence[float]] = None) -> None:
        self._batch = False
        _gp.gp_lower_ir(self.handle, ir, rates)

    def lower_batch_ir(self, irs: Sequence[dict],
                       rates: Optional[Sequence[Optional[Sequence[float]]]] = None) -> None:
        self._batch = True
        _gp.gp_lower_batch_ir(self.handle, irs, rates)

    def compile_batch_ir(self, irs: Sequence[dict],
                         rates: Optional[Sequence[Optional[Sequence[float]]]] = None) -> List[Hypergraph]:
        self.lower_batch_ir(irs, rates)
        self.run()
        return self.fetch_batch()

    def fetch_batch(self) -> List[Hypergraph]:
        """One Hypergraph per circuit of the batch (one host copy of the
        result; each circuit's arrays are views of it, its offsets rebased)."""
        n = int(self.info()["n_circuits"])
        _, _, off, bits, q, coff = _gp.gp_fetch_arrays(self.handle, n)
        out = []
        for k in range(n):
            a, b = int(coff[k]), int(coff[k + 1])
            nd, no = _gp.gp_circuit_shape(self.handle, k)
            o = off[a:b + 1]
            out.append(Hypergraph(n_detectors=nd, n_observables=no, offsets=o - o[0],
                                  bits=bits[int(o[0]):int(o[-1])], q=q[a:b]))
        return out

    def run(self) -> None:
        _gp.gp_run(self.handle)

    def sync(self) -> None:
        _gp.gp_sync(self.handle)

    def fetch(self) -> Hypergraph:
        """The current compile's hyperedges (a batch: all circuits', listed
        circuit by circuit, as one Hypergraph; see fetch_batch)."""
        if self._batch:
            return _take(_gp.gp_fetch(self.handle))
        nd, no, off, bits, q, _ = _gp.gp_fetch_arrays(self.handle)
        return Hypergraph(n_detectors=nd, n_observables=no, offsets=off, bits=bits, q=q)

    def info(self) -> dict:
        return _gp.gp_circuit_info_get(self.handle).as_dict()

    def autotune(self, circuit: str, iters: int = 10) -> Dict[str, float]:
        """Time the stage-1 candidates (observable range cut, work-group size)
        on `circuit` and keep the fastest for the following compiles; a shape
        tuned before in this process comes from the cache (see gp_autotune)."""
        return _gp.gp_autotune(self.handle, circuit, iters)

    def autotune_batch(self, circuits: Sequence[str], iters: int = 10) -> Dict[str, float]:
        """The same for a batch of circuits (see gp_autotune_batch)."""
        return _gp.gp_autotune_batch(self.handle, list(circuits), iters)

    def set_correlation_level(self, level: int) -> None:
        """Table 1 level (0, 1 or 2 = every Pauli) for the following compiles."""
        _gp.gp_set_correlation_level(self.handle, level)

    # fixed structure: new rates, and the adjoint of stage 2
    def refresh_rates(self, rates: Sequence[float]) -> Hypergraph:
        """Same hyperedges (same order) as the last fetched compile, with the
        probabilities for `rates` (per channel, program order)."""
        _gp.gp_refresh_rates(self.handle, rates)
        return self.fetch()

    def rates_gradient(self, dl_dq: Sequence[float]) -> np.ndarray:
        """dL/d(rate) per channel (program order) from dL/dq per hyperedge
        (order of the last fetch), at the current rates."""
        return _gp.gp_rates_gradient(self.handle, dl_dq, int(self.info()["n_channels"]))

    def set_timing(self, enable: bool) -> None:
        _gp.gp_set_timing(self.handle, enable)

    def reset_timing(self) -> None:
        _gp.gp_reset_timing(self.handle)

    def timing(self) -> Dict[str, Tuple[float, int]]:
        out = {}
        for k in range(_gp.gp_timing_count(self.handle)):
            name, ms, n = _gp.gp_timing_entry(self.handle, k)
            if n:
                out[name] = (ms, n)
        return out


class Server:
    """Continuous-batching request server (gp_server): submit circuits as they
    arrive, wait for each one's hypergraph. `batch_bounds` bound one batch
    (see Driver.from_batch / gp_bounds_from_batch for a set of circuits that
    must fit in one)."""

    def __init__(self, batch_bounds: _gp.GpBounds, device: int = 0):
        self.bounds = batch_bounds
        self.handle = _gp.gp_server_create(batch_bounds, device)

    @classmethod
    def for_circuits(cls, circuits: Sequence[str], max_batch: Optional[int] = None, device: int = 0) -> "Server":
        """A server sized so that a batch may hold all of `circuits` at once;
        `max_batch` (if given) caps the circuits per batch."""
        b = _gp.gp_bounds_from_batch(circuits)
        if max_batch is not None:
            b.max_branches = max(1, min(int(max_batch), b.max_branches))
        return cls(b, device)

    def submit(self, circuit: str, rates: Optional[Sequence[float]] = None) -> int:
        """-> ticket. Raises GpError GP_E_BUSY (code -11) when the server holds
        its admission limit (see set_admission)."""
        return _gp.gp_server_submit(self.handle, circuit, rates)

    def submit_ir(self, ir: dict, rates: Optional[Sequence[float]] = None) -> int:
        """submit() for a circuit in binary form (its arrays are copied)."""
        return _gp.gp_server_submit_ir(self.handle, ir, rates)

    def set_admission(self, max_requests: int, max_bytes: int) -> None:
        """Limits on live requests (submitted, not yet collected) and on the
        host bytes they hold (see gp_server_set_admission)."""
        _gp.gp_server_set_admission(self.handle, max_requests, max_bytes)

    def wait(self, ticket: int, timeout_us: int = -1) -> Tuple[Hypergraph, float]:
        """-> (hypergraph, latency in ms from submit to completion)."""
        h, lat = _gp.gp_server_wait(self.handle, ticket, timeout_us)
        return _take(h), lat * 1e-6

    def stats(self) -> Dict[str, int]:
        b, r, m = _gp.gp_server_stats(self.handle)
        lo, up, fe, wa, dl = _gp.gp_server_timing(self.handle)
        return {"batches": b, "requests": r, "max_batch": m, "worker_lower_ms": lo, "worker_upload_ms": up,
                "worker_fetch_ms": fe, "worker_wait_ms": wa, "worker_download_ms": dl}

    def close(self) -> None:
        if self.handle:
            _gp.gp_server_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def save_tuning(path: str) -> int:
    """Write the process-wide tuning cache to `path` as JSON (one entry per
    lowered shape); returns the number of entries."""
    import json
    entries = _gp.gp_tuning_cache()
    for e in entries:
        e.pop("cached", None)
    with open(path, "w") as fh:
        json.dump({"gp_tuning": entries}, fh, indent=1)
    return len(entries)


def load_tuning(path: str) -> int:
    """Insert the entries of a JSON file written by save_tuning into the
    cache; returns how many were read."""
    import json
    with open(path) as fh:
        entries = json.load(fh)["gp_tuning"]
    for e in entries:
        _gp.gp_tuning_cache_put(e)
    return len(entries)


def get_driver(max_circuit: str, device: int = 0) -> Driver:
    """Listing 1: a driver whose buffers are sized for `max_circuit`."""
    return Driver.from_circuit(max_circuit, device)
