"""ctypes binding of ``include/gp.h``: one Python function per C entry point,
same names, argument marshalling only. Every computation happens in
``libgp.so``; if the library is missing this module raises instead of falling
back to anything else."""

from __future__ import annotations

import ctypes
import os
import sys
from typing import Optional, Sequence, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgp.so")

GP_OK = 0
STATUS = {
    -1: "GP_E_ARG", -2: "GP_E_PARSE", -3: "GP_E_UNSUPPORTED", -4: "GP_E_BOUNDS",
    -5: "GP_E_NONDETERMINISTIC", -6: "GP_E_NOISE", -7: "GP_E_HIP", -8: "GP_E_OOM",
    -9: "GP_E_COLLISION", -10: "GP_E_STATE", -11: "GP_E_BUSY", -12: "GP_E_INTERNAL",
}

#: every symbol include/gp.h declares
EXPORTS = (
    "gp_last_error", "gp_bounds_from_circuit", "gp_driver_create", "gp_driver_create_from_circuit",
    "gp_driver_destroy", "gp_compile_hypergraph", "gp_lower", "gp_run", "gp_fetch", "gp_sync",
    "gp_driver_stream", "gp_circuit_info_get", "gp_set_timing", "gp_reset_timing", "gp_timing_count",
    "gp_timing_entry", "gp_edges_count", "gp_edges_detectors", "gp_edges_observables",
    "gp_edges_offsets", "gp_edges_bits", "gp_edges_probabilities", "gp_edges_to_dem_text",
    "gp_edges_free", "gp_free", "gp_debug_set_key_bits", "gp_debug_collision_retries",
    "gp_debug_sweep_times", "gp_debug_capture_keys", "gp_debug_class_keys", "gp_debug_set_sort_mode", "gp_refresh_rates", "gp_rates_gradient",
    "gp_set_correlation_level", "gp_bounds_from_batch", "gp_driver_create_from_batch", "gp_lower_batch",
    "gp_edges_circuits", "gp_edges_circuit_ids", "gp_edges_circuit_shape", "gp_edges_circuit_dem_text",
    "gp_edges_circuit_offsets", "gp_server_create", "gp_server_submit", "gp_server_wait", "gp_server_stats",
    "gp_server_destroy", "gp_server_timing", "gp_debug_set_graph", "gp_autotune", "gp_set_fault_cost",
    "gp_debug_set_sweep_shape", "gp_autotune_batch", "gp_tuning_cache_size", "gp_tuning_cache_get",
    "gp_tuning_cache_put", "gp_server_set_admission", "gp_fetch_sizes", "gp_fetch_copy",
    "gp_fetch_circuit_offsets", "gp_circuit_shape",
    "gp_debug_retry_counts", "gp_debug_set_spin_limit", "gp_debug_device_flags",
    "gp_compile_ir", "gp_lower_ir", "gp_lower_batch_ir", "gp_bounds_from_ir", "gp_bounds_from_batch_ir",
    "gp_server_submit_ir", "gp_edges_words", "gp_edges_signatures", "gp_aggregate", "gp_aggregate_backward",
    "gp_structure_id", "gp_aggregate_backward_noalloc",
)


class GpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class GpBounds(ctypes.Structure):
    _fields_ = [
        ("max_qubits", ctypes.c_uint32), ("max_layers", ctypes.c_uint32),
        ("max_measurements", ctypes.c_uint32), ("max_detectors", ctypes.c_uint32),
        ("max_observables", ctypes.c_uint32), ("max_channels", ctypes.c_uint32),
        ("max_faults", ctypes.c_uint64), ("max_ops", ctypes.c_uint64),
        ("max_leaf_bits", ctypes.c_uint64), ("max_slab_words", ctypes.c_uint64),
        ("max_items", ctypes.c_uint64), ("max_branches", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GpCircuitInfo(ctypes.Structure):
    _fields_ = [
        ("n_qubits", ctypes.c_uint32), ("n_layers", ctypes.c_uint32),
        ("n_measurements", ctypes.c_uint32), ("n_detectors", ctypes.c_uint32),
        ("n_observables", ctypes.c_uint32), ("n_words", ctypes.c_uint32),
        ("n_channels", ctypes.c_uint64), ("n_faults", ctypes.c_uint64), ("n_ops", ctypes.c_uint64),
        ("n_items", ctypes.c_uint64), ("slab_words", ctypes.c_uint64),
        ("n_classes", ctypes.c_uint64), ("n_edges", ctypes.c_uint64), ("n_edge_bits", ctypes.c_uint64),
        ("n_live_words", ctypes.c_uint64), ("n_live_faults", ctypes.c_uint64),
        ("n_nonzero_words", ctypes.c_uint64), ("n_circuits", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GpTuning(ctypes.Structure):
    _fields_ = [
        ("fault_cost", ctypes.c_double), ("sweep_block", ctypes.c_int32), ("cached", ctypes.c_int32),
        ("ms", ctypes.c_double),
        ("n_circuits", ctypes.c_uint32), ("n_qubits", ctypes.c_uint32), ("n_layers", ctypes.c_uint32),
        ("n_det", ctypes.c_uint32), ("n_faults", ctypes.c_uint64),
        ("n_obs", ctypes.c_uint32), ("level", ctypes.c_uint32),
        ("grouping", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GpCircuitIr(ctypes.Structure):
    """gp_circuit_ir: a circuit in binary form (parallel per-operation arrays)."""
    _fields_ = [
        ("n_ops", ctypes.c_uint64), ("code", ctypes.POINTER(ctypes.c_uint8)),
        ("q0", ctypes.POINTER(ctypes.c_uint32)), ("q1", ctypes.POINTER(ctypes.c_uint32)),
        ("rate", ctypes.POINTER(ctypes.c_double)), ("n_rec", ctypes.c_uint64),
        ("rec", ctypes.POINTER(ctypes.c_uint32)),
    ]


def circuit_ir(ir: dict):
    """-> (GpCircuitIr, arrays to keep alive) for a dict of numpy arrays "code",
    "q0", "q1", "rate" (one entry per operation) and "rec"."""
    keep = {
        "code": np.ascontiguousarray(ir["code"], dtype=np.uint8),
        "q0": np.ascontiguousarray(ir["q0"], dtype=np.uint32),
        "q1": np.ascontiguousarray(ir["q1"], dtype=np.uint32),
        "rate": np.ascontiguousarray(ir["rate"], dtype=np.float64),
        "rec": np.ascontiguousarray(ir["rec"], dtype=np.uint32),
    }
    n = len(keep["code"])
    for k in ("q0", "q1", "rate"):
        if len(keep[k]) != n:
            raise ValueError(f"binary circuit: '{k}' has {len(keep[k])} entries, 'code' has {n}")

    def ptr(a, t):
        return a.ctypes.data_as(ctypes.POINTER(t)) if len(a) else ctypes.POINTER(t)()

    s = GpCircuitIr(n, ptr(keep["code"], ctypes.c_uint8), ptr(keep["q0"], ctypes.c_uint32),
                    ptr(keep["q1"], ctypes.c_uint32), ptr(keep["rate"], ctypes.c_double), len(keep["rec"]),
                    ptr(keep["rec"], ctypes.c_uint32))
    return s, keep


_lib = None
_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64


def _share_hip_runtime_with_torch() -> None:
    """One HIP runtime per process. PyTorch's ROCm wheel carries its own copy
    of the HIP and HSA runtimes and loads them by file path, while libgp.so
    names the HIP runtime by its soname. If libgp.so came first, the process
    would hold two runtimes and torch would see no GPU (device tensors for
    gp_aggregate and the autograd wrapper would be impossible). Loading
    torch's copy first (by path, without importing torch) lets libgp.so bind
    to it by soname, and a later ``import torch`` finds the same file already
    loaded. Without torch installed, the system runtime is used."""
    import importlib.util
    if "torch" in sys.modules:
        return  # torch's runtime is already the process's runtime
    try:
        spec = importlib.util.find_spec("torch")
    except (ImportError, ValueError):
        spec = None
    if spec is None or not spec.submodule_search_locations:
        return
    hip = os.path.join(list(spec.submodule_search_locations)[0], "lib", "libamdhip64.so")
    if os.path.exists(hip):
        ctypes.CDLL(hip, mode=ctypes.RTLD_GLOBAL)


def load():
    """Load libgp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the compiler has no other implementation to fall back to)")
    _share_hip_runtime_with_torch()
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "gp_last_error": ([], ctypes.c_char_p),
        "gp_bounds_from_circuit": ([ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(GpBounds)], ctypes.c_int),
        "gp_driver_create": ([ctypes.POINTER(GpBounds), ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
        "gp_driver_create_from_circuit": ([ctypes.c_char_p, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_vp)],
                                          ctypes.c_int),
        "gp_driver_destroy": ([_vp], None),
        "gp_compile_hypergraph": ([_vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
        "gp_compile_ir": ([_vp, ctypes.POINTER(GpCircuitIr), ctypes.POINTER(ctypes.c_double), ctypes.c_size_t,
                           ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
        "gp_lower_ir": ([_vp, ctypes.POINTER(GpCircuitIr), ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
                        ctypes.c_int),
        "gp_lower_batch_ir": ([_vp, ctypes.POINTER(GpCircuitIr), ctypes.c_size_t,
                               ctypes.POINTER(ctypes.POINTER(ctypes.c_double)), ctypes.POINTER(ctypes.c_size_t)],
                              ctypes.c_int),
        "gp_bounds_from_ir": ([ctypes.POINTER(GpCircuitIr), ctypes.POINTER(GpBounds)], ctypes.c_int),
        "gp_bounds_from_batch_ir": ([ctypes.POINTER(GpCircuitIr), ctypes.c_size_t, ctypes.POINTER(GpBounds)],
                                    ctypes.c_int),
        "gp_server_submit_ir": ([_vp, ctypes.POINTER(GpCircuitIr), ctypes.POINTER(ctypes.c_double), ctypes.c_size_t,
                                 ctypes.POINTER(_u64)], ctypes.c_int),
        "gp_edges_words": ([_vp], ctypes.c_uint32),
        "gp_aggregate": ([_vp, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
        "gp_aggregate_backward": ([_vp, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp, _vp], ctypes.c_int),
        "gp_aggregate_backward_noalloc": ([_vp, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp, _vp],
                                          ctypes.c_int),
        "gp_structure_id": ([_vp], _u64),
        "gp_edges_signatures": ([_vp], ctypes.POINTER(_u64)),
        "gp_lower": ([_vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
                     ctypes.c_int),
        "gp_run": ([_vp], ctypes.c_int),
        "gp_fetch": ([_vp, ctypes.POINTER(_vp)], ctypes.c_int),
        "gp_sync": ([_vp], ctypes.c_int),
        "gp_driver_stream": ([_vp], _vp),
        "gp_circuit_info_get": ([_vp, ctypes.POINTER(GpCircuitInfo)], ctypes.c_int),
        "gp_set_timing": ([_vp, ctypes.c_int], ctypes.c_int),
        "gp_reset_timing": ([_vp], ctypes.c_int),
        "gp_timing_count": ([_vp], ctypes.c_int),
        "gp_timing_entry": ([_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(_u64)], ctypes.c_int),
        "gp_edges_count": ([_vp], _u64),
        "gp_edges_detectors": ([_vp], ctypes.c_uint32),
        "gp_edges_observables": ([_vp], ctypes.c_uint32),
        "gp_edges_offsets": ([_vp], ctypes.POINTER(_u64)),
        "gp_edges_bits": ([_vp], ctypes.POINTER(ctypes.c_uint32)),
        "gp_edges_probabilities": ([_vp], ctypes.POINTER(ctypes.c_double)),
        "gp_edges_to_dem_text": ([_vp, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_size_t)],
                                 ctypes.c_int),
        "gp_edges_free": ([_vp], None),
        "gp_free": ([_vp], None),
        "gp_debug_set_key_bits": ([_vp, ctypes.c_int], ctypes.c_int),
        "gp_debug_collision_retries": ([_vp], _u64),
        "gp_debug_set_sort_mode": ([_vp, ctypes.c_int], ctypes.c_int),
        "gp_debug_set_graph": ([_vp, ctypes.c_int], ctypes.c_int),
        "gp_debug_set_sweep_shape": ([_vp, ctypes.c_int], ctypes.c_int),
        "gp_autotune": ([_vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(GpTuning)],
                        ctypes.c_int),
        "gp_autotune_batch": ([_vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_size_t),
                               ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(GpTuning)], ctypes.c_int),
        "gp_tuning_cache_size": ([], ctypes.c_size_t),
        "gp_tuning_cache_get": ([ctypes.c_size_t, ctypes.POINTER(GpTuning)], ctypes.c_int),
        "gp_tuning_cache_put": ([ctypes.POINTER(GpTuning)], ctypes.c_int),
        "gp_set_fault_cost": ([_vp, ctypes.c_double], ctypes.c_int),
        "gp_refresh_rates": ([_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t], ctypes.c_int),
        "gp_set_correlation_level": ([_vp, ctypes.c_int], ctypes.c_int),
        "gp_rates_gradient": ([_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t,
                               ctypes.POINTER(ctypes.c_double), ctypes.c_size_t], ctypes.c_int),
        "gp_debug_sweep_times": ([_vp, ctypes.POINTER(_u64), _u64, ctypes.POINTER(_u64),
                                  ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "gp_debug_capture_keys": ([_vp, ctypes.c_int], ctypes.c_int),
        "gp_debug_class_keys": ([_vp, ctypes.POINTER(_u64), _u64, ctypes.POINTER(_u64),
                                 ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
        "gp_bounds_from_batch": ([ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_size_t), ctypes.c_size_t,
                                  ctypes.POINTER(GpBounds)], ctypes.c_int),
        "gp_driver_create_from_batch": ([ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_size_t),
                                         ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
        "gp_lower_batch": ([_vp, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_size_t),
                            ctypes.POINTER(ctypes.POINTER(ctypes.c_double)), ctypes.POINTER(ctypes.c_size_t),
                            ctypes.c_size_t], ctypes.c_int),
        "gp_edges_circuits": ([_vp], ctypes.c_uint32),
        "gp_edges_circuit_ids": ([_vp], ctypes.POINTER(ctypes.c_uint32)),
        "gp_edges_circuit_offsets": ([_vp], ctypes.POINTER(_u64)),
        "gp_server_create": ([ctypes.POINTER(GpBounds), ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
        "gp_server_submit": ([_vp, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t,
                              ctypes.POINTER(_u64)], ctypes.c_int),
        "gp_server_wait": ([_vp, _u64, ctypes.c_int64, ctypes.POINTER(_vp), ctypes.POINTER(_u64)], ctypes.c_int),
        "gp_server_stats": ([_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64)], ctypes.c_int),
        "gp_server_set_admission": ([_vp, _u64, _u64], ctypes.c_int),
        "gp_fetch_sizes": ([_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_uint32),
                            ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
        "gp_fetch_copy": ([_vp, _vp, _vp, _vp], ctypes.c_int),
        "gp_fetch_circuit_offsets": ([_vp, _vp], ctypes.c_int),
        "gp_circuit_shape": ([_vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)],
                             ctypes.c_int),
        "gp_server_destroy": ([_vp], None),
        "gp_server_timing": ([_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "gp_edges_circuit_shape": ([_vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                    ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
        "gp_edges_circuit_dem_text": ([_vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "gp_debug_retry_counts": ([_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64)],
                                  ctypes.c_int),
        "gp_debug_set_spin_limit": ([_vp, ctypes.c_uint32], ctypes.c_int),
        "gp_debug_device_flags": ([_vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                   ctypes.c_int], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != GP_OK:
        raise GpError(rc, load().gp_last_error().decode(errors="replace"))


def _rates(rates: Optional[Sequence[float]]):
    if rates is None:
        return None, 0, None
    arr = np.ascontiguousarray(rates, dtype=np.float64)
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(arr), arr


# ---------------------------------------------------------------- functions

def gp_last_error() -> str:
    return load().gp_last_error().decode(errors="replace")


def gp_bounds_from_circuit(text: str) -> GpBounds:
    raw = text.encode()
    b = GpBounds()
    _check(load().gp_bounds_from_circuit(raw, len(raw), ctypes.byref(b)))
    return b


def gp_driver_create(bounds: GpBounds, device: int = 0) -> int:
    h = _vp()
    _check(load().gp_driver_create(ctypes.byref(bounds), device, ctypes.byref(h)))
    return h.value


def gp_driver_create_from_circuit(text: str, device: int = 0) -> int:
    raw = text.encode()
    h = _vp()
    _check(load().gp_driver_create_from_circuit(raw, len(raw), device, ctypes.byref(h)))
    return h.value


def _texts(texts: Sequence[str]):
    raw = [t.encode() for t in texts]
    arr = (ctypes.c_char_p * max(len(raw), 1))(*raw)
    lens = (ctypes.c_size_t * max(len(raw), 1))(*[len(r) for r in raw])
    return arr, lens, raw


def gp_bounds_from_batch(texts: Sequence[str]) -> GpBounds:
    arr, lens, _keep = _texts(texts)
    b = GpBounds()
    _check(load().gp_bounds_from_batch(arr, lens, len(texts), ctypes.byref(b)))
    return b


def gp_driver_create_from_batch(texts: Sequence[str], device: int = 0) -> int:
    arr, lens, _keep = _texts(texts)
    h = _vp()
    _check(load().gp_driver_create_from_batch(arr, lens, len(texts), device, ctypes.byref(h)))
    return h.value


def gp_lower_batch(drv: int, texts: Sequence[str], rates: Optional[Sequence[Optional[Sequence[float]]]] = None) -> None:
    arr, lens, _keep = _texts(texts)
    n = len(texts)
    if rates is None:
        _check(load().gp_lower_batch(drv, arr, lens, None, None, n))
        return
    if len(rates) != n:
        raise ValueError("one rate array (or None) per circuit")
    dp = ctypes.POINTER(ctypes.c_double)
    keep = [None if r is None else np.ascontiguousarray(r, dtype=np.float64) for r in rates]
    ptrs = (dp * max(n, 1))(*[dp() if r is None else r.ctypes.data_as(dp) for r in keep])
    nr = (ctypes.c_size_t * max(n, 1))(*[0 if r is None else len(r) for r in keep])
    _check(load().gp_lower_batch(drv, arr, lens, ptrs, nr, n))


def gp_driver_destroy(drv: int) -> None:
    load().gp_driver_destroy(drv)


def gp_compile_hypergraph(drv: int, text: str, rates: Optional[Sequence[float]] = None, level: int = -1) -> int:
    raw = text.encode()
    rp, nr, _keep = _rates(rates)
    h = _vp()
    _check(load().gp_compile_hypergraph(drv, raw, len(raw), rp, nr, level, ctypes.byref(h)))
    return h.value


def gp_compile_ir(drv: int, ir: dict, rates: Optional[Sequence[float]] = None, level: int = -1) -> int:
    s, _keep = circuit_ir(ir)
    rp, nr, _keep_r = _rates(rates)
    h = _vp()
    _check(load().gp_compile_ir(drv, ctypes.byref(s), rp, nr, level, ctypes.byref(h)))
    return h.value


def gp_lower_ir(drv: int, ir: dict, rates: Optional[Sequence[float]] = None) -> None:
    s, _keep = circuit_ir(ir)
    rp, nr, _keep_r = _rates(rates)
    _check(load().gp_lower_ir(drv, ctypes.byref(s), rp, nr))


def _ir_array(irs: Sequence[dict]):
    made = [circuit_ir(ir) for ir in irs]
    arr = (GpCircuitIr * max(len(made), 1))(*[m[0] for m in made])
    return arr, made


def gp_lower_batch_ir(drv: int, irs: Sequence[dict],
                      rates: Optional[Sequence[Optional[Sequence[float]]]] = None) -> None:
    arr, _keep = _ir_array(irs)
    n = len(irs)
    if rates is None:
        _check(load().gp_lower_batch_ir(drv, arr, n, None, None))
        return
    if len(rates) != n:
        raise ValueError("one rate array (or None) per circuit")
    dp = ctypes.POINTER(ctypes.c_double)
    keep = [None if r is None else np.ascontiguousarray(r, dtype=np.float64) for r in rates]
    ptrs = (dp * max(n, 1))(*[dp() if r is None else r.ctypes.data_as(dp) for r in keep])
    nr = (ctypes.c_size_t * max(n, 1))(*[0 if r is None else len(r) for r in keep])
    _check(load().gp_lower_batch_ir(drv, arr, n, ptrs, nr))


def gp_bounds_from_ir(ir: dict) -> GpBounds:
    s, _keep = circuit_ir(ir)
    b = GpBounds()
    _check(load().gp_bounds_from_ir(ctypes.byref(s), ctypes.byref(b)))
    return b


def gp_bounds_from_batch_ir(irs: Sequence[dict]) -> GpBounds:
    arr, _keep = _ir_array(irs)
    b = GpBounds()
    _check(load().gp_bounds_from_batch_ir(arr, len(irs), ctypes.byref(b)))
    return b


def gp_edges_words(e: int) -> int:
    return int(load().gp_edges_words(e))


def gp_edges_signatures(e: int) -> np.ndarray:
    """-> the U x W packed signatures (uint64), copied."""
    n, w = gp_edges_count(e), gp_edges_words(e)
    p = load().gp_edges_signatures(e)
    if not p:
        _check(-8)
    if n == 0 or w == 0:
        return np.zeros((n, w), dtype=np.uint64)
    return np.ctypeslib.as_array(p, shape=(n * w,)).reshape(n, w).copy()


def gp_lower(drv: int, text: str, rates: Optional[Sequence[float]] = None) -> None:
    raw = text.encode()
    rp, nr, _keep = _rates(rates)
    _check(load().gp_lower(drv, raw, len(raw), rp, nr))


def gp_run(drv: int) -> None:
    _check(load().gp_run(drv))


def gp_fetch(drv: int) -> int:
    h = _vp()
    _check(load().gp_fetch(drv, ctypes.byref(h)))
    return h.value


def gp_fetch_arrays(drv: int, n_circuits: int = 1):
    """Result with one host copy -> (n_det, n_obs, offsets, bits, q,
    circuit_offsets); the hyperedges are listed circuit by circuit."""
    lib = load()
    U, nb = _u64(), _u64()
    nd, no = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib.gp_fetch_sizes(drv, ctypes.byref(U), ctypes.byref(nb), ctypes.byref(nd), ctypes.byref(no)))
    off = np.empty(U.value + 1, dtype=np.uint64)
    bits = np.empty(nb.value, dtype=np.uint32)
    q = np.empty(U.value, dtype=np.float64)
    _check(lib.gp_fetch_copy(drv, off.ctypes.data, bits.ctypes.data if nb.value else None,
                             q.ctypes.data if U.value else None))
    coff = np.empty(n_circuits + 1, dtype=np.uint64)
    _check(lib.gp_fetch_circuit_offsets(drv, coff.ctypes.data))
    return nd.value, no.value, off, bits, q, coff


def gp_sync(drv: int) -> None:
    _check(load().gp_sync(drv))


def gp_driver_stream(drv: int) -> int:
    return load().gp_driver_stream(drv) or 0


def gp_circuit_info_get(drv: int) -> GpCircuitInfo:
    i = GpCircuitInfo()
    _check(load().gp_circuit_info_get(drv, ctypes.byref(i)))
    return i


def gp_set_timing(drv: int, enable: bool) -> None:
    _check(load().gp_set_timing(drv, int(enable)))


def gp_reset_timing(drv: int) -> None:
    _check(load().gp_reset_timing(drv))


def gp_timing_count(drv: int) -> int:
    return load().gp_timing_count(drv)


def gp_timing_entry(drv: int, index: int) -> Tuple[str, float, int]:
    name = ctypes.c_char_p()
    ms = ctypes.c_double()
    n = _u64()
    _check(load().gp_timing_entry(drv, index, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(n)))
    return name.value.decode(), ms.value, n.value


def gp_edges_count(e: int) -> int:
    return int(load().gp_edges_count(e))


def gp_edges_detectors(e: int) -> int:
    return int(load().gp_edges_detectors(e))


def gp_edges_observables(e: int) -> int:
    return int(load().gp_edges_observables(e))


def gp_edges_offsets(e: int) -> np.ndarray:
    n = gp_edges_count(e) + 1
    return np.ctypeslib.as_array(load().gp_edges_offsets(e), shape=(n,)).copy()


def gp_edges_bits(e: int) -> np.ndarray:
    n = gp_edges_count(e) + 1
    nb = int(np.ctypeslib.as_array(load().gp_edges_offsets(e), shape=(n,))[-1])
    if nb == 0:
        return np.zeros(0, dtype=np.uint32)
    return np.ctypeslib.as_array(load().gp_edges_bits(e), shape=(nb,)).copy()


def gp_edges_probabilities(e: int) -> np.ndarray:
    n = gp_edges_count(e)
    if n == 0:
        return np.zeros(0, dtype=np.float64)
    return np.ctypeslib.as_array(load().gp_edges_probabilities(e), shape=(n,)).copy()


def gp_edges_to_dem_text(e: int) -> str:
    p = ctypes.c_void_p()
    n = ctypes.c_size_t()
    _check(load().gp_edges_to_dem_text(e, ctypes.byref(p), ctypes.byref(n)))
    try:
        return ctypes.string_at(p.value, n.value).decode() if n.value else ""
    finally:
        load().gp_free(p)


def gp_edges_circuits(e: int) -> int:
    return int(load().gp_edges_circuits(e))


def gp_edges_circuit_ids(e: int) -> np.ndarray:
    n = gp_edges_count(e)
    if n == 0:
        return np.zeros(0, dtype=np.uint32)
    return np.ctypeslib.as_array(load().gp_edges_circuit_ids(e), shape=(n,)).copy()


def gp_edges_circuit_offsets(e: int) -> np.ndarray:
    n = gp_edges_circuits(e) + 1
    return np.ctypeslib.as_array(load().gp_edges_circuit_offsets(e), shape=(n,)).copy()


def gp_circuit_shape(drv: int, circuit: int) -> Tuple[int, int]:
    """(detectors, observables) of circuit `circuit` of the driver's lowering."""
    d = ctypes.c_uint32()
    o = ctypes.c_uint32()
    _check(load().gp_circuit_shape(drv, circuit, ctypes.byref(d), ctypes.byref(o)))
    return d.value, o.value


def gp_edges_circuit_shape(e: int, circuit: int) -> Tuple[int, int]:
    d = ctypes.c_uint32()
    o = ctypes.c_uint32()
    _check(load().gp_edges_circuit_shape(e, circuit, ctypes.byref(d), ctypes.byref(o)))
    return d.value, o.value


def gp_edges_circuit_dem_text(e: int, circuit: int) -> str:
    p = ctypes.c_void_p()
    n = ctypes.c_size_t()
    _check(load().gp_edges_circuit_dem_text(e, circuit, ctypes.byref(p), ctypes.byref(n)))
    try:
        return ctypes.string_at(p.value, n.value).decode() if n.value else ""
    finally:
        load().gp_free(p)


def gp_edges_free(e: int) -> None:
    load().gp_edges_free(e)


def gp_debug_set_key_bits(drv: int, bits: int) -> None:
    _check(load().gp_debug_set_key_bits(drv, bits))


def gp_set_correlation_level(drv: int, level: int) -> None:
    _check(load().gp_set_correlation_level(drv, level))


def gp_refresh_rates(drv: int, rates: Sequence[float]) -> None:
    r = np.ascontiguousarray(rates, dtype=np.float64)
    _check(load().gp_refresh_rates(drv, r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(r)))


def gp_rates_gradient(drv: int, dl_dq: Sequence[float], n_rates: int) -> np.ndarray:
    g = np.ascontiguousarray(dl_dq, dtype=np.float64)
    out = np.zeros(n_rates, dtype=np.float64)
    _check(load().gp_rates_gradient(drv, g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(g),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n_rates))
    return out


def gp_debug_set_sort_mode(drv: int, mode: int) -> None:
    _check(load().gp_debug_set_sort_mode(drv, mode))


def gp_debug_set_graph(drv: int, enable: bool) -> None:
    _check(load().gp_debug_set_graph(drv, int(enable)))


def gp_autotune(drv: int, text: str, iters: int = 10) -> dict:
    """-> the chosen tuning (fault cost, sweep work-group, ms, cached, shape key)."""
    raw = text.encode()
    t = GpTuning()
    _check(load().gp_autotune(drv, raw, len(raw), iters, ctypes.byref(t)))
    return t.as_dict()


def gp_autotune_batch(drv: int, texts: Sequence[str], iters: int = 10) -> dict:
    arr, lens, _keep = _texts(texts)
    t = GpTuning()
    _check(load().gp_autotune_batch(drv, arr, lens, len(texts), iters, ctypes.byref(t)))
    return t.as_dict()


def gp_tuning_cache() -> list:
    """Every entry of the process-wide tuning cache, as dicts."""
    lib = load()
    out = []
    for i in range(lib.gp_tuning_cache_size()):
        t = GpTuning()
        _check(lib.gp_tuning_cache_get(i, ctypes.byref(t)))
        out.append(t.as_dict())
    return out


def gp_tuning_cache_put(entry: dict) -> None:
    t = GpTuning()
    for k, _ in GpTuning._fields_:
        if k in ("grouping", "reserved"):
            setattr(t, k, entry.get(k, 0))   # files written before the grouping was tuned
        elif k != "cached":
            setattr(t, k, entry[k])
    _check(load().gp_tuning_cache_put(ctypes.byref(t)))


def gp_set_fault_cost(drv: int, fault_cost: float) -> None:
    _check(load().gp_set_fault_cost(drv, fault_cost))


def gp_debug_set_sweep_shape(drv: int, shape: int) -> None:
    _check(load().gp_debug_set_sweep_shape(drv, shape))


def gp_debug_collision_retries(drv: int) -> int:
    return int(load().gp_debug_collision_retries(drv))


def gp_debug_sweep_times(drv: int, cap: int = 1 << 16):
    """-> (array of (start, end) device clock stamps per sweep item, clock Hz)."""
    buf = np.zeros(cap, dtype=np.uint64)
    n = _u64()
    hz = ctypes.c_double()
    _check(load().gp_debug_sweep_times(drv, buf.ctypes.data_as(ctypes.POINTER(_u64)), cap, ctypes.byref(n),
                                       ctypes.byref(hz)))
    m = min(int(n.value), cap // 2)
    return buf[:2 * m].reshape(-1, 2), hz.value


def gp_debug_capture_keys(drv: int, enable: bool = True) -> None:
    _check(load().gp_debug_capture_keys(drv, int(enable)))


def gp_debug_class_keys(drv: int):
    """-> (per-position class keys of the last gp_run as uint64, key bits kept)."""
    n = _u64()
    bits = ctypes.c_uint32()
    _check(load().gp_debug_class_keys(drv, None, 0, ctypes.byref(n), ctypes.byref(bits)))
    buf = np.zeros(max(int(n.value), 1), dtype=np.uint64)
    _check(load().gp_debug_class_keys(drv, buf.ctypes.data_as(ctypes.POINTER(_u64)), int(n.value),
                                      ctypes.byref(n), ctypes.byref(bits)))
    return buf[:int(n.value)], int(bits.value)


def gp_server_create(bounds: GpBounds, device: int = 0) -> int:
    h = _vp()
    _check(load().gp_server_create(ctypes.byref(bounds), device, ctypes.byref(h)))
    return h.value


def gp_server_submit(srv: int, text: str, rates: Optional[Sequence[float]] = None) -> int:
    raw = text.encode()
    rp, nr, _keep = _rates(rates)
    t = _u64()
    _check(load().gp_server_submit(srv, raw, len(raw), rp, nr, ctypes.byref(t)))
    return t.value


def gp_server_submit_ir(srv: int, ir: dict, rates: Optional[Sequence[float]] = None) -> int:
    s, _keep = circuit_ir(ir)
    rp, nr, _keep_r = _rates(rates)
    t = _u64()
    _check(load().gp_server_submit_ir(srv, ctypes.byref(s), rp, nr, ctypes.byref(t)))
    return t.value


def gp_server_wait(srv: int, ticket: int, timeout_us: int = -1) -> Tuple[int, int]:
    """-> (gp_edges handle, latency in ns from submit to completion)."""
    h = _vp()
    lat = _u64()
    _check(load().gp_server_wait(srv, ticket, timeout_us, ctypes.byref(h), ctypes.byref(lat)))
    return h.value, lat.value


def gp_server_set_admission(srv: int, max_requests: int, max_bytes: int) -> None:
    _check(load().gp_server_set_admission(srv, max_requests, max_bytes))


def gp_server_stats(srv: int) -> Tuple[int, int, int]:
    b, r, m = _u64(), _u64(), _u64()
    _check(load().gp_server_stats(srv, ctypes.byref(b), ctypes.byref(r), ctypes.byref(m)))
    return b.value, r.value, m.value


def gp_server_destroy(srv: int) -> None:
    load().gp_server_destroy(srv)


def gp_server_timing(srv: int) -> Tuple[float, float, float, float, float]:
    v = [ctypes.c_double() for _ in range(5)]
    _check(load().gp_server_timing(srv, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)



def gp_debug_retry_counts(drv: int) -> dict:
    """-> re-runs by cause: {"lookback", "bucket", "collision"}."""
    a, b, c = _u64(), _u64(), _u64()
    _check(load().gp_debug_retry_counts(drv, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return {"lookback": a.value, "bucket": b.value, "collision": c.value}


def gp_debug_set_spin_limit(drv: int, limit: int) -> None:
    _check(load().gp_debug_set_spin_limit(drv, limit))


def gp_debug_device_flags(drv: int, clear_seen: bool = False) -> Tuple[int, int]:
    """-> (flags of the last compile, flags raised since the last clear)."""
    f, seen = ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().gp_debug_device_flags(drv, ctypes.byref(f), ctypes.byref(seen), int(clear_seen)))
    return f.value, seen.value


def gp_aggregate(drv: int, d_rates: int, n_rates: int, d_q: int, n_edges: int, stream: int = 0) -> None:
    """Device pointers (integers) and a hipStream_t (0: the driver's stream)."""
    _check(load().gp_aggregate(drv, d_rates or None, n_rates, d_q or None, n_edges, stream or None))


def gp_aggregate_backward(drv: int, d_rates: int, n_rates: int, d_gq: int, n_edges: int, d_grates: int,
                          stream: int = 0) -> None:
    _check(load().gp_aggregate_backward(drv, d_rates or None, n_rates, d_gq or None, n_edges, d_grates or None,
                                        stream or None))


def gp_aggregate_backward_noalloc(drv: int, d_rates: int, n_rates: int, d_gq: int, n_edges: int, d_grates: int,
                                  stream: int = 0) -> None:
    """gp_aggregate_backward with its per-fault scratch in the library's
    static device array (no allocation in the call)."""
    _check(load().gp_aggregate_backward_noalloc(drv, d_rates or None, n_rates, d_gq or None, n_edges,
                                                d_grates or None, stream or None))


def gp_structure_id(drv: int) -> int:
    return int(load().gp_structure_id(drv))
