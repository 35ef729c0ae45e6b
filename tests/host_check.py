"""Loader for the test-only CPU interpreter of the lowered tables (host_check.cpp)."""

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "host_check.cpp")
LOWER = os.path.join(ROOT, "paper_2604_16613_amd", "csrc", "lower.cpp")
OUT = os.path.join(HERE, "_build", "libhostcheck.so")

_lib = None


def _load():
    global _lib
    if _lib is None:
        os.makedirs(os.path.dirname(OUT), exist_ok=True)
        newest = max(os.path.getmtime(SRC), os.path.getmtime(LOWER),
                     os.path.getmtime(os.path.join(ROOT, "paper_2604_16613_amd", "csrc", "lower.h")))
        if not os.path.exists(OUT) or os.path.getmtime(OUT) < newest:
            # built under a name of this process's own, then renamed into place
            # in one step: parallel test workers never load a half-written file
            tmp = f"{OUT}.{os.getpid()}.tmp"
            subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                            "-I", os.path.join(ROOT, "include"),
                            "-I", os.path.join(ROOT, "paper_2604_16613_amd", "csrc"),
                            SRC, LOWER, "-o", tmp], check=True)
            os.replace(tmp, OUT)
        lib = ctypes.CDLL(OUT)
        P = ctypes.POINTER
        lib.hc_run.argtypes = [ctypes.c_char_p, ctypes.c_size_t, P(ctypes.c_double), ctypes.c_size_t,
                               P(ctypes.c_uint64), P(ctypes.c_uint32), ctypes.c_uint64, P(ctypes.c_uint32),
                               P(ctypes.c_uint32), P(ctypes.c_uint64), ctypes.c_uint64]
        lib.hc_run.restype = ctypes.c_int
        lib.hc_error.restype = ctypes.c_char_p
        lib.hc_lower_digest.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.c_int, P(ctypes.c_uint64)]
        lib.hc_lower_digest.restype = ctypes.c_int
        _lib = lib
    return _lib


def run(text, rates=None, max_faults=4_000_000, bits_per_fault=16):
    """-> (stats dict, {(channel, pauli code): signature tuple}) or raises."""
    lib = _load()
    raw = text.encode()
    off = np.zeros(max_faults + 1, dtype=np.uint64)
    bits = np.zeros(max_faults * bits_per_fault, dtype=np.uint32)
    src = np.zeros(max_faults, dtype=np.uint32)
    code = np.zeros(max_faults, dtype=np.uint32)
    stats = np.zeros(9, dtype=np.uint64)
    P = ctypes.POINTER
    if rates is not None:
        r = np.ascontiguousarray(rates, dtype=np.float64)
        rp, nr = r.ctypes.data_as(P(ctypes.c_double)), len(r)
    else:
        rp, nr = None, 0
    rc = lib.hc_run(raw, len(raw), rp, nr, off.ctypes.data_as(P(ctypes.c_uint64)),
                    bits.ctypes.data_as(P(ctypes.c_uint32)), len(bits), src.ctypes.data_as(P(ctypes.c_uint32)),
                    code.ctypes.data_as(P(ctypes.c_uint32)), stats.ctypes.data_as(P(ctypes.c_uint64)), max_faults)
    if rc != 0:
        raise RuntimeError(f"host check failed ({rc}): {lib.hc_error().decode()}")
    names = ["faults", "items", "slab_words", "layers", "gauge", "written", "words", "qubits", "max_col_inj"]
    st = {k: int(v) for k, v in zip(names, stats)}
    F = st["faults"]
    sigs = {}
    for p in range(F):
        sigs[(int(src[p]), int(code[p]))] = tuple(int(x) for x in bits[off[p]:off[p + 1]])
    return st, sigs


def run_batch(texts, slots=None, max_faults=4_000_000, bits_per_fault=16):
    """Replay a merged batch -> (stats, [per circuit {(channel, pauli code): signature}]).
    Channels are numbered per circuit (program order), as in `run`."""
    lib = _load()
    P = ctypes.POINTER
    lib.hc_run_batch.argtypes = [P(ctypes.c_char_p), P(ctypes.c_size_t), ctypes.c_size_t, ctypes.c_uint32,
                                 P(ctypes.c_uint64), P(ctypes.c_uint32), ctypes.c_uint64, P(ctypes.c_uint32),
                                 P(ctypes.c_uint32), P(ctypes.c_uint64), ctypes.c_uint64, P(ctypes.c_uint32)]
    lib.hc_run_batch.restype = ctypes.c_int
    n = len(texts)
    if slots is None:
        slots = max(1, -(-256 // n))
    raw = [t.encode() for t in texts]
    arr = (ctypes.c_char_p * n)(*raw)
    lens = (ctypes.c_size_t * n)(*[len(r) for r in raw])
    off = np.zeros(max_faults + 1, dtype=np.uint64)
    bits = np.zeros(max_faults * bits_per_fault, dtype=np.uint32)
    src = np.zeros(max_faults, dtype=np.uint32)
    code = np.zeros(max_faults, dtype=np.uint32)
    circ = np.zeros(max_faults, dtype=np.uint32)
    stats = np.zeros(9, dtype=np.uint64)
    rc = lib.hc_run_batch(arr, lens, n, slots, off.ctypes.data_as(P(ctypes.c_uint64)),
                          bits.ctypes.data_as(P(ctypes.c_uint32)), len(bits), src.ctypes.data_as(P(ctypes.c_uint32)),
                          code.ctypes.data_as(P(ctypes.c_uint32)), stats.ctypes.data_as(P(ctypes.c_uint64)),
                          max_faults, circ.ctypes.data_as(P(ctypes.c_uint32)))
    if rc != 0:
        raise RuntimeError(f"host check failed ({rc}): {lib.hc_error().decode()}")
    names = ["faults", "items", "slab_words", "layers", "gauge", "written", "words", "qubits", "max_col_inj"]
    st = {k: int(v) for k, v in zip(names, stats)}
    # channel numbers of the batch -> per circuit: subtract the channels of the circuits before
    counts = [0] * n
    for p in range(st["faults"]):
        k = int(circ[p])
        counts[k] = max(counts[k], int(src[p]) + 1)
    base = [0] * n
    for k in range(1, n):
        base[k] = max(base[k - 1], counts[k - 1])
    out = [dict() for _ in range(n)]
    for p in range(st["faults"]):
        k = int(circ[p])
        out[k][(int(src[p]) - base[k], int(code[p]))] = tuple(int(x) for x in bits[off[p]:off[p + 1]])
    return st, out


def set_fault_cost(c: float) -> None:
    lib = _load()
    lib.hc_set_fault_cost.argtypes = [ctypes.c_double]
    lib.hc_set_fault_cost.restype = None
    lib.hc_set_fault_cost(c)



def lower_digest(text, reuse):
    """Digest of every lowered table of `text`, lowered into tables kept
    across calls (reuse) or into fresh ones."""
    lib = _load()
    raw = text.encode()
    out = ctypes.c_uint64()
    rc = lib.hc_lower_digest(raw, len(raw), int(bool(reuse)), ctypes.byref(out))
    if rc:
        raise RuntimeError(f"lowering failed ({rc}): {lib.hc_error().decode()}")
    return out.value
