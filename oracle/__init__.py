"""CPU oracle for decoding hypergraphs -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The compiler package never imports it and
shares no code with it (see ``gp_oracle.c`` for what it computes and which
passages of the paper it follows).

``build()`` compiles ``gp_oracle.c`` with gcc into ``liboracle.so`` next to it.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

#: channel kind codes understood by ``fault_probability``
KIND = {"X_ERROR": 1, "Y_ERROR": 2, "Z_ERROR": 3, "DEPOLARIZE1": 4, "DEPOLARIZE2": 5}


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
           "-o", _LIB, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return _LIB


class _Result(ctypes.Structure):
    _fields_ = [
        ("n_qubits", ctypes.c_int64),
        ("n_measurements", ctypes.c_int64),
        ("n_detectors", ctypes.c_int64),
        ("n_observables", ctypes.c_int64),
        ("n_channels", ctypes.c_int64),
        ("n_faults", ctypes.c_int64),
        ("n_empty", ctypes.c_int64),
        ("n_edges", ctypes.c_int64),
        ("edge_off", ctypes.POINTER(ctypes.c_int64)),
        ("edge_bits", ctypes.POINTER(ctypes.c_int32)),
        ("edge_q", ctypes.POINTER(ctypes.c_double)),
        ("n_edge_bits", ctypes.c_int64),
        ("fault_off", ctypes.POINTER(ctypes.c_int64)),
        ("fault_bits", ctypes.POINTER(ctypes.c_int32)),
        ("fault_p", ctypes.POINTER(ctypes.c_double)),
        ("fault_channel", ctypes.POINTER(ctypes.c_int32)),
        ("fault_code", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_run.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_int64, ctypes.c_int, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.POINTER(_Result))]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_run_threads.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double),
                                           ctypes.c_int64, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                           ctypes.POINTER(ctypes.POINTER(_Result))]
        lib.oracle_run_threads.restype = ctypes.c_int
        lib.oracle_free.argtypes = [ctypes.POINTER(_Result)]
        lib.oracle_free.restype = None
        lib.oracle_last_error.restype = ctypes.c_char_p
        lib.oracle_fault_probability.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.oracle_fault_probability.restype = ctypes.c_double
        lib.oracle_gradient.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double),
                                        ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_int64]
        lib.oracle_gradient.restype = ctypes.c_int
        lib.oracle_set_level.argtypes = [ctypes.c_int]
        lib.oracle_set_level.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


@dataclasses.dataclass
class OracleResult:
    n_qubits: int
    n_measurements: int
    n_detectors: int
    n_observables: int
    n_channels: int
    n_faults: int
    n_empty: int
    edge_off: np.ndarray
    edge_bits: np.ndarray
    edge_q: np.ndarray
    fault_off: Optional[np.ndarray] = None
    fault_bits: Optional[np.ndarray] = None
    fault_p: Optional[np.ndarray] = None
    fault_channel: Optional[np.ndarray] = None
    fault_code: Optional[np.ndarray] = None

    @property
    def n_edges(self) -> int:
        return len(self.edge_q)

    def edges(self) -> Dict[Tuple[int, ...], float]:
        """{sorted signature bits: q}; bit b < D is detector b, else observable b - D."""
        out = {}
        for e in range(self.n_edges):
            sig = tuple(int(x) for x in self.edge_bits[self.edge_off[e]:self.edge_off[e + 1]])
            out[sig] = float(self.edge_q[e])
        return out

    def fault_signatures(self) -> List[Tuple[int, int, Tuple[int, ...], float]]:
        """[(channel, pauli code, signature, p)] per analysed fault, in fault order.
        Pauli code bits: x on first qubit, z on first, x on second, z on second."""
        assert self.fault_off is not None, "run with keep_faults=True"
        out = []
        for f in range(self.n_faults):
            sig = tuple(int(x) for x in self.fault_bits[self.fault_off[f]:self.fault_off[f + 1]])
            out.append((int(self.fault_channel[f]), int(self.fault_code[f]), sig, float(self.fault_p[f])))
        return out


def _arr(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def _level(lib, level: int) -> None:
    if lib.oracle_set_level(int(level)) != 0:
        raise OracleError(-1, lib.oracle_last_error().decode())


def run(text: str, rates: Optional[Sequence[float]] = None, keep_faults: bool = False,
        fault_stride: int = 1, level: int = 2, threads: int = 1) -> OracleResult:
    """Compile `text` with the oracle. `rates`: optional per-channel rate array;
    `level`: correlation level (Table 1), 2 = every Pauli; `threads`: host
    threads for the forward tracking (the result is the same for any count)."""
    lib = _load()
    _level(lib, level)
    raw = text.encode()
    out = ctypes.POINTER(_Result)()
    if rates is not None:
        r = np.ascontiguousarray(rates, dtype=np.float64)
        rp = r.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        nr = len(r)
    else:
        rp, nr = None, 0
    rc = lib.oracle_run_threads(raw, len(raw), rp, nr, int(keep_faults), int(fault_stride), int(threads),
                                ctypes.byref(out))
    if rc != 0:
        raise OracleError(rc, lib.oracle_last_error().decode())
    try:
        s = out.contents
        ne = s.n_edges
        res = OracleResult(
            n_qubits=s.n_qubits, n_measurements=s.n_measurements, n_detectors=s.n_detectors,
            n_observables=s.n_observables, n_channels=s.n_channels, n_faults=s.n_faults,
            n_empty=s.n_empty,
            edge_off=_arr(s.edge_off, ne + 1, np.int64),
            edge_bits=_arr(s.edge_bits, s.n_edge_bits, np.int32),
            edge_q=_arr(s.edge_q, ne, np.float64),
        )
        if keep_faults:
            nf = s.n_faults
            res.fault_off = _arr(s.fault_off, nf + 1, np.int64)
            res.fault_bits = _arr(s.fault_bits, int(res.fault_off[-1]) if nf else 0, np.int32)
            res.fault_p = _arr(s.fault_p, nf, np.float64)
            res.fault_channel = _arr(s.fault_channel, nf, np.int32)
            res.fault_code = _arr(s.fault_code, nf, np.int32)
    finally:
        lib.oracle_free(out)
    return res


def gradient(text: str, dl_dq: Sequence[float], rates: Optional[Sequence[float]] = None,
             level: int = 2) -> np.ndarray:
    """dL/d(rate) per channel (program order) given dL/dq per hyperedge in the
    order `run` returns the hyperedges (explicit products over each class's
    other members, chain rule through the per-fault split)."""
    lib = _load()
    raw = text.encode()
    g = np.ascontiguousarray(dl_dq, dtype=np.float64)
    if rates is not None:
        r = np.ascontiguousarray(rates, dtype=np.float64)
        rp, nr = r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(r)
        nch = nr
    else:
        rp, nr = None, 0
        nch = run(text).n_channels
    _level(lib, level)
    out = np.zeros(nch, dtype=np.float64)
    rc = lib.oracle_gradient(raw, len(raw), rp, nr, g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(g),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nch)
    if rc != 0:
        raise OracleError(rc, lib.oracle_last_error().decode())
    return out


def loss_and_dl_dq(q: np.ndarray, w: np.ndarray):
    """The differentiation workload's loss L = sum_k w_k log(q_k / (1 - q_k))
    and its derivative w_k / (q_k (1 - q_k))."""
    q = np.asarray(q, dtype=np.float64)
    return float(np.sum(w * np.log(q / (1.0 - q)))), w / (q * (1.0 - q))


def fault_probability(kind: str, rate: float) -> float:
    """Per-fault probability the oracle assigns to one Pauli of a channel."""
    return float(_load().oracle_fault_probability(KIND[kind], float(rate)))
