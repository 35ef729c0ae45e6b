"""The binary circuit form (gp_circuit_ir) on the CPU: the generators record
every circuit both as text and as per-operation arrays; lowering either gives
the same bounds (every table size), and malformed binary circuits are refused
with the documented status codes. (GPU results of both forms are compared
bit for bit in test_gpu_ir.py.)"""

import numpy as np
import pytest

from paper_2604_16613_amd import GpError
from paper_2604_16613_amd import _gp
from workloads import (bit_flip_code_fig1, bivariate_bicycle_memory, iceberg_surface_batch, mirror_circuit,
                       repetition_code_memory, rotated_surface_code_memory)


def circuits():
    yield "fig1", bit_flip_code_fig1()
    yield "rep7", repetition_code_memory(7, 5, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04)
    yield "sc3", rotated_surface_code_memory(3, 3)
    yield "sc11", rotated_surface_code_memory(11, 11)
    yield "bb144", bivariate_bicycle_memory()
    yield "iceberg5", iceberg_surface_batch(5, n_branches=1, seed=9)[0]
    for s in range(3):
        yield f"mirror{s}", mirror_circuit(5, 6, s, x_basis=[s % 5, (s + 1) % 5])


@pytest.mark.parametrize("name,c", list(circuits()))
def test_binary_and_text_lower_alike(name, c):
    a = _gp.gp_bounds_from_circuit(c.text).as_dict()
    b = _gp.gp_bounds_from_ir(c.ir).as_dict()
    assert a == b, name
    assert len(c.ir["code"]) == len(c.ir["q0"]) == len(c.ir["q1"]) == len(c.ir["rate"])


def test_binary_batch_bounds():
    cs = [cc for _, cc in circuits()]
    a = _gp.gp_bounds_from_batch([cc.text for cc in cs]).as_dict()
    b = _gp.gp_bounds_from_batch_ir([cc.ir for cc in cs]).as_dict()
    assert a == b


def _ir(ops, rec=()):
    """ops: (code, q0, q1, rate) tuples."""
    ops = list(ops)
    return {"code": np.array([o[0] for o in ops], dtype=np.uint8),
            "q0": np.array([o[1] for o in ops], dtype=np.uint32),
            "q1": np.array([o[2] for o in ops], dtype=np.uint32),
            "rate": np.array([o[3] for o in ops], dtype=np.float64),
            "rec": np.array(rec, dtype=np.uint32)}


R, M, CX, XE, D2, DET, OBS = 7, 9, 4, 16, 20, 32, 33


def test_small_binary_circuit_matches_text():
    text = "R 0 1\nX_ERROR(0.1) 0\nCX 0 1\nDEPOLARIZE2(0.01) 0 1\nM 0 1\nDETECTOR rec[-1]\nOBSERVABLE_INCLUDE(2) rec[-2] rec[-1]\n"
    ir = _ir([(R, 0, 0, 0), (R, 1, 0, 0), (XE, 0, 0, 0.1), (CX, 0, 1, 0), (D2, 0, 1, 0.01), (M, 0, 0, 0),
              (M, 1, 0, 0), (DET, 0, 1, 0), (OBS, 2, 2, 0)], rec=[1, 0, 1])
    assert _gp.gp_bounds_from_ir(ir).as_dict() == _gp.gp_bounds_from_circuit(text).as_dict()


@pytest.mark.parametrize("ops,rec,code", [
    ([(99, 0, 0, 0)], [], -3),                                    # unknown operation code
    ([(CX, 1, 1, 0)], [], -2),                                    # repeated qubit
    ([(XE, 0, 0, 0.7)], [], -6),                                  # rate out of range
    ([(D2, 0, 1, 0.99)], [], -6),
    ([(M, 0, 0, 0), (DET, 0, 1, 0)], [1], -2),                    # record of a future measurement
    ([(M, 0, 0, 0), (DET, 0, 2, 0)], [0], -1),                    # records past the array
    ([(M, 0, 0, 0), (DET, 0, 1, 0)], [0, 0], -1),                 # array longer than used
    ([(OBS, 70000, 0, 0)], [], -2),                               # observable index too large
    ([(R, 1 << 28, 0, 0)], [], -4),                               # qubit index too large
])
def test_malformed_binary_circuits(ops, rec, code):
    with pytest.raises(GpError) as e:
        _gp.gp_bounds_from_ir(_ir(ops, rec))
    assert e.value.code == code, e.value
    assert "operation" in str(e.value) or "record" in str(e.value)


def test_missing_arrays_are_refused():
    ir = _ir([(R, 0, 0, 0), (M, 0, 0, 0), (DET, 0, 1, 0)], rec=[0])
    s, keep = _gp.circuit_ir(ir)
    import ctypes
    s.q1 = ctypes.POINTER(ctypes.c_uint32)()
    b = _gp.GpBounds()
    rc = _gp.load().gp_bounds_from_ir(ctypes.byref(s), ctypes.byref(b))
    assert rc == -1 and "missing" in _gp.gp_last_error()
