"""Correlation levels (Table 1) and the paper's noise preset, on the oracle
(CPU only): the fault counts that give Table 1's factors, the classes each
level forms on one two-qubit channel (closed forms), one-qubit channels, and
the preset's rates."""

import math
import re

import pytest

import oracle
from workloads import paper_noise, rotated_surface_code_memory


def _split_dep2(r):
    # (1 - 2p)^8 = 1 - 16 r / 15
    return 0.5 * (1 - (1 - 16 * r / 15) ** 0.125)


def _merged(p, n):
    return 0.5 * (1 - (1 - 2 * p) ** n)


@pytest.mark.parametrize("level,n,alpha", [(0, 6, 3), (1, 10, 5), (2, 15, 8)])
def test_table1_fault_counts(level, n, alpha):
    res = oracle.run("DEPOLARIZE2(0.01) 0 1\nM 0 1\nDETECTOR rec[-2]\nDETECTOR rec[-1]\n", level=level)
    assert res.n_faults == n
    assert math.ceil(n / 2) == alpha  # Table 1's factor: half the included set, rounded up


@pytest.mark.parametrize("level,counts", [(0, (1, 1, 1)), (1, (3, 3, 1)), (2, (4, 4, 4))])
def test_two_qubit_classes_per_level(level, counts):
    # detector 0 sees X/Y on qubit 0, detector 1 sees X/Y on qubit 1:
    # L0 {IX, IZ, XI, XX, ZI, ZZ} -> {0}: XI, {1}: IX, {0,1}: XX
    # L1 adds IY -> {1}, XZ -> {0}, YI -> {0}, ZX -> {1}
    # L2 adds XY, YX, YY -> {0,1}, YZ -> {0}, ZY -> {1}
    r = 0.02
    res = oracle.run(f"DEPOLARIZE2({r!r}) 0 1\nM 0 1\nDETECTOR rec[-2]\nDETECTOR rec[-1]\n", level=level)
    e = res.edges()
    p = _split_dep2(r)
    assert set(e) == {(0,), (1,), (0, 1)}
    for sig, n in zip([(0,), (1,), (0, 1)], counts):
        assert math.isclose(e[sig], _merged(p, n), rel_tol=1e-13)


def test_one_qubit_channels_per_level():
    # DEPOLARIZE1: X, Z at level 0 (only X flips the Z measurement: q = p);
    # Y joins at level 1 (q = 2r/3)
    r = 0.03
    text = f"DEPOLARIZE1({r!r}) 0\nM 0\nDETECTOR rec[-1]\n"
    p = 0.5 * (1 - math.sqrt(1 - 4 * r / 3))
    assert math.isclose(oracle.run(text, level=0).edges()[(0,)], p, rel_tol=1e-13)
    assert math.isclose(oracle.run(text, level=1).edges()[(0,)], 2 * r / 3, rel_tol=1e-13)
    ytext = "Y_ERROR(0.1) 0\nM 0\nDETECTOR rec[-1]\n"
    assert oracle.run(ytext, level=0).n_faults == 0
    assert oracle.run(ytext, level=1).edges() == {(0,): 0.1}


def test_levels_nest():
    c = rotated_surface_code_memory(3, 3)
    n = [oracle.run(c.text, level=l).n_faults for l in (0, 1, 2)]
    assert n[0] < n[1] < n[2] == 1308


def test_paper_preset_rates():
    p = 2e-3
    c = rotated_surface_code_memory(3, 3, p=p, x_detectors=False, **paper_noise(p))
    rates = {}
    for kind, rate in re.findall(r"^(DEPOLARIZE1|DEPOLARIZE2|X_ERROR)\(([^)]*)\)", c.text, flags=re.M):
        rates.setdefault(kind, set()).add(float(rate))
    assert rates["DEPOLARIZE1"] == {p / 10}   # one-qubit gates and idle qubits
    assert rates["DEPOLARIZE2"] == {p}        # two-qubit gates
    assert rates["X_ERROR"] == {p}            # measurement flips and failed resets
    # idle noise lands on the qubits a gate layer leaves alone: with it the
    # circuit has more channels than without
    assert c.n_channels > rotated_surface_code_memory(3, 3, p=p).n_channels
    # no X-check detectors: 4 Z checks x 3 rounds + 4 final
    assert oracle.run(c.text).n_detectors == 16
