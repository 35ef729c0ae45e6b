"""Pins of the CPU oracle against things other than itself (no GPU needed).

* brute-force tableau simulation of every single fault (signatures);
* exhaustive enumeration of every joint channel outcome on tiny circuits
  (probabilities: the per-fault split and Eq. 3 together);
* closed forms (2r/3 for DEPOLARIZE1 with X and Y in one class, m equal faults,
  the two-qubit depolarising classes, the repetition-code phenomenological
  edge set);
* invariants (q <= 1/2, conservation of sum log(1-2p), time translation,
  circuit distance 3 of the d = 3 surface code);
* the paper's Fig. 1 worked example (partial pin, fixture in tests/golden/).
"""

import itertools
import json
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import brute_sim as bs
import oracle
from workloads import (bit_flip_code_fig1, log_uniform_rates, mirror_circuit,
                       repetition_code_memory, rotated_surface_code_memory)
from workloads.circuits import (bb_check_matrices, bb_logical_z, _gf2_rank,
                                rotated_surface_code_checks, bivariate_bicycle_memory)

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------- helpers

def check_against_brute_force(text, engine="tableau"):
    runner = bs.Runner(text, engine=engine)
    res = oracle.run(text, keep_faults=True)
    assert res.n_faults == sum(len(bs.channel_paulis(k)) for _, k, _, _ in runner.chans)
    for ch, code, sig, _ in res.fault_signatures():
        assert runner.signature(ch, code) == sig, (ch, code)
    return res


def mask(sig):
    m = 0
    for b in sig:
        m |= 1 << b
    return m


def exact_distribution(text, rates=None):
    """Exact distribution of the detector/observable flip pattern: every joint
    outcome of every channel, each channel applying one specific Pauli with its
    own probability (r, r/3, r/15) or nothing, patterns combined by XOR of the
    brute-force single-fault signatures (Pauli insertion is linear)."""
    runner = bs.Runner(text)
    chans = runner.chans
    per_chan = []
    for c, (_, kind, _, rate) in enumerate(chans):
        r = rate if rates is None else rates[c]
        opts = [(0, 1.0 - r)]                  # no Pauli fires
        for code in bs.channel_paulis(kind):
            opts.append((mask(runner.signature(c, code)), bs.pauli_probability(kind, r)))
        per_chan.append(opts)
    dist = {0: 1.0}
    for opts in per_chan:
        new = {}
        for m, pr in dist.items():
            for s, ps in opts:
                new[m ^ s] = new.get(m ^ s, 0.0) + pr * ps
        dist = new
    return dist


def hyperedge_distribution(res):
    dist = {0: 1.0}
    for sig, q in res.edges().items():
        s = mask(sig)
        new = {}
        for m, pr in dist.items():
            new[m] = new.get(m, 0.0) + pr * (1.0 - q)
            new[m ^ s] = new.get(m ^ s, 0.0) + pr * q
        dist = new
    return dist


def assert_same_distribution(a, b):
    keys = set(a) | set(b)
    for k in keys:
        x, y = a.get(k, 0.0), b.get(k, 0.0)
        assert abs(x - y) <= 1e-13 + 1e-11 * max(abs(x), abs(y)), (k, x, y)


# ------------------------------------------------------- brute-force signatures

def test_tableau_matches_state_vector():
    for seed in range(6):
        c = mirror_circuit(4, 4, seed, x_basis=[seed % 4])
        for forced in (0, 1):
            a = bs.Runner(c.text, engine="tableau", forced=forced)
            b = bs.Runner(c.text, engine="statevector", forced=forced)
            assert a.record == b.record
    c = repetition_code_memory(3, 2)
    for forced in (0, 1):
        assert bs.Runner(c.text, forced=forced).record == bs.Runner(c.text, "statevector", forced=forced).record


def test_brute_force_fig1_and_repetition():
    check_against_brute_force(bit_flip_code_fig1().text)
    check_against_brute_force(repetition_code_memory(3, 2, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04).text)
    check_against_brute_force(repetition_code_memory(5, 3, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04,
                                                     data_noise="DEPOLARIZE1").text)


@pytest.mark.parametrize("seed", range(8))
def test_brute_force_mirror_circuits(seed):
    """All gate kinds (H, S, S_DAG, SQRT_X(_DAG), Paulis, CX, CZ, SWAP), X-basis
    preparation and measurement, MR, repeated records and split observables."""
    c = mirror_circuit(4, 5, seed, x_basis=[seed % 4, (seed + 2) % 4])
    check_against_brute_force(c.text)


def test_brute_force_x_basis_measure_reset():
    """MRX (X-basis measure and reset) as the depth-8 bivariate bicycle cycle
    uses it: two data qubits in |+>, their X parity read through an ancilla
    that is measured and reset in the X basis every round, flips before the
    X-basis measurements."""
    lines = ["RX 0 1 2", "DEPOLARIZE1(0.02) 0 1 2"]
    for r in range(3):
        lines += ["CX 2 0", "DEPOLARIZE2(0.03) 2 0", "CX 2 1", "DEPOLARIZE2(0.04) 2 1",
                  "Z_ERROR(0.05) 2", "MRX 2", "DEPOLARIZE1(0.01) 2"]
        lines.append("DETECTOR rec[-1]" if r == 0 else "DETECTOR rec[-1] rec[-2]")
    lines += ["Z_ERROR(0.06) 0 1", "MX 0 1", "DETECTOR rec[-1] rec[-2] rec[-3]", "OBSERVABLE_INCLUDE(0) rec[-2]"]
    text = "\n".join(lines) + "\n"
    res = check_against_brute_force(text)
    assert res.n_detectors == 4 and res.n_observables == 1


def test_brute_force_mirror_state_vector_engine():
    c = mirror_circuit(3, 3, 11, x_basis=[0])
    check_against_brute_force(c.text, engine="statevector")


def test_brute_force_surface_code_d3_all_faults():
    c = rotated_surface_code_memory(3, 3)
    res = check_against_brute_force(c.text)
    assert res.n_faults == 1308
    assert (res.n_qubits, res.n_detectors, res.n_observables, res.n_channels) == (17, 24, 1, 170)


def test_generators_deterministic():
    """Noiseless runs give every detector and observable the value 0 whatever
    the random measurement outcomes are."""
    circuits = [rotated_surface_code_memory(3, 3), rotated_surface_code_memory(5, 2),
                repetition_code_memory(5, 3), bit_flip_code_fig1(),
                bivariate_bicycle_memory(rounds=2, l=6, m=6),
                bivariate_bicycle_memory(rounds=2, l=6, m=6, schedule="sequential"),
                bivariate_bicycle_memory(rounds=2, l=12, m=6)]
    circuits += [mirror_circuit(4, 4, s, x_basis=[1]) for s in range(3)]
    for c in circuits:
        for kw in (dict(forced=0), dict(forced=1), dict(seed=5)):
            r = bs.Runner(c.text, **kw)
            assert not any(r.values), (c.name, kw)


def test_bb_depth8_schedule_condition():
    """The depth-8 slots meet every constraint they were searched under: one CX
    per ancilla and per data qubit in each slot, seven CX slots, and the
    pairwise order condition for X and Z checks sharing data; an assignment
    that breaks only the order condition gives random detectors."""
    import workloads.circuits as wc
    s = wc.BB_DEPTH8_SLOTS
    assert len(set(s["A"] + s["B"])) == 6 and len(set(s["BT"] + s["AT"])) == 6
    assert not set(s["A"]) & set(s["BT"]) and not set(s["B"]) & set(s["AT"])
    assert max(s["A"] + s["B"] + s["BT"] + s["AT"]) == 6
    assert all((s["A"][k] > s["BT"][m]) == (s["B"][m] > s["AT"][k]) for k in range(3) for m in range(3))
    c = bivariate_bicycle_memory(rounds=12)
    assert _gp_layers(c.text) == 86      # seven layers per round in steady state
    bad = dict(s, AT=(1, 5, 6))
    assert not all((bad["A"][k] > bad["BT"][m]) == (bad["B"][m] > bad["AT"][k]) for k in range(3) for m in range(3))
    old = wc.BB_DEPTH8_SLOTS
    try:
        wc.BB_DEPTH8_SLOTS = bad
        c = wc.bivariate_bicycle_memory(rounds=3, l=6, m=6)
    finally:
        wc.BB_DEPTH8_SLOTS = old
    assert any(bs.Runner(c.text, seed=5).values)


def _gp_layers(text):
    from paper_2604_16613_amd import _gp
    return _gp.gp_bounds_from_circuit(text).max_layers


def test_generator_codes():
    for d in (3, 5, 7):
        hx, hz = rotated_surface_code_checks(d)
        assert not ((hx.astype(int) @ hz.T.astype(int)) % 2).any()
        assert len(hx) == len(hz) == (d * d - 1) // 2
        row0 = np.zeros(d * d, dtype=int)
        row0[:d] = 1
        assert not ((hx.astype(int) @ row0) % 2).any()          # Z on row 0 is a logical
        assert _gf2_rank(np.vstack([hz, row0])) == _gf2_rank(hz) + 1
    hx, hz = bb_check_matrices()
    assert not ((hx.astype(int) @ hz.T.astype(int)) % 2).any()
    assert _gf2_rank(hx) == 66 and _gf2_rank(hz) == 66          # k = 144 - 132 = 12
    lz = bb_logical_z()
    assert lz.shape == (12, 144)
    assert not ((hx.astype(int) @ lz.T.astype(int)) % 2).any()
    assert _gf2_rank(np.vstack([hz, lz])) == 66 + 12


# --------------------------------------------------- exhaustive probabilities

def test_exhaustive_two_qubit_depolarising():
    c = repetition_code_memory(3, 1, p2=0.1)
    rates = [0.05, 0.1, 0.15, 0.2]
    assert c.n_channels == 4
    res = oracle.run(c.text, rates=rates)
    assert_same_distribution(exact_distribution(c.text, rates), hyperedge_distribution(res))


def test_exhaustive_single_qubit_and_flips():
    c = repetition_code_memory(3, 1, p_data=0.1, p_meas=0.07, data_noise="DEPOLARIZE1")
    rates = np.linspace(0.03, 0.3, c.n_channels)
    res = oracle.run(c.text, rates=rates)
    assert_same_distribution(exact_distribution(c.text, rates), hyperedge_distribution(res))


def test_exhaustive_bell_pair_mixed_channels():
    text = ("R 0 1\nH 0\nDEPOLARIZE1(0.2) 0\nCX 0 1\nDEPOLARIZE2(0.3) 0 1\n"
            "Y_ERROR(0.05) 1\nZ_ERROR(0.1) 0\nX_ERROR(0.11) 0 1\nM 0 1\n"
            "DETECTOR rec[-1] rec[-2]\n")
    res = oracle.run(text)
    assert_same_distribution(exact_distribution(text), hyperedge_distribution(res))


def test_exhaustive_detects_swapped_rates():
    """A rate array applied in the wrong channel order must change the answer."""
    c = repetition_code_memory(3, 1, p2=0.1)
    rates = [0.05, 0.1, 0.15, 0.2]
    res = oracle.run(c.text, rates=rates[::-1])
    a = exact_distribution(c.text, rates)
    b = hyperedge_distribution(res)
    assert max(abs(a.get(k, 0) - b.get(k, 0)) for k in set(a) | set(b)) > 1e-4


# ------------------------------------------------------------ closed forms

def test_split_formulas_high_precision():
    getcontext().prec = 60
    for r in (1e-6, 1e-4, 1e-3, 5e-3, 0.1, 0.5, 0.74):
        p = Decimal(oracle.fault_probability("DEPOLARIZE1", r))
        lhs = (1 - 2 * p) ** 2
        rhs = 1 - Decimal(4) * Decimal(r) / 3
        pe = (1 - rhs.sqrt()) / 2
        assert abs(p - pe) <= abs(pe) * Decimal("1e-15")
        assert abs(lhs - rhs) <= Decimal("1e-15")
    for r in (1e-6, 1e-4, 1e-3, 5e-3, 0.1, 0.5, 0.9):
        p = Decimal(oracle.fault_probability("DEPOLARIZE2", r))
        x = 1 - Decimal(16) * Decimal(r) / 15
        pe = (1 - x.sqrt().sqrt().sqrt()) / 2
        assert abs(p - pe) <= abs(pe) * Decimal("1e-15")
    for k in ("X_ERROR", "Y_ERROR", "Z_ERROR"):
        assert oracle.fault_probability(k, 0.0123) == 0.0123


@pytest.mark.parametrize("r", [1e-4, 1e-3, 0.05, 0.3])
def test_depolarize1_two_thirds(r):
    res = oracle.run(f"R 0\nDEPOLARIZE1({r!r}) 0\nM 0\nDETECTOR rec[-1]\n")
    e = res.edges()
    assert list(e) == [(0,)]
    assert e[(0,)] == pytest.approx(2 * r / 3, rel=2e-15, abs=0)
    assert res.n_empty == 1          # the Z fault


@pytest.mark.parametrize("m,p", [(2, 1e-3), (5, 1e-4), (7, 0.01), (3, 0.4)])
def test_equal_faults_merge(m, p):
    text = "R 0\n" + "X_ERROR(%r) 0\n" % p * m + "M 0\nDETECTOR rec[-1]\nOBSERVABLE_INCLUDE(0) rec[-1]\n"
    res = oracle.run(text)
    e = res.edges()
    assert list(e) == [(0, 1)]
    exact = (1 - (1 - 2 * Fraction(p)) ** m) / 2
    assert e[(0, 1)] == pytest.approx(float(exact), rel=1e-14)


@pytest.mark.parametrize("r", [1e-4, 1e-3, 0.2])
def test_depolarize2_classes(r):
    res = oracle.run(f"R 0 1\nDEPOLARIZE2({r!r}) 0 1\nM 0 1\nDETECTOR rec[-2]\nDETECTOR rec[-1]\n")
    e = res.edges()
    assert set(e) == {(0,), (1,), (0, 1)}
    getcontext().prec = 60
    exact = float((1 - (1 - Decimal(16) * Decimal(r) / 15).sqrt()) / 2)
    for k in e:
        assert e[k] == pytest.approx(exact, rel=1e-14)
    assert res.n_empty == 3


@pytest.mark.parametrize("d,rounds", [(3, 2), (5, 3), (6, 4)])
def test_repetition_phenomenological_edges(d, rounds):
    """Data flips before each round and measurement flips: every class holds one
    fault (q = p) and the edge set follows from the check structure."""
    p = 0.01
    c = repetition_code_memory(d, rounds, p_data=p, p_meas=p)
    res = oracle.run(c.text)
    nc = d - 1
    det = lambda k, j: k * nc + j          # round k, check j (final row k = rounds)
    obs = rounds * nc + nc                  # observable bit index = D
    expect = set()
    for k in range(rounds):
        for i in range(d):                  # data flip before round k
            s = {det(k, j) for j in (i - 1, i) if 0 <= j < nc}
            if i == 0:
                s.add(obs)
            expect.add(tuple(sorted(s)))
        for j in range(nc):                 # ancilla measurement flip in round k
            expect.add((det(k, j), det(k + 1, j)))
    for i in range(d):                      # final data measurement flip
        s = {det(rounds, j) for j in (i - 1, i) if 0 <= j < nc}
        if i == 0:
            s.add(obs)
        expect.add(tuple(sorted(s)))
    e = res.edges()
    assert set(e) == expect
    assert all(q == p for q in e.values())
    assert res.n_empty == 0


# -------------------------------------------------------------- invariants

@pytest.mark.parametrize("d,rounds,seed", [(3, 3, None), (5, 5, None), (5, 4, 1)])
def test_invariants_surface_code(d, rounds, seed):
    c = rotated_surface_code_memory(d, rounds)
    rates = None if seed is None else log_uniform_rates(c.n_channels, seed)
    res = oracle.run(c.text, rates=rates, keep_faults=True)
    assert res.n_detectors == c.n_detectors and res.n_observables == 1
    assert res.n_qubits == 2 * d * d - 1
    assert np.all(res.edge_q <= 0.5) and np.all(res.edge_q > 0)
    faults = res.fault_signatures()
    # Eq. 3 keeps 1 - 2q multiplicative: sum over classes of log(1 - 2q) equals
    # the sum over their faults of log(1 - 2p) (the dropped empty class aside)
    lhs = float(np.sum(np.log1p(-2 * res.edge_q)))
    rhs = sum(math.log1p(-2 * p) for _, _, s, p in faults if s)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    assert res.n_empty == sum(1 for f in faults if not f[2])
    # every analysed fault lands in exactly one class
    sigs = {f[2] for f in faults if f[2]}
    assert sigs == set(res.edges())


def test_time_translation():
    counts = [oracle.run(rotated_surface_code_memory(3, r).text).n_edges for r in (3, 4, 5, 6)]
    diffs = np.diff(counts)
    assert len(set(diffs.tolist())) == 1, counts


def test_circuit_distance_three():
    """d = 3 surface code: no one or two hyperedges flip only the observable,
    some three do (the N-Z CX order keeps the circuit distance at 3)."""
    res = oracle.run(rotated_surface_code_memory(3, 3).text)
    D = res.n_detectors
    target = 1 << D
    masks = [mask(s) for s in res.edges()]
    mset = set(masks)
    assert target not in mset
    for a, b in itertools.combinations(masks, 2):
        assert a ^ b != target
    found = any((a ^ b ^ target) in mset for a, b in itertools.combinations(masks, 2))
    assert found


def test_fig1_worked_example():
    with open(os.path.join(HERE, "golden", "fig1_bitflip.json")) as fh:
        g = json.load(fh)
    res = oracle.run(bit_flip_code_fig1().text, keep_faults=True)
    (ch, code, sig, _), = res.fault_signatures()
    assert ch == g["fault"]["channel"] and code == 1
    assert list(sig) == g["expected_signature"]


# ------------------------------------------------------------- error paths

def test_oracle_errors():
    with pytest.raises(oracle.OracleError) as e:
        oracle.run("REPEAT 3 {\nH 0\n}\n")
    assert e.value.code == -3
    with pytest.raises(oracle.OracleError) as e:
        oracle.run("R 0\nX_ERROR(0.7) 0\nM 0\n")
    assert e.value.code == -6
    with pytest.raises(oracle.OracleError) as e:
        oracle.run("R 0\nX_ERROR(0.1) 0\nM 0\n", rates=[0.1, 0.2])
    assert e.value.code == -6
    with pytest.raises(oracle.OracleError) as e:
        oracle.run("R 0\nT 0\nM 0\n")
    assert e.value.code == -3
    with pytest.raises(oracle.OracleError):
        oracle.run("M 0\nDETECTOR rec[-2]\n")


@pytest.mark.parametrize("threads", [2, 3, 8])
def test_threaded_tracking_is_identical(threads):
    """The forward tracking split over contiguous fault ranges on several
    threads, concatenated in fault order before the grouping, gives the
    single-thread result bit for bit (every fault's signature, every
    hyperedge and probability), also on a sampled fault subset."""
    c = rotated_surface_code_memory(7, 7)
    rates = log_uniform_rates(c.n_channels, 3)
    for stride in (1, 7):
        a = oracle.run(c.text, rates=rates, keep_faults=True, fault_stride=stride)
        b = oracle.run(c.text, rates=rates, keep_faults=True, fault_stride=stride, threads=threads)
        for f in ("edge_off", "edge_bits", "fault_off", "fault_bits", "fault_channel", "fault_code"):
            assert np.array_equal(getattr(a, f), getattr(b, f)), f
        for f in ("edge_q", "fault_p"):
            assert np.array_equal(getattr(a, f).view(np.uint64), getattr(b, f).view(np.uint64)), f
