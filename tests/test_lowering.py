"""The compiler's host lowering, replayed on the CPU by tests/host_check.cpp
(same tables, same work items, same slab addressing, every access bounds
checked), must give every fault the oracle's signature. No GPU needed."""

import numpy as np
import pytest

import host_check
import oracle
from workloads import (bit_flip_code_fig1, bivariate_bicycle_memory, log_uniform_rates, mirror_circuit,
                       repetition_code_memory, rotated_surface_code_memory)


def compare(text, rates=None):
    st, sigs = host_check.run(text, rates)
    res = oracle.run(text, rates=rates, keep_faults=True)
    osig = {(ch, code): sig for ch, code, sig, _ in res.fault_signatures()}
    assert st["faults"] == res.n_faults == len(sigs)
    assert sigs == osig
    assert st["gauge"] == 0
    return st


def test_small_circuits():
    compare(bit_flip_code_fig1().text)
    compare(repetition_code_memory(5, 4, p_data=0.01, p_meas=0.01, p2=0.01, p1=0.01).text)
    for s in range(6):
        compare(mirror_circuit(5, 6, s, x_basis=[s % 5]).text)


@pytest.mark.parametrize("d,r", [(3, 3), (5, 5), (7, 4), (9, 9)])
def test_surface_code(d, r):
    st = compare(rotated_surface_code_memory(d, r).text)
    assert st["qubits"] == 2 * d * d - 1


def test_surface_code_rates():
    c = rotated_surface_code_memory(5, 3)
    compare(c.text, log_uniform_rates(c.n_channels, 3))


def test_bivariate_bicycle_short():
    compare(bivariate_bicycle_memory(rounds=3).text)


def test_bivariate_bicycle_paper_preset():
    """[[72,12,6]], [[108,8,10]] and [[144,12,12]] under the paper's noise preset (idle noise,
    resets that fail by a flip in their basis), both schedules."""
    from workloads import paper_noise
    for l, m, sched in ((6, 6, "depth8"), (9, 6, "depth8"), (12, 6, "depth8"), (6, 6, "sequential")):
        st = compare(bivariate_bicycle_memory(rounds=2, l=l, m=m, schedule=sched, **paper_noise(1e-3)).text)
        assert st["qubits"] == 4 * l * m


def test_gauge_flagged():
    st, _ = host_check.run("R 0\nH 0\nM 0\nDETECTOR rec[-1]\n")
    assert st["gauge"] == 1
    st, _ = host_check.run("H 0\nM 0\nDETECTOR rec[-1]\n")
    assert st["gauge"] == 1
    st, _ = host_check.run("R 0\nM 0\nDETECTOR rec[-1]\n")
    assert st["gauge"] == 0


def test_merged_batch_replays_like_each_circuit():
    """A batch of mixed circuits, merged and replayed through the circuit
    descriptors with every access checked, gives every circuit the signatures
    its own lowering gives (and so the oracle's)."""
    texts = [rotated_surface_code_memory(5, 5).text, bit_flip_code_fig1().text, "",
             repetition_code_memory(7, 5, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04).text,
             "R 0 1\nCX 0 1\nM 0 1\nDETECTOR rec[-1] rec[-2]\n", "R 0\nX_ERROR(0.1) 0\nM 0\n",
             mirror_circuit(5, 6, 1, x_basis=[1, 2]).text, bivariate_bicycle_memory(rounds=2).text,
             rotated_surface_code_memory(3, 3).text]
    st, per = host_check.run_batch(texts)
    assert st["gauge"] == 0
    total = 0
    for t, sigs in zip(texts, per):
        _, single = host_check.run(t)
        assert sigs == single
        total += len(single)
    assert st["faults"] == total
    # the same circuit many times, each with a share of one slot
    c = rotated_surface_code_memory(3, 3).text
    st, per = host_check.run_batch([c] * 300)
    _, single = host_check.run(c)
    assert all(s == single for s in per)


@pytest.mark.parametrize("cost", [2.5e-4, 1.4e-3, 0.02])
def test_observable_cut_does_not_change_signatures(cost):
    """The autotuner's knob (cost per fault when cutting observable columns
    into ranges) moves item boundaries only: every fault keeps its signature."""
    texts = [rotated_surface_code_memory(5, 5).text, bivariate_bicycle_memory(rounds=2).text]
    ref = [host_check.run(t)[1] for t in texts]
    host_check.set_fault_cost(cost)
    try:
        for t, r in zip(texts, ref):
            st, sigs = host_check.run(t)
            assert sigs == r
    finally:
        host_check.set_fault_cost(6.2e-4)


def test_text_split_across_tokenizer_threads():
    """A circuit text long enough to be tokenized in many chunks on several
    threads while the first chunks are scheduled (0.53 MB, d = 17) replays to
    the oracle's signatures."""
    c = rotated_surface_code_memory(17, 17)
    assert len(c.text) > 4 * (1 << 17)
    compare(c.text)


def test_text_in_chunks_on_the_scheduling_thread():
    """A text of several 32 KB chunks but below the 256 KB that start
    tokenizer threads (0.23 MB, d = 13) is tokenized chunk by chunk on the
    scheduling thread and replays to the oracle's signatures."""
    c = rotated_surface_code_memory(13, 13)
    assert 4 * (1 << 15) < len(c.text) < 2 * (1 << 17)
    compare(c.text)


def _error_line(text):
    from paper_2604_16613_amd import GpError, _gp
    with pytest.raises(GpError) as e:
        _gp.gp_bounds_from_circuit(text)
    return str(e.value)


def test_error_lines_keep_program_order_across_chunks():
    """Errors in a multi-chunk text name their own line, and the first error
    in program order wins, whether it is found while tokenizing (a chunk's
    syntax) or while scheduling (record look-back)."""
    lines = rotated_surface_code_memory(25, 25).text.split("\n")
    n = len(lines)
    late = int(n * 0.9)
    bad = lines[:late] + ["FOO 1"] + lines[late:]
    assert f"line {late + 1}: unsupported instruction FOO" in _error_line("\n".join(bad))
    early = int(n * 0.2)
    both = lines[:early] + ["DETECTOR rec[-99999999]"] + lines[early:late] + ["FOO 1"] + lines[late:]
    assert f"line {early + 1}: record looks back too far" in _error_line("\n".join(both))
    mid = int(n * 0.5)
    two = lines[:mid] + ["CX 0"] + lines[mid:late] + ["H rec[-1]"] + lines[late:]
    assert f"line {mid + 1}: odd number of targets" in _error_line("\n".join(two))


def test_tokenizer_chunks_ignore_layout():
    """The same circuit written with CRLF line endings, comments, blank lines
    and lower-case instruction names (a multi-chunk text) lowers to the same
    signatures as the plain text."""
    import random
    c = rotated_surface_code_memory(17, 17)
    rng = random.Random(9)
    out = []
    for ln in c.text.split("\n"):
        if rng.random() < 0.05:
            out.append("# a comment line")
        if rng.random() < 0.05:
            out.append("   ")
        if ln and rng.random() < 0.3:
            head, _, rest = ln.partition(" ")
            ln = head.lower() + (" " + rest if rest else "")
        if ln and rng.random() < 0.1:
            ln += "  # trailing comment"
        out.append(ln)
    messy = "\r\n".join(out)
    assert len(messy) > 4 * (1 << 17)
    st_a, sig_a = host_check.run(c.text)
    st_b, sig_b = host_check.run(messy)
    assert st_a == st_b and sig_a == sig_b


def test_tables_lowered_into_reused_storage_equal_fresh_ones():
    """A driver lowers circuit after circuit into the same tables, keeping
    their storage: each lowering must give exactly the tables a fresh lowering
    gives, whatever was lowered before (larger, smaller, other families, the
    multi-threaded path of a large circuit included)."""
    circuits = [rotated_surface_code_memory(23, 23).text,  # large: tokenizer, channel-table and injection threads
                bit_flip_code_fig1().text,
                bivariate_bicycle_memory(rounds=3).text,
                mirror_circuit(12, 6, seed=3).text,
                rotated_surface_code_memory(5, 5).text,
                rotated_surface_code_memory(23, 23).text]
    fresh = [host_check.lower_digest(t, reuse=False) for t in circuits]
    kept = [host_check.lower_digest(t, reuse=True) for t in circuits]
    assert kept == fresh
    assert fresh[0] == fresh[-1] and len(set(fresh[:-1])) == len(circuits) - 1
