"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Signatures must match exactly (same set of hyperedges, same bits) and
probabilities to 1e-12 relative, on every workload: the d = 3 surface code,
d = 11 / 17 / 25 with uniform and seeded log-uniform rates, the [[144,12,12]]
bivariate bicycle code, d = 9 with per-channel rates, plus small circuits that
exercise every gate kind, the empty and degenerate cases, and error paths.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from paper_2604_16613_amd import Driver, GpError, get_driver
from paper_2604_16613_amd import _gp
from workloads import (bit_flip_code_fig1, bivariate_bicycle_memory, log_uniform_rates, mirror_circuit,
                       repetition_code_memory, rotated_surface_code_memory)

pytestmark = pytest.mark.gpu

REL_TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def assert_parity(hg, ref, label=""):
    g = hg.edges()
    assert len(g) == len(hg), "duplicate hyperedges in the GPU output"
    o = ref.edges()
    missing = set(o) - set(g)
    extra = set(g) - set(o)
    assert not missing and not extra, f"{label}: {len(missing)} missing, {len(extra)} extra hyperedges"
    worst = 0.0
    for k, qo in o.items():
        qg = g[k]
        rel = abs(qg - qo) / qo if qo > 0 else abs(qg)
        worst = max(worst, rel)
    assert worst <= REL_TOL, f"{label}: worst relative error {worst:.3e}"
    for e in range(len(hg)):
        seg = hg.bits[hg.offsets[e]:hg.offsets[e + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)
    return worst


def merged_bounds(texts):
    """Element-wise maximum of the bounds of several circuits; the derived
    sizes (signature slab, sweep items) are left for the driver to compute."""
    out = _gp.GpBounds()
    for t in texts:
        b = _gp.gp_bounds_from_circuit(t)
        for k, _ in b._fields_:
            setattr(out, k, max(getattr(out, k), getattr(b, k)))
    out.max_observables = max(out.max_observables, 16)
    out.max_slab_words = 0
    out.max_items = 0
    return out


@pytest.fixture(scope="module")
def drv25():
    say("creating a driver for d=25 r=25 and the [[144,12,12]] code")
    d = Driver(merged_bounds([rotated_surface_code_memory(25, 25).text, bivariate_bicycle_memory().text]))
    yield d
    d.close()


def check(drv, text, rates=None, label="", level=2):
    say("case", label)
    hg = drv.compile_hypergraph(text, rates)
    ref = oracle.run(text, rates=rates, level=level)
    return assert_parity(hg, ref, label)


def test_small_circuits(drv25):
    check(drv25, bit_flip_code_fig1().text, label="fig1")
    check(drv25, repetition_code_memory(3, 2, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04).text, label="rep3")
    check(drv25, repetition_code_memory(7, 5, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04,
                                        data_noise="DEPOLARIZE1").text, label="rep7")
    for s in range(6):
        check(drv25, mirror_circuit(5, 6, s, x_basis=[s % 5, (s + 1) % 5]).text, label=f"mirror{s}")


def test_surface_code_d3(drv25):
    """The d = 3, 3-round surface code with uniform p = 1e-3."""
    c = rotated_surface_code_memory(3, 3)
    check(drv25, c.text, label="sc3")
    info = drv25.info()
    assert info["n_faults"] == 1308 and info["n_channels"] == 170


@pytest.mark.parametrize("d,r", [(5, 5), (7, 7), (5, 2)])
def test_surface_code_small(drv25, d, r):
    check(drv25, rotated_surface_code_memory(d, r).text, label=f"sc{d}r{r}")


def test_surface_code_d9_rates(drv25):
    """d = 9, 9 rounds, per-channel log-uniform rates (seed 0)."""
    c = rotated_surface_code_memory(9, 9)
    check(drv25, c.text, log_uniform_rates(c.n_channels, 0), label="sc9 seed0")


@pytest.mark.parametrize("seed", [None, 0, 1, 2])
def test_surface_code_d11(drv25, seed):
    c = rotated_surface_code_memory(11, 11)
    rates = None if seed is None else log_uniform_rates(c.n_channels, seed)
    check(drv25, c.text, rates, label=f"sc11 seed{seed}")


def test_bivariate_bicycle(drv25):
    c = bivariate_bicycle_memory()
    check(drv25, c.text, label="bb144")
    assert drv25.info()["n_observables"] == 12


@pytest.mark.parametrize("seed", [None, 0, 1, 2])
def test_surface_code_d17(drv25, seed):
    c = rotated_surface_code_memory(17, 17)
    rates = None if seed is None else log_uniform_rates(c.n_channels, seed)
    check(drv25, c.text, rates, label=f"sc17 seed{seed}")


@pytest.mark.parametrize("seed", [None, 0, 1, 2])
def test_surface_code_d25(drv25, seed):
    """The largest workload at full size, every hyperedge compared."""
    c = rotated_surface_code_memory(25, 25)
    rates = None if seed is None else log_uniform_rates(c.n_channels, seed)
    check(drv25, c.text, rates, label=f"sc25 seed{seed}")
    info = drv25.info()
    assert info["n_faults"] == 1013572
    # (fault, column) pairs the hash read, summed per compaction tile: the
    # value the earlier single-counter sum gave for this circuit and range cut
    assert info["n_live_words"] == 30459023


def test_deterministic_and_split_path(drv25):
    c = rotated_surface_code_memory(11, 11)
    a = drv25.compile_hypergraph(c.text)
    drv25.lower(c.text)
    for _ in range(3):
        drv25.run()
    b = drv25.fetch()
    assert np.array_equal(a.offsets, b.offsets)
    assert np.array_equal(a.bits, b.bits)
    assert np.array_equal(a.q.view(np.uint64), b.q.view(np.uint64))


def test_driver_reuse_and_bounds():
    say("case reuse")
    with get_driver(rotated_surface_code_memory(5, 5).text) as drv:
        for d, r in ((3, 3), (5, 5), (3, 1), (5, 2)):
            c = rotated_surface_code_memory(d, r)
            assert_parity(drv.compile_hypergraph(c.text), oracle.run(c.text), f"reuse d{d}r{r}")
        with pytest.raises(GpError) as e:
            drv.compile_hypergraph(rotated_surface_code_memory(7, 7).text)
        assert e.value.code == -4
        # the driver still works after a refused circuit
        c = rotated_surface_code_memory(3, 3)
        assert_parity(drv.compile_hypergraph(c.text), oracle.run(c.text), "after refusal")


def test_degenerate_circuits(drv25):
    say("case degenerate")
    # no noise at all
    hg = drv25.compile_hypergraph("R 0 1\nCX 0 1\nM 0 1\nDETECTOR rec[-1] rec[-2]\n")
    assert len(hg) == 0
    # only undetectable faults
    hg = drv25.compile_hypergraph("R 0\nZ_ERROR(0.1) 0\nM 0\nDETECTOR rec[-1]\n")
    assert len(hg) == 0
    # no detectors or observables at all: every fault is empty
    hg = drv25.compile_hypergraph("R 0\nX_ERROR(0.1) 0\nM 0\n")
    assert len(hg) == 0
    # empty circuit
    hg = drv25.compile_hypergraph("")
    assert len(hg) == 0
    # a single fault; observable only
    hg = drv25.compile_hypergraph("R 0\nX_ERROR(0.25) 0\nM 0\nOBSERVABLE_INCLUDE(3) rec[-1]\n")
    assert hg.edges() == {(3,): 0.25}
    # DEPOLARIZE1 merges X and Y: q = 2r/3
    hg = drv25.compile_hypergraph("R 0\nDEPOLARIZE1(0.003) 0\nM 0\nDETECTOR rec[-1]\n")
    assert math.isclose(hg.edges()[(0,)], 0.002, rel_tol=1e-14)
    # rate 0 keeps the structure with q = 0
    text = "R 0 1\nX_ERROR(0) 0\nCX 0 1\nM 0 1\nDETECTOR rec[-1]\nDETECTOR rec[-2]\n"
    assert_parity(drv25.compile_hypergraph(text), oracle.run(text), "zero rate")


def test_error_paths(drv25):
    say("case errors")
    with pytest.raises(GpError) as e:
        drv25.compile_hypergraph("R 0\nH 0\nM 0\nDETECTOR rec[-1]\n")
    assert e.value.code == -5
    with pytest.raises(GpError) as e:
        drv25.compile_hypergraph("H 0\nM 0\nOBSERVABLE_INCLUDE(0) rec[-1]\n")
    assert e.value.code == -5
    c = rotated_surface_code_memory(3, 3)
    with pytest.raises(GpError) as e:
        drv25.compile_hypergraph(c.text, [1e-3] * (c.n_channels - 1))
    assert e.value.code == -6
    with pytest.raises(GpError) as e:
        drv25.compile_hypergraph(c.text, [0.9] * c.n_channels)
    assert e.value.code == -6
    # still healthy afterwards
    check(drv25, c.text, label="after errors")


def test_dem_text_round_trip(drv25):
    say("case dem")
    c = rotated_surface_code_memory(3, 3)
    dem = drv25.compile_detector_error_model(c.text)
    ref = oracle.run(c.text).edges()
    got = {}
    D = 24
    for line in dem.strip().splitlines():
        head, *targets = line.split()
        q = float(head[len("error("):-1])
        bits = tuple(int(t[1:]) if t[0] == "D" else D + int(t[1:]) for t in targets)
        got[bits] = q
    assert set(got) == set(ref)
    for k in ref:
        assert math.isclose(got[k], ref[k], rel_tol=1e-12)


@pytest.mark.parametrize("bits", [8, 1])
def test_forced_key_collisions(drv25, bits):
    """Class keys cut to a few bits collide massively; the device detects it
    through the check hash and the compile re-runs keyed on both hashes, so the
    hypergraph is unchanged."""
    c = rotated_surface_code_memory(7, 7)
    _gp.gp_debug_set_key_bits(drv25.handle, bits)
    try:
        before = _gp.gp_debug_collision_retries(drv25.handle)
        check(drv25, c.text, label=f"key bits {bits}")
        assert _gp.gp_debug_collision_retries(drv25.handle) == before + 1
    finally:
        _gp.gp_debug_set_key_bits(drv25.handle, 64)
    before = _gp.gp_debug_collision_retries(drv25.handle)
    check(drv25, c.text, label="full keys again")
    assert _gp.gp_debug_collision_retries(drv25.handle) == before


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_grouping_paths(drv25, mode):
    """Every stage-2 grouping (256 buckets sorted and merged in LDS, the full
    LSD radix sort, 65,536 buckets on the top two key digits) against the
    oracle on the same workloads."""
    _gp.gp_debug_set_sort_mode(drv25.handle, mode)
    try:
        c = rotated_surface_code_memory(11, 11)
        check(drv25, c.text, log_uniform_rates(c.n_channels, 2), label=f"sort mode {mode} sc11")
        check(drv25, bivariate_bicycle_memory().text, label=f"sort mode {mode} bb")
        c = rotated_surface_code_memory(25, 25)
        check(drv25, c.text, log_uniform_rates(c.n_channels, 0), label=f"sort mode {mode} sc25")
    finally:
        _gp.gp_debug_set_sort_mode(drv25.handle, 0)


@pytest.mark.parametrize("copies", [3000, 9000])
def test_large_classes(drv25, copies):
    """Thousands of faults with one signature: a class merged by a whole
    block (3000 members), and one larger than a bucket's LDS capacity (9000),
    which makes the compile redo the grouping with the full sort."""
    rates = np.linspace(1e-7, 2e-5, copies)
    lines = [f"X_ERROR({r:.17g}) 0" for r in rates]
    lines += ["X_ERROR(0.01) 1", "M 0 1", "DETECTOR rec[-2]", "DETECTOR rec[-1]", "OBSERVABLE_INCLUDE(0) rec[-1]"]
    check(drv25, "\n".join(lines) + "\n", label=f"{copies} copies")



@pytest.mark.parametrize("copies", [1500, 3000])
def test_large_classes_in_small_buckets(drv25, copies):
    """The 65,536-bucket grouping: a class merged by the whole 256-thread
    block (1500 members), and one over its 2048-fault capacity (3000), which
    makes the compile redo the grouping with the full sort."""
    rates = np.linspace(1e-7, 2e-5, copies)
    lines = [f"X_ERROR({r:.17g}) 0" for r in rates]
    lines += ["X_ERROR(0.01) 1", "M 0 1", "DETECTOR rec[-2]", "DETECTOR rec[-1]", "OBSERVABLE_INCLUDE(0) rec[-1]"]
    _gp.gp_debug_set_sort_mode(drv25.handle, 2)
    try:
        check(drv25, "\n".join(lines) + "\n", label=f"{copies} copies, 16-bit buckets")
    finally:
        _gp.gp_debug_set_sort_mode(drv25.handle, 0)


@pytest.mark.parametrize("level", [0, 1])
def test_correlation_levels(drv25, level):
    """Table 1 levels: the device keeps the same Paulis as the oracle."""
    from workloads import paper_noise
    drv25.set_correlation_level(level)
    try:
        c = rotated_surface_code_memory(11, 11)
        hg = drv25.compile_hypergraph(c.text, log_uniform_rates(c.n_channels, 0))
        assert_parity(hg, oracle.run(c.text, rates=log_uniform_rates(c.n_channels, 0), level=level),
                      f"level {level} sc11")
        c = bivariate_bicycle_memory()
        assert_parity(drv25.compile_hypergraph(c.text), oracle.run(c.text, level=level), f"level {level} bb")
        c = rotated_surface_code_memory(7, 7, p=1e-3, x_detectors=False, **paper_noise(1e-3))
        assert_parity(drv25.compile_hypergraph(c.text), oracle.run(c.text, level=level), f"level {level} preset")
        c = rotated_surface_code_memory(25, 25)
        assert_parity(drv25.compile_hypergraph(c.text), oracle.run(c.text, level=level), f"level {level} sc25")
    finally:
        drv25.set_correlation_level(2)
    with pytest.raises(GpError) as e:
        drv25.set_correlation_level(3)
    assert e.value.code == -1


@pytest.mark.parametrize("level", [0, 1, 2])
def test_paper_table2_workloads(drv25, level):
    """The paper's memory benchmark (Table 2): rotated surface codes d = 3, 5, 7, 9
    and the bivariate bicycle codes [[72,12,6]], [[108,8,10]] and [[144,12,12]],
    d rounds each, under its noise preset, at each correlation level."""
    from workloads import paper_noise
    noise = paper_noise(1e-3)
    drv25.set_correlation_level(level)
    try:
        for d in (3, 5, 7, 9):
            c = rotated_surface_code_memory(d, d, p=1e-3, **noise)
            check(drv25, c.text, label=f"level {level} sc{d} preset", level=level)
        for l, m, r in ((6, 6, 6), (9, 6, 10), (12, 6, 12)):
            c = bivariate_bicycle_memory(rounds=r, l=l, m=m, **noise)
            check(drv25, c.text, label=f"level {level} bb{2 * l * m} preset", level=level)
    finally:
        drv25.set_correlation_level(2)


def test_graph_replays_match_eager_launches(drv25):
    """gp_run replays the compile as a captured HIP graph. Every replay, with
    eager launches, other circuits and rate changes in between, gives exactly
    the eagerly launched result."""
    say("case graph replays")
    ca = rotated_surface_code_memory(9, 9)
    cb = bivariate_bicycle_memory(rounds=3)
    ra = log_uniform_rates(ca.n_channels, 5)

    def compile_with(graph, text, rates=None):
        _gp.gp_debug_set_graph(drv25.handle, graph)
        try:
            return drv25.compile_hypergraph(text, rates).edges()
        finally:
            _gp.gp_debug_set_graph(drv25.handle, 1)

    try:
        eager_a = compile_with(0, ca.text)
        eager_b = compile_with(0, cb.text)
        eager_ar = compile_with(0, ca.text, ra)
        with Driver.from_circuit(ca.text) as other:
            for rep in range(3):
                assert compile_with(1, ca.text) == eager_a, f"replay {rep} a"
                # one lowering replayed several times, with eager work (another
                # driver, synchronised) in between
                drv25.lower(cb.text)
                for k in range(3):
                    drv25.run()
                    assert drv25.fetch().edges() == eager_b, f"replay {rep}.{k} b"
                    assert other.compile_hypergraph(ca.text, ra).edges() == eager_ar
                assert compile_with(1, ca.text, ra) == eager_ar, f"replay {rep} a rates"
    finally:
        _gp.gp_debug_set_graph(drv25.handle, 0)
    assert oracle.run(ca.text).edges().keys() == eager_a.keys()


def test_autotune_keeps_results(drv25):
    """The autotuner picks one of its candidates, the compiles after it still
    match the oracle, and the same shape tuned again comes from the cache."""
    say("case autotune")
    c = rotated_surface_code_memory(11, 11)
    try:
        res = drv25.autotune(c.text, iters=3)
        assert res["fault_cost"] in (2.5e-4, 4.0e-4, 6.2e-4, 9.0e-4, 1.4e-3) and res["ms"] > 0
        assert res["sweep_block"] in (256, 1024)
        assert (res["n_circuits"], res["n_qubits"], res["level"]) == (1, 241, 2)
        with pytest.raises(GpError):
            drv25.run()  # no lowering is current after tuning
        check(drv25, c.text, label="after autotune")
        check(drv25, bivariate_bicycle_memory().text, label="bb after autotune")
        again = drv25.autotune(c.text, iters=3)
        assert again["cached"] == 1 and again["fault_cost"] == res["fault_cost"]
        assert again["sweep_block"] == res["sweep_block"] and again["ms"] == res["ms"]
        check(drv25, c.text, label="after cached tuning")
    finally:
        _gp.gp_set_fault_cost(drv25.handle, 6.2e-4)
        _gp.gp_debug_set_sweep_shape(drv25.handle, 0)


def test_fetch_into_caller_arrays(drv25):
    """gp_fetch_sizes + gp_fetch_copy give exactly gp_fetch's arrays; the copy
    needs a current gp_fetch_sizes (GP_E_STATE after a new run); a batch is
    fetched the same way, with its per-circuit hyperedge offsets."""
    import ctypes
    say("case fetch into caller arrays")
    c = rotated_surface_code_memory(11, 11)
    rates = log_uniform_rates(c.n_channels, 4)
    drv25.lower(c.text, rates)
    drv25.run()
    h = _gp.gp_fetch(drv25.handle)
    try:
        off, bits, q = _gp.gp_edges_offsets(h), _gp.gp_edges_bits(h), _gp.gp_edges_probabilities(h)
        nd, no = _gp.gp_edges_detectors(h), _gp.gp_edges_observables(h)
    finally:
        _gp.gp_edges_free(h)
    drv25.run()
    nd2, no2, off2, bits2, q2, coff2 = _gp.gp_fetch_arrays(drv25.handle)
    assert (nd2, no2) == (nd, no) and list(coff2) == [0, len(q)]
    assert np.array_equal(off2, off) and np.array_equal(bits2, bits)
    assert np.array_equal(q2.view(np.uint64), q.view(np.uint64))
    hg = drv25.fetch()
    assert_parity(hg, oracle.run(c.text, rates=rates), "fetch into caller arrays")
    lib = _gp.load()
    buf = np.empty(len(off), dtype=np.uint64)
    drv25.run()
    assert lib.gp_fetch_copy(drv25.handle, buf.ctypes.data, None, None) == -10
    drv25.fetch()
    # a batch comes out circuit by circuit, each circuit's hyperedges in the
    # order (and with the bits and probabilities) of its compile alone
    with Driver.from_batch([c.text, c.text]) as bd:
        bd.lower_batch([c.text, c.text], [rates, rates])
        bd.run()
        nd3, no3, off3, bits3, q3, coff3 = _gp.gp_fetch_arrays(bd.handle, 2)
        U = len(q2)
        assert (nd3, no3) == (nd, no) and list(coff3) == [0, U, 2 * U]
        nb = int(off2[-1])
        for k in range(2):
            assert np.array_equal(off3[k * U:(k + 1) * U + 1] - off3[k * U], off2)
            assert np.array_equal(bits3[int(off3[k * U]):int(off3[(k + 1) * U])], bits2)
            assert np.array_equal(q3[k * U:(k + 1) * U].view(np.uint64), q2.view(np.uint64))
        assert int(off3[-1]) == 2 * nb
        bd.run()
        got = bd.fetch_batch()
        assert len(got) == 2 and all(np.array_equal(g.q.view(np.uint64), q2.view(np.uint64)) for g in got)


def test_widest_frame_the_lds_holds():
    """The sweep keeps a column's whole qubit frame in LDS. On gfx950 (160 KB per
    work-group, 1 KB kept for static arrays) the 1024-thread sweep holds
    2,783 qubits (32 bytes each next to 72 KB of tables): a circuit that
    reaches qubit 2,782 compiles and equals the oracle, one that reaches qubit
    2,783 fails with GP_E_BOUNDS (-4) and leaves the driver usable."""
    def far(q):
        return (f"R 0 {q}\nX_ERROR(0.1) 0 {q}\nCX 0 {q}\nDEPOLARIZE2(0.01) 0 {q}\nM 0 {q}\n"
                "DETECTOR rec[-1]\nDETECTOR rec[-2]\nOBSERVABLE_INCLUDE(0) rec[-1]\n")
    fits, over = far(2782), far(2783)
    say("case widest frame")
    with Driver(merged_bounds([fits, over])) as d:
        assert_parity(d.compile_hypergraph(fits), oracle.run(fits), "2,783 qubits")
        with pytest.raises(GpError) as e:
            d.compile_hypergraph(over)
        assert e.value.code == -4 and "LDS" in str(e.value)
        assert_parity(d.compile_hypergraph(fits), oracle.run(fits), "2,783 qubits again")
