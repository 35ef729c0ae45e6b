"""GPU parity of batched compiles: several circuits lowered together and run
by one pass of each stage (paper Sec. 3.4 compiles many instances of a
circuit; Sec. 3.3 notes the stages parallelise over faults, so a batch is one
larger data-parallel job).

Every circuit of a batch must come out exactly as it does alone: the same
hyperedges (bit for bit), probabilities equal to the single compile's bitwise
and to the oracle's within 1e-12 relative. Identical circuits in one batch
must not merge across circuits. Covered: mixed families and sizes, per-circuit
rates, degenerate members (empty, noise-free, no detectors), both stage-2
groupings, forced key collisions, rate refresh and the stage-2 adjoint over a
batch, and the bounds checks.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_2604_16613_amd import Driver, GpError
from paper_2604_16613_amd import _gp
from workloads import (bit_flip_code_fig1, log_uniform_rates, mirror_circuit, repetition_code_memory,
                       rotated_surface_code_memory)

pytestmark = pytest.mark.gpu

REL_TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def assert_same(hg, ref, label, exact=False):
    """Same hyperedge set; probabilities bitwise equal (exact) or within REL_TOL."""
    g = hg.edges()
    assert len(g) == len(hg), f"{label}: duplicate hyperedges"
    o = ref.edges()
    missing = set(o) - set(g)
    extra = set(g) - set(o)
    assert not missing and not extra, f"{label}: {len(missing)} missing, {len(extra)} extra hyperedges"
    assert hg.n_detectors == ref.n_detectors and hg.n_observables == ref.n_observables, label
    for k, qo in o.items():
        if exact:
            assert g[k] == qo, f"{label}: {k} {g[k]!r} != {qo!r}"
        else:
            rel = abs(g[k] - qo) / qo if qo > 0 else abs(g[k])
            assert rel <= REL_TOL, f"{label}: {k} relative error {rel:.3e}"


def mixed_batch():
    cs = [
        ("sc5", rotated_surface_code_memory(5, 5).text, None),
        ("fig1", bit_flip_code_fig1().text, None),
        ("empty", "", None),
        ("sc3_rates", None, None),
        ("rep7", repetition_code_memory(7, 5, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04).text, None),
        ("noise_free", "R 0 1\nCX 0 1\nM 0 1\nDETECTOR rec[-1] rec[-2]\n", None),
        ("no_det", "R 0\nX_ERROR(0.1) 0\nM 0\n", None),
        ("mirror", mirror_circuit(5, 6, 1, x_basis=[1, 2]).text, None),
        ("sc9", rotated_surface_code_memory(9, 9).text, None),
        ("obs_only", "R 0\nX_ERROR(0.25) 0\nM 0\nOBSERVABLE_INCLUDE(3) rec[-1]\n", None),
    ]
    c3 = rotated_surface_code_memory(3, 3)
    cs[3] = ("sc3_rates", c3.text, log_uniform_rates(c3.n_channels, 7))
    return cs


@pytest.fixture(scope="module")
def batch_driver():
    cs = mixed_batch()
    say("creating a batch driver for", len(cs), "circuits")
    d = Driver.from_batch([t for _, t, _ in cs])
    yield d
    d.close()


def test_batch_bounds_cover_the_batch(batch_driver):
    cs = mixed_batch()
    b = batch_driver.bounds
    assert b.max_branches == len(cs)
    singles = [_gp.gp_bounds_from_circuit(t) for _, t, _ in cs]
    assert b.max_faults == sum(s.max_faults for s in singles)
    assert b.max_channels == sum(s.max_channels for s in singles)
    assert b.max_qubits == max(s.max_qubits for s in singles)
    assert b.max_detectors == max(s.max_detectors for s in singles)


def test_mixed_batch_matches_oracle_and_single_compiles(batch_driver):
    cs = mixed_batch()
    say("case mixed batch")
    got = batch_driver.compile_batch([t for _, t, _ in cs], [r for _, _, r in cs])
    info = batch_driver.info()
    assert info["n_circuits"] == len(cs)
    assert len(got) == len(cs)
    for (name, text, rates), hg in zip(cs, got):
        assert_same(hg, oracle.run(text, rates=rates), f"batch {name} vs oracle")
    # the same circuits compiled one at a time by the same driver
    for (name, text, rates), hg in zip(cs, got):
        assert_same(hg, batch_driver.compile_hypergraph(text, rates), f"batch {name} vs single", exact=True)


def test_identical_circuits_do_not_merge(batch_driver):
    """Equal signatures in different circuits stay in their own circuits."""
    say("case identical circuits")
    c = rotated_surface_code_memory(5, 5)
    rates = [log_uniform_rates(c.n_channels, s) for s in range(4)]
    got = batch_driver.compile_batch([c.text] * 4, rates)
    for k, hg in enumerate(got):
        assert_same(hg, oracle.run(c.text, rates=rates[k]), f"copy {k}")
        assert_same(hg, batch_driver.compile_hypergraph(c.text, rates[k]), f"copy {k} vs single", exact=True)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_grouping_paths(batch_driver, mode):
    cs = mixed_batch()
    _gp.gp_debug_set_sort_mode(batch_driver.handle, mode)
    try:
        say("case batch sort mode", mode)
        got = batch_driver.compile_batch([t for _, t, _ in cs], [r for _, _, r in cs])
        for (name, text, rates), hg in zip(cs, got):
            assert_same(hg, oracle.run(text, rates=rates), f"mode {mode} {name}")
    finally:
        _gp.gp_debug_set_sort_mode(batch_driver.handle, 0)


def test_batch_forced_key_collisions(batch_driver):
    cs = mixed_batch()
    _gp.gp_debug_set_key_bits(batch_driver.handle, 6)
    try:
        say("case batch key collisions")
        before = _gp.gp_debug_collision_retries(batch_driver.handle)
        got = batch_driver.compile_batch([t for _, t, _ in cs], [r for _, _, r in cs])
        assert _gp.gp_debug_collision_retries(batch_driver.handle) == before + 1
        for (name, text, rates), hg in zip(cs, got):
            assert_same(hg, oracle.run(text, rates=rates), f"collisions {name}")
    finally:
        _gp.gp_debug_set_key_bits(batch_driver.handle, 64)


def test_batch_of_one_is_a_plain_compile(batch_driver):
    say("case batch of one")
    c = rotated_surface_code_memory(9, 9)
    (hg,) = batch_driver.compile_batch([c.text])
    assert_same(hg, batch_driver.compile_hypergraph(c.text), "batch of one", exact=True)


def test_batch_refresh_and_gradient(batch_driver):
    """Channels of a batch are numbered circuit by circuit; refresh and the
    adjoint over the batch equal those of each circuit alone."""
    say("case batch refresh and gradient")
    ca = rotated_surface_code_memory(3, 3)
    cb = repetition_code_memory(5, 3, p_data=0.01, p_meas=0.02, p2=0.03, p1=0.04)
    texts = [ca.text, cb.text]
    batch_driver.compile_batch(texts)
    ra = log_uniform_rates(ca.n_channels, 11)
    rb = log_uniform_rates(cb.n_channels, 12)
    _gp.gp_refresh_rates(batch_driver.handle, np.concatenate([ra, rb]))
    got = batch_driver.fetch_batch()
    assert_same(got[0], oracle.run(ca.text, rates=ra), "refresh a")
    assert_same(got[1], oracle.run(cb.text, rates=rb), "refresh b")
    # adjoint with dL/dq = 1 on circuit a's hyperedges and 2 on circuit b's
    batch_driver.lower_batch(texts, [ra, rb])
    batch_driver.run()
    h = _gp.gp_fetch(batch_driver.handle)
    try:
        n_edges = _gp.gp_edges_count(h)
        circuit_of = _gp.gp_edges_circuit_ids(h)
    finally:
        _gp.gp_edges_free(h)
    weight = np.where(circuit_of == 0, 1.0, 2.0)
    g = _gp.gp_rates_gradient(batch_driver.handle, weight, ca.n_channels + cb.n_channels)
    ga = oracle.gradient(ca.text, np.ones(oracle.run(ca.text, rates=ra).n_edges), rates=ra)
    gb = oracle.gradient(cb.text, np.ones(oracle.run(cb.text, rates=rb).n_edges), rates=rb)
    np.testing.assert_allclose(g[:ca.n_channels], ga, rtol=1e-11, atol=1e-300)
    np.testing.assert_allclose(g[ca.n_channels:], 2.0 * gb, rtol=1e-11, atol=1e-300)
    assert n_edges == len(circuit_of)


def test_batch_bounds_errors():
    say("case batch bounds")
    c3 = rotated_surface_code_memory(3, 3).text
    with Driver.from_batch([c3, c3]) as d:
        with pytest.raises(GpError) as e:
            d.compile_batch([c3, c3, c3])
        assert e.value.code == -4
        with pytest.raises(GpError) as e:
            d.compile_batch([c3, rotated_surface_code_memory(5, 5).text])
        assert e.value.code == -4
        with pytest.raises(GpError) as e:
            d.compile_batch([c3, "R 0\nH 0\nM 0\nDETECTOR rec[-1]\n"])
        assert e.value.code == -5
        with pytest.raises(GpError) as e:
            d.compile_batch([c3, "CX 0\n"])
        assert e.value.code == -2 and "circuit 1" in str(e.value)
        got = d.compile_batch([c3, c3])
        for hg in got:
            assert_same(hg, oracle.run(c3), "after errors")
        # a plain compile on a batch driver; DEM text per circuit of a batch
        single = d.compile_detector_error_model(c3)
        _gp.gp_lower_batch(d.handle, [c3, c3])
        _gp.gp_run(d.handle)
        h = _gp.gp_fetch(d.handle)
        try:
            with pytest.raises(GpError) as e:
                _gp.gp_edges_to_dem_text(h)
            assert e.value.code == -10
            for k in range(2):
                assert sorted(_gp.gp_edges_circuit_dem_text(h, k).splitlines()) == sorted(single.splitlines())
        finally:
            _gp.gp_edges_free(h)


@pytest.mark.parametrize("d,n", [(3, 64), (4, 32), (5, 16), (6, 8), (8, 4)])
def test_concatenated_branches_batch(d, n):
    """Realised branches of the adaptive [[4,2,2]]-concatenated surface code
    (uneven lengths), compiled as one batch, against the oracle per branch;
    the even outer distances are those of the paper's adaptive benchmark
    (Table 3)."""
    from workloads import iceberg_surface_batch
    texts = [c.text for c in iceberg_surface_batch(d, n_branches=n, seed=100)]
    say("case concatenated batch", d, n)
    with Driver.from_batch(texts) as drv:
        got = drv.compile_batch(texts)
        for k, (t, hg) in enumerate(zip(texts, got)):
            assert_same(hg, oracle.run(t), f"d{d} branch {k}")


@pytest.mark.parametrize("level", [0, 1])
def test_concatenated_batch_at_correlation_levels(level):
    """The adaptive benchmark at the lower correlation levels (Table 3 reports
    all three): a batch of branches at outer distance 4 keeps, per branch, the
    oracle's classes at that level, and equals the branch compiled alone at that
    level."""
    from workloads import iceberg_surface_batch
    texts = [c.text for c in iceberg_surface_batch(4, n_branches=12, seed=300)]
    say("case concatenated batch at level", level)
    with Driver.from_batch(texts) as drv:
        drv.set_correlation_level(level)
        got = drv.compile_batch(texts)
        for k in (0, 5, 11):
            assert_same(got[k], oracle.run(texts[k], level=level), f"level {level} branch {k} vs oracle")
        for k, t in enumerate(texts):
            assert_same(got[k], drv.compile_hypergraph(t), f"level {level} branch {k} vs single", exact=True)


def test_concatenated_d10_batch_samples():
    """Outer distance 10: a batch of 12 branches; every branch equals its own
    compile, two of them are checked against the oracle."""
    from workloads import iceberg_surface_batch
    texts = [c.text for c in iceberg_surface_batch(10, n_branches=12, seed=7)]
    say("case concatenated d10 batch")
    with Driver.from_batch(texts) as drv:
        got = drv.compile_batch(texts)
        for k in (0, 11):
            assert_same(got[k], oracle.run(texts[k]), f"d10 branch {k} vs oracle")
        for k, t in enumerate(texts):
            assert_same(got[k], drv.compile_hypergraph(t), f"d10 branch {k} vs single", exact=True)


def test_batch_result_is_listed_circuit_by_circuit(batch_driver):
    cs = mixed_batch()
    batch_driver.lower_batch([t for _, t, _ in cs], [r for _, _, r in cs])
    batch_driver.run()
    h = _gp.gp_fetch(batch_driver.handle)
    try:
        ids = _gp.gp_edges_circuit_ids(h)
        cut = _gp.gp_edges_circuit_offsets(h)
        assert len(cut) == len(cs) + 1 and cut[0] == 0 and cut[-1] == len(ids)
        assert np.all(np.diff(ids.astype(np.int64)) >= 0)
        for k in range(len(cs)):
            assert np.all(ids[cut[k]:cut[k + 1]] == k)
    finally:
        _gp.gp_edges_free(h)


@pytest.mark.parametrize("shape", [1, 2])
def test_forced_sweep_shapes_match_oracle(batch_driver, shape):
    """Both stage-1 work-group shapes (1024 threads with the large LDS tables,
    256 threads with the small ones) give the oracle's hypergraphs on the mixed
    batch; the automatic choice only picks the small one for large batches."""
    cs = mixed_batch()
    say("case forced sweep shape", shape)
    _gp.gp_debug_set_sweep_shape(batch_driver.handle, shape)
    try:
        got = batch_driver.compile_batch([t for _, t, _ in cs], [r for _, _, r in cs])
    finally:
        _gp.gp_debug_set_sweep_shape(batch_driver.handle, 0)
    for (name, t, r), hg in zip(cs, got):
        assert_same(hg, oracle.run(t, r), f"{name} shape {shape}")


def test_small_shape_with_long_injection_lists():
    """Outer distance 10 branches under the 256-thread shape: some columns carry
    more injections than its LDS list holds, so they are read from global
    memory. Equal to the 1024-thread shape bit for bit, and to the oracle on one
    branch."""
    from workloads import iceberg_surface_batch
    texts = [c.text for c in iceberg_surface_batch(10, n_branches=6, seed=3)]
    say("case small shape d10")
    with Driver.from_batch(texts) as drv:
        _gp.gp_debug_set_sweep_shape(drv.handle, 1)
        big = drv.compile_batch(texts)
        _gp.gp_debug_set_sweep_shape(drv.handle, 2)
        small = drv.compile_batch(texts)
    for k in range(len(texts)):
        assert_same(small[k], big[k], f"d10 branch {k} small vs big", exact=True)
    assert_same(small[5], oracle.run(texts[5]), "d10 branch 5 vs oracle")


def test_batch_autotune_keeps_results():
    """Batch tuning over the work-group sizes and range cuts: the choice is one
    of the candidates, compiles after it match the oracle, and a second call
    comes from the cache."""
    from workloads import iceberg_surface_batch
    texts = [c.text for c in iceberg_surface_batch(3, n_branches=48, seed=11)]
    say("case batch autotune")
    with Driver.from_batch(texts) as drv:
        res = drv.autotune_batch(texts, iters=2)
        assert res["sweep_block"] in (256, 1024) and res["ms"] > 0 and res["n_circuits"] == 48
        got = drv.compile_batch(texts)
        for k in (0, 17, 47):
            assert_same(got[k], oracle.run(texts[k]), f"branch {k} after batch tuning")
        again = drv.autotune_batch(texts, iters=2)
        assert again["cached"] == 1 and again["sweep_block"] == res["sweep_block"]


@pytest.mark.parametrize("d,n,b16", [(5, 64, False), (7, 192, True)])
def test_batch_past_the_256_buckets(d, n, b16):
    """Batches larger than the 256 buckets take: 64 branches at outer distance
    5 (1.65 M faults: the automatic grouping runs the full sort) and 192 at
    distance 7 (13.4 M faults: the 65,536 buckets). Every branch equals its own
    compile bitwise, three equal the oracle."""
    from workloads import iceberg_surface_batch
    texts = [c.text for c in iceberg_surface_batch(d, n_branches=n, seed=21)]
    say("case past the 256 buckets", d, n)
    with Driver.from_batch(texts) as drv:
        got = drv.compile_batch(texts)
        info = drv.info()
        F = info["n_faults"]
        assert F > 1572864 and (F >= 12000000) == b16
        for k in (0, n // 2, n - 1):
            assert_same(got[k], oracle.run(texts[k]), f"branch {k} vs oracle")
        live = nz = 0
        for k, t in enumerate(texts):
            assert_same(got[k], drv.compile_hypergraph(t), f"branch {k} vs single", exact=True)
            live += drv.info()["n_live_faults"]
            nz += drv.info()["n_nonzero_words"]
        # the batch's counters (summed per compaction tile; over 1024 tiles by
        # the tile-prefix pass) equal the sums over the circuits
        assert (info["n_live_faults"], info["n_nonzero_words"]) == (live, nz)
