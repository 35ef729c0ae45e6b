"""GPU tests at the sizes the benchmark measures, and of the sort's bounded
look-back wait.

- The batched workload exactly as benchmarked: 256 realised branches of the
  adaptive [[4,2,2]]-concatenated surface code at outer distance 10 (seeds
  0..255, 51 M faults, the 65,536-bucket grouping), compiled as one batch.
  Every branch must equal its own compile bit for bit, and four branches
  (first, two middle, last) the oracle to 1e-12.
- A radix-sort tile that gives up waiting for its predecessor (forced from the
  host with a spin limit of 0, so that no kernel ever waits) must fail the
  fetch, under every grouping, instead of returning misplaced pairs.
"""

import sys

import numpy as np
import pytest

import oracle
from canon import assert_bitwise_equal
from paper_2604_16613_amd import Driver, GpError
from paper_2604_16613_amd import _gp
from workloads import iceberg_surface_batch, rotated_surface_code_memory

pytestmark = pytest.mark.gpu

REL_TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def assert_oracle(hg, text, label):
    ref = oracle.run(text)
    g, o = hg.edges(), ref.edges()
    assert set(g) == set(o), f"{label}: hyperedge sets differ ({len(g)} vs {len(o)})"
    worst = max((abs(g[k] - q) / q if q > 0 else abs(g[k]) for k, q in o.items()), default=0.0)
    assert worst <= REL_TOL, f"{label}: worst relative error {worst:.3e}"


@pytest.mark.timeout(600)
def test_benchmarked_batch_256_branches_d10():
    say("case batch 256 x d10: generating")
    texts = [c.text for c in iceberg_surface_batch(10, n_branches=256, seed=0)]
    say("case batch 256 x d10: compiling the batch")
    with Driver.from_batch(texts) as drv:
        got = drv.compile_batch(texts)
        info = drv.info()
        flags, seen = _gp.gp_debug_device_flags(drv.handle, clear_seen=True)
        retries = _gp.gp_debug_retry_counts(drv.handle)
    assert info["n_faults"] > 50_000_000 and info["n_circuits"] == 256
    assert flags == 0 and seen == 0 and retries == {"lookback": 0, "bucket": 0, "collision": 0}
    assert len(got) == 256
    say("case batch 256 x d10: every branch against its own compile")
    sizes = [_gp.gp_bounds_from_circuit(t) for t in texts]
    bounds = _gp.GpBounds()
    for f, _ in bounds._fields_:
        setattr(bounds, f, max(getattr(b, f) for b in sizes))
    bounds.max_slab_words = 0
    bounds.max_items = 0
    total = 0
    with Driver(bounds) as single:
        for k, t in enumerate(texts):
            alone = single.compile_hypergraph(t)
            assert_bitwise_equal(got[k], alone, f"branch {k}")
            total += len(alone)
            if k % 64 == 63:
                say(f"  {k + 1} branches equal")
    assert total == sum(len(h) for h in got)
    for k in (0, 85, 170, 255):
        say(f"case batch 256 x d10: branch {k} against the oracle")
        assert_oracle(got[k], texts[k], f"branch {k}")


@pytest.fixture(scope="module")
def d17():
    c = rotated_surface_code_memory(17, 17)
    drv = Driver.from_circuit(c.text)
    yield drv, c.text
    drv.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_lookback_give_up_fails_the_fetch(d17, mode):
    """Spin limit 0: every sort tile after the first gives up at once. The
    later grouping kernels do nothing, the fetch runs the compile once more
    and then fails with GP_E_HIP; with the default limit the next compile is
    the oracle's again."""
    drv, text = d17
    say("case look-back give-up, sort mode", mode)
    _gp.gp_debug_set_sort_mode(drv.handle, mode)
    before = _gp.gp_debug_retry_counts(drv.handle)["lookback"]
    try:
        _gp.gp_debug_set_spin_limit(drv.handle, 0)
        with pytest.raises(GpError) as e:
            drv.compile_hypergraph(text)
        assert e.value.code == -7 and "gave up" in str(e.value)
        assert _gp.gp_debug_retry_counts(drv.handle)["lookback"] == before + 1
        _, seen = _gp.gp_debug_device_flags(drv.handle, clear_seen=True)
        assert seen & 8
    finally:
        _gp.gp_debug_set_spin_limit(drv.handle, 1 << 22)
        _gp.gp_debug_set_sort_mode(drv.handle, 0)
    assert_oracle(drv.compile_hypergraph(text), text, "after the give-up")
    flags, seen = _gp.gp_debug_device_flags(drv.handle, clear_seen=True)
    assert flags == 0 and seen == 0
