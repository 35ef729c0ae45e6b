"""The adaptive [[4,2,2]]-concatenated surface-code workload (paper Sec. 5):
the Eq. 6 pairing and its constraints, and realised branches that are valid
inputs (every detector deterministic, the oracle and the CPU replay of the
compiler's tables agree on every fault). No GPU needed."""

import pytest

import host_check
import oracle
from paper_2604_16613_amd import _gp
from workloads import (iceberg_pairing, iceberg_pairing_violations, iceberg_surface_batch,
                       iceberg_surface_branch)


@pytest.mark.parametrize("d", [3, 4, 5, 7, 10])
def test_pairing_covers_every_outer_data_qubit_once(d):
    blocks = iceberg_pairing(d)
    flat = [q for b in blocks for q in b]
    assert sorted(flat) == list(range(d * d))
    assert sum(len(b) == 1 for b in blocks) % 2 == (d * d) % 2
    # no outer check holds both logical qubits of one block (Sec. 5.1.1)
    ft, _ = iceberg_pairing_violations(d)
    assert ft == 0


def test_pairing_is_eq6_where_the_map_is_an_involution():
    # d = 4: (r, c) -> (3 - r, (c + 2) mod 4) is its own inverse, so every block is {x, f(x)}
    d = 4
    for b in iceberg_pairing(d):
        assert len(b) == 2
        r, c = divmod(b[0], d)
        assert b[1] == (d - 1 - r) * d + (c + 2) % d
    # odd d: pairs are still (x, f(x)) along the map's cycles
    d = 5
    for b in iceberg_pairing(d):
        if len(b) == 2:
            r, c = divmod(b[0], d)
            assert b[1] == (d - 1 - r) * d + (c + 2) % d


def test_pairing_violations_detects_a_bad_pairing():
    # pairing outer data 0 and 1 (both in the first X check) breaks the first constraint
    d = 3
    blocks = [(0, 1)] + [(q,) for q in range(2, 9)]
    ft, _ = iceberg_pairing_violations(d, blocks)
    assert ft >= 1


@pytest.mark.parametrize("d,seed", [(3, 0), (3, 5), (5, 1), (5, 2)])
def test_branch_is_deterministic_and_replays(d, seed):
    c = iceberg_surface_branch(d, seed)
    st, sigs = host_check.run(c.text)
    res = oracle.run(c.text, keep_faults=True)
    osig = {(ch, code): sig for ch, code, sig, _ in res.fault_signatures()}
    assert st["gauge"] == 0
    assert sigs == osig
    assert res.n_detectors == c.n_detectors and res.n_observables == 1


def test_branches_are_uneven_and_seeded():
    a = iceberg_surface_batch(5, n_branches=6, seed=10)
    b = iceberg_surface_batch(5, n_branches=6, seed=10)
    assert [x.text for x in a] == [x.text for x in b]
    faults = {_gp.gp_bounds_from_circuit(x.text).max_faults for x in a}
    assert len(faults) > 1


def test_outer_checks_follow_the_refresh_rule():
    # nothing fires: outer checks run only in the first and last cycle and every
    # gamma cycles, so with gamma > cycles they run twice (two detector rounds
    # for Z checks, one comparison for X checks)
    d, cycles = 3, 4
    quiet = iceberg_surface_branch(d, 0, cycles=cycles, p_excite=0.0, gamma=100)
    busy = iceberg_surface_branch(d, 0, cycles=cycles, p_excite=1.0, gamma=100)
    n_outer = d * d - 1
    assert busy.n_detectors - quiet.n_detectors == (cycles - 2) * n_outer


def test_d10_batch_has_columns_longer_than_the_small_injection_list():
    """The 256-thread stage-1 shape keeps up to 256 injection entries per column
    in LDS; the distance-10 GPU case must include longer lists so that the
    global-memory path is exercised there."""
    texts = [c.text for c in iceberg_surface_batch(10, n_branches=6, seed=3)]
    st, _ = host_check.run_batch(texts)
    assert st["max_col_inj"] > 256
