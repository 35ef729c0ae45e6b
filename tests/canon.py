"""Canonical order of a hypergraph's edges, for bit-for-bit comparisons of
large results without building Python dictionaries: every hyperedge becomes a
row (weight, bit_0, bit_1, ..., padded with -1), rows sorted
lexicographically, probabilities carried along."""

import numpy as np


def canonical(hg):
    off = np.asarray(hg.offsets, dtype=np.int64)
    U = len(hg.q)
    w = np.diff(off)
    width = int(w.max()) if U else 0
    rows = np.full((U, width + 1), -1, dtype=np.int64)
    rows[:, 0] = w
    if len(hg.bits):
        edge = np.repeat(np.arange(U), w)
        col = np.arange(len(hg.bits), dtype=np.int64) - np.repeat(off[:-1], w) + 1
        rows[edge, col] = hg.bits
    order = np.lexsort(rows.T[::-1]) if U else np.zeros(0, dtype=np.int64)
    return rows[order], np.asarray(hg.q)[order]


def assert_bitwise_equal(a, b, label):
    """Same hyperedges with bitwise equal probabilities (any edge order)."""
    assert a.n_detectors == b.n_detectors and a.n_observables == b.n_observables, label
    ra, qa = canonical(a)
    rb, qb = canonical(b)
    assert ra.shape == rb.shape, f"{label}: {ra.shape[0]} vs {rb.shape[0]} hyperedges (or widths differ)"
    assert np.array_equal(ra, rb), f"{label}: hyperedge sets differ"
    assert np.array_equal(qa.view(np.uint64), qb.view(np.uint64)), f"{label}: probabilities differ"
    # no duplicate hyperedges
    if len(ra) > 1:
        assert np.any(ra[1:] != ra[:-1], axis=1).all(), f"{label}: duplicate hyperedges"
