"""Pins of the oracle's stage-2 adjoint (CPU only).

The oracle differentiates q_k = 1/2 (1 - prod (1 - 2 p_i)) with explicit
products over each class's other members and the analytic derivative of the
per-fault split. These tests tie it to things other than its own formula:
central finite differences of the oracle's forward pass, closed forms of the
channel splits (a DEPOLARIZE1 class has q = 2r/3 exactly), and the two-flip
merge rule, including a member at p = 1/2.
"""

import math

import numpy as np
import pytest

import oracle
from workloads import log_uniform_rates, rotated_surface_code_memory


def _loss(text, rates, w):
    return oracle.loss_and_dl_dq(oracle.run(text, rates=rates).edge_q, w)[0]


def test_gradient_matches_central_differences_d3():
    c = rotated_surface_code_memory(3, 3)
    r = log_uniform_rates(c.n_channels, 0)
    res = oracle.run(c.text, rates=r)
    w = np.random.default_rng(1).uniform(-1.0, 1.0, res.n_edges)
    _, g = oracle.loss_and_dl_dq(res.edge_q, w)
    grad = oracle.gradient(c.text, g, rates=r)
    h = 1e-7
    for ch in range(c.n_channels):
        rp, rm = r.copy(), r.copy()
        rp[ch] += h
        rm[ch] -= h
        fd = (_loss(c.text, rp, w) - _loss(c.text, rm, w)) / (2 * h)
        # central differences: truncation O(h^2) plus rounding ~ eps |L| / h
        assert abs(fd - grad[ch]) <= 1e-6 * abs(grad[ch]) + 1e-6, (ch, fd, grad[ch])


@pytest.mark.parametrize("r", [1e-4, 3e-3, 0.2, 0.7])
def test_dep1_class_closed_form(r):
    # X and Y flip the Z measurement: one class of two faults, q = 2r/3, dq/dr = 2/3
    text = f"DEPOLARIZE1({r!r}) 0\nM 0\nDETECTOR rec[-1]\n"
    res = oracle.run(text)
    assert res.n_edges == 1
    assert math.isclose(res.edge_q[0], 2 * r / 3, rel_tol=1e-14)
    g = oracle.gradient(text, [1.0])
    assert math.isclose(g[0], 2.0 / 3.0, rel_tol=1e-13)


@pytest.mark.parametrize("r", [1e-4, 3e-3, 0.5])
def test_dep2_classes_closed_form(r):
    # three classes of four faults each: q = 1/2 (1 - (1 - 16r/15)^(1/2))
    text = f"DEPOLARIZE2({r!r}) 0 1\nM 0 1\nDETECTOR rec[-2]\nDETECTOR rec[-1]\n"
    res = oracle.run(text)
    assert res.n_edges == 3
    q = 0.5 * (1 - math.sqrt(1 - 16 * r / 15))
    assert np.allclose(res.edge_q, q, rtol=1e-13)
    dq = (4.0 / 15.0) / math.sqrt(1 - 16 * r / 15)
    for k in range(3):
        dl = np.zeros(3)
        dl[k] = 1.0
        assert math.isclose(oracle.gradient(text, dl)[0], dq, rel_tol=1e-12)


@pytest.mark.parametrize("p1,p2", [(0.01, 0.2), (0.5, 0.1), (0.3, 0.5)])
def test_two_flip_merge(p1, p2):
    # q = p1 + p2 - 2 p1 p2: dq/dp1 = 1 - 2 p2, dq/dp2 = 1 - 2 p1 (zero at p = 1/2)
    text = f"X_ERROR({p1!r}) 0\nX_ERROR({p2!r}) 0\nM 0\nDETECTOR rec[-1]\n"
    g = oracle.gradient(text, [1.0])
    assert math.isclose(g[0], 1 - 2 * p2, rel_tol=1e-15, abs_tol=1e-300)
    assert math.isclose(g[1], 1 - 2 * p1, rel_tol=1e-15, abs_tol=1e-300)


def test_empty_signature_has_no_gradient():
    # a Z flip before a Z measurement changes nothing
    text = "Z_ERROR(0.1) 0\nX_ERROR(0.2) 0\nM 0\nDETECTOR rec[-1]\n"
    g = oracle.gradient(text, [1.0])
    assert g[0] == 0.0 and math.isclose(g[1], 1.0)
