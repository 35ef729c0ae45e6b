"""GPU parity of the fixed-structure rate refresh and of the stage-2 adjoint
(through the C ABI), against the oracle.

Workload of the differentiation row: rotated surface code d = 9, 9 rounds,
per-channel rates log-uniform in [1e-4, 5e-3) (seed 0); loss
L = sum_k w_k log(q_k / (1 - q_k)) with w_k ~ U[-1, 1] (seed 1) assigned to
the hyperedges in sorted-signature order. The gradient must match the
oracle's to 1e-9 relative and central differences of the device forward
pass within their error.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from paper_2604_16613_amd import GpError, get_driver
from paper_2604_16613_amd import _gp
from workloads import log_uniform_rates, logit_loss, rotated_surface_code_memory

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _weights(sigs, seed=1):
    """w per signature, drawn in sorted-signature order."""
    order = sorted(sigs)
    w = np.random.default_rng(seed).uniform(-1.0, 1.0, len(order))
    return dict(zip(order, w))


def _gpu_dl_dq(hg, wmap):
    sigs = [tuple(int(b) for b in hg.bits[hg.offsets[e]:hg.offsets[e + 1]]) for e in range(len(hg))]
    w = np.array([wmap[s] for s in sigs])
    return logit_loss(hg.q, w)


def _oracle_dl_dq(res, wmap):
    sigs = [tuple(int(b) for b in res.edge_bits[res.edge_off[e]:res.edge_off[e + 1]]) for e in range(res.n_edges)]
    w = np.array([wmap[s] for s in sigs])
    return oracle.loss_and_dl_dq(res.edge_q, w)


@pytest.fixture(scope="module")
def c5():
    c = rotated_surface_code_memory(9, 9)
    rates = log_uniform_rates(c.n_channels, 0)
    drv = get_driver(c.text)
    yield c, rates, drv
    drv.close()


def test_gradient_matches_oracle_c5(c5):
    c, rates, drv = c5
    say("case c5 gradient vs oracle")
    hg = drv.compile_hypergraph(c.text, rates)
    res = oracle.run(c.text, rates=rates)
    wmap = _weights(hg.edges().keys())
    _, g_gpu_q = _gpu_dl_dq(hg, wmap)
    _, g_orc_q = _oracle_dl_dq(res, wmap)
    g_gpu = drv.rates_gradient(g_gpu_q)
    g_orc = oracle.gradient(c.text, g_orc_q, rates=rates)
    assert g_gpu.shape == (c.n_channels,)
    scale = np.abs(g_orc)
    err = np.abs(g_gpu - g_orc)
    assert np.all(err <= 1e-9 * scale + 1e-300), float(np.max(err / np.maximum(scale, 1e-300)))


def test_refresh_equals_full_compile(c5):
    c, rates, drv = c5
    say("case refresh vs compile")
    drv.compile_hypergraph(c.text, rates)
    r2 = log_uniform_rates(c.n_channels, 7)
    refreshed = drv.refresh_rates(r2)
    full = drv.compile_hypergraph(c.text, r2)
    assert np.array_equal(refreshed.offsets, full.offsets)
    assert np.array_equal(refreshed.bits, full.bits)
    assert np.array_equal(refreshed.q.view(np.uint64), full.q.view(np.uint64))


@pytest.mark.parametrize("mode", [1, 2])
def test_refresh_and_gradient_after_other_groupings(c5, mode):
    """The class structure left by the full sort and by the 65,536-bucket
    grouping: a refresh equals a full compile bitwise, and the adjoint equals
    the oracle's gradient."""
    c, rates, drv = c5
    say("case refresh and gradient, sort mode", mode)
    _gp.gp_debug_set_sort_mode(drv.handle, mode)
    try:
        hg = drv.compile_hypergraph(c.text, rates)
        wmap = _weights(hg.edges().keys())
        _, g_gpu_q = _gpu_dl_dq(hg, wmap)
        res = oracle.run(c.text, rates=rates)
        _, g_orc_q = _oracle_dl_dq(res, wmap)
        g_gpu = drv.rates_gradient(g_gpu_q)
        g_orc = oracle.gradient(c.text, g_orc_q, rates=rates)
        err = np.abs(g_gpu - g_orc)
        assert np.all(err <= 1e-9 * np.abs(g_orc) + 1e-300)
        r2 = log_uniform_rates(c.n_channels, 7)
        refreshed = drv.refresh_rates(r2)
        full = drv.compile_hypergraph(c.text, r2)
        assert np.array_equal(refreshed.offsets, full.offsets)
        assert np.array_equal(refreshed.bits, full.bits)
        assert np.array_equal(refreshed.q.view(np.uint64), full.q.view(np.uint64))
    finally:
        _gp.gp_debug_set_sort_mode(drv.handle, 0)


def test_gradient_matches_device_finite_differences(c5):
    """Central differences (h = 1e-7) of the device forward pass against the
    device adjoint, each within the difference quotient's own error bound:
    truncation h^2 |L3| / 6, with the third derivative L3 taken from a
    five-point stencil of step 1e-2 r, plus rounding 2 u_L / (2h), where u_L
    bounds the error of evaluating L_c = sum over the hyperedges channel c
    moves of w_k log(q_k / (1 - q_k)) (a few ulps of each q, one ulp of each
    log). Only the hyperedges the channel touches enter L_c, as the other
    terms cancel exactly."""
    c, rates, drv = c5
    say("case c5 gradient vs central differences")
    hg = drv.compile_hypergraph(c.text, rates)
    wmap = _weights(hg.edges().keys())
    sigs = [tuple(int(b) for b in hg.bits[hg.offsets[e]:hg.offsets[e + 1]]) for e in range(len(hg))]
    w = np.array([wmap[s_] for s_ in sigs])
    _, g_q = logit_loss(hg.q, w)
    grad = drv.rates_gradient(g_q)
    base = hg.q.copy()
    h = 1e-7
    eps = np.finfo(np.float64).eps
    rng = np.random.default_rng(3)
    worst = 0.0
    for ch in rng.choice(c.n_channels, 24, replace=False):
        def q_at(x):
            r = rates.copy()
            r[ch] = x
            return drv.refresh_rates(r).q

        r0 = rates[ch]
        qp, qm = q_at(r0 + h), q_at(r0 - h)
        touched = (qp != base) | (qm != base)
        assert touched.any()
        wt = w[touched]

        def L(q):
            qt = q[touched]
            return float(np.sum(wt * np.log(qt / (1.0 - qt))))

        fd = (L(qp) - L(qm)) / (2 * h)
        H = 1e-2 * r0
        f3 = (L(q_at(r0 + 2 * H)) - 2 * L(q_at(r0 + H)) + 2 * L(q_at(r0 - H)) - L(q_at(r0 - 2 * H))) / (2 * H ** 3)
        trunc = h * h * abs(f3) / 6.0
        qt = base[touched]
        u_l = float(np.sum(np.abs(wt) * (8 * eps / (1.0 - qt) + eps * np.abs(np.log(qt / (1.0 - qt))))))
        bound = trunc + 2 * u_l / (2 * h)
        err = abs(fd - grad[ch])
        worst = max(worst, err / bound)
        assert err <= 2.0 * bound, (int(ch), fd, grad[ch], trunc, bound)
    say(f"  worst |fd - adjoint| / bound = {worst:.3f}")
    drv.refresh_rates(rates)


def test_gradient_with_half_probability_members(c5):
    _, _, drv = c5
    say("case p = 1/2 members")
    text = ("X_ERROR(0.5) 0\nX_ERROR(0.1) 0\nX_ERROR(0.2) 1\nX_ERROR(0.5) 1\nX_ERROR(0.5) 1\n"
            "DEPOLARIZE1(0.75) 2\nM 0 1 2\nDETECTOR rec[-3]\nDETECTOR rec[-2]\nDETECTOR rec[-1]\n")
    hg = drv.compile_hypergraph(text)
    res = oracle.run(text)
    wmap = _weights(hg.edges().keys(), seed=5)
    g_gpu = drv.rates_gradient(_gpu_dl_dq(hg, wmap)[1])
    g_orc = oracle.gradient(text, _oracle_dl_dq(res, wmap)[1])
    finite = np.isfinite(g_orc)
    assert np.array_equal(finite, np.isfinite(g_gpu))
    assert np.allclose(g_gpu[finite], g_orc[finite], rtol=1e-12, atol=1e-300)


def test_gradient_through_the_bucket_overflow_path(c5):
    _, _, drv = c5
    say("case gradient, class larger than a bucket")
    rates = np.linspace(1e-7, 2e-5, 9000)
    text = "\n".join(f"X_ERROR({r:.17g}) 0" for r in rates) + "\nX_ERROR(0.01) 1\nM 0 1\nDETECTOR rec[-2]\nDETECTOR rec[-1]\n"
    with get_driver(text) as big:
        hg = big.compile_hypergraph(text)
        res = oracle.run(text)
        wmap = _weights(hg.edges().keys(), seed=2)
        g_gpu = big.rates_gradient(_gpu_dl_dq(hg, wmap)[1])
        g_orc = oracle.gradient(text, _oracle_dl_dq(res, wmap)[1])
    assert np.allclose(g_gpu, g_orc, rtol=1e-9, atol=0)


def test_state_and_argument_errors(c5):
    c, rates, drv = c5
    say("case adjoint error paths")
    drv.lower(c.text, rates)
    with pytest.raises(GpError) as e:
        drv.rates_gradient(np.zeros(3))
    assert e.value.code == -10  # GP_E_STATE: no fetched compile of this lowering
    hg = drv.compile_hypergraph(c.text, rates)
    with pytest.raises(GpError) as e:
        _gp.gp_rates_gradient(drv.handle, np.zeros(len(hg) + 1), c.n_channels)
    assert e.value.code == -1
    with pytest.raises(GpError) as e:
        drv.refresh_rates(np.full(c.n_channels, 2.0))
    assert e.value.code == -6
    # the failed refresh left the rates alone
    again = drv.refresh_rates(rates)
    assert np.array_equal(again.q.view(np.uint64), hg.q.view(np.uint64))


def _cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("torch sees no GPU")
    return torch


def test_device_pointer_aggregate_and_backward(c5):
    """gp_aggregate / gp_aggregate_backward on device arrays and torch's
    stream give bitwise what the host-array refresh and adjoint give."""
    torch = _cuda()
    c, rates, drv = c5
    say("case device-pointer aggregate")
    hg = drv.compile_hypergraph(c.text, rates)
    r2 = log_uniform_rates(c.n_channels, 11)
    dr = torch.tensor(r2, dtype=torch.float64, device="cuda")
    dq = torch.empty(len(hg), dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    _gp.gp_aggregate(drv.handle, dr.data_ptr(), dr.numel(), dq.data_ptr(), dq.numel(), s)
    ref = drv.refresh_rates(r2)
    assert np.array_equal(dq.cpu().numpy().view(np.uint64), ref.q.view(np.uint64))
    wmap = _weights(hg.edges().keys(), seed=9)
    _, g_q = _gpu_dl_dq(ref, wmap)
    dg = torch.tensor(g_q, dtype=torch.float64, device="cuda")
    dgr = torch.empty_like(dr)
    # the backward takes its rates as an argument: apply others first
    drv.refresh_rates(rates)
    _gp.gp_aggregate_backward(drv.handle, dr.data_ptr(), dr.numel(), dg.data_ptr(), dg.numel(), dgr.data_ptr(), s)
    host = drv.refresh_rates(r2)
    expect = drv.rates_gradient(g_q)
    assert np.array_equal(host.q.view(np.uint64), ref.q.view(np.uint64))
    assert np.array_equal(dgr.cpu().numpy().view(np.uint64), expect.view(np.uint64))
    with pytest.raises(GpError) as e:
        _gp.gp_aggregate(drv.handle, dr.data_ptr(), dr.numel() - 1, dq.data_ptr(), dq.numel(), s)
    assert e.value.code == -1


def test_device_pointer_aggregate_on_a_batch():
    """A batch result is listed circuit by circuit; the device aggregate
    writes q in that order too (bitwise equal to the host refresh)."""
    torch = _cuda()
    from paper_2604_16613_amd import Driver
    from workloads import iceberg_surface_batch
    say("case device-pointer aggregate, batch")
    texts = [cc.text for cc in iceberg_surface_batch(3, n_branches=8, seed=40)]
    with Driver.from_batch(texts) as drv:
        drv.compile_batch(texts)
        U = int(drv.info()["n_edges"])
        C = int(drv.info()["n_channels"])
        r = log_uniform_rates(C, 4)
        dr = torch.tensor(r, dtype=torch.float64, device="cuda")
        dq = torch.empty(U, dtype=torch.float64, device="cuda")
        _gp.gp_aggregate(drv.handle, dr.data_ptr(), C, dq.data_ptr(), U, torch.cuda.current_stream().cuda_stream)
        ref = drv.refresh_rates(r)
        assert len(ref.q) == U
        assert np.array_equal(dq.cpu().numpy().view(np.uint64), ref.q.view(np.uint64))


def test_torch_autograd_wrapper(c5):
    torch = _cuda()
    from paper_2604_16613_amd.autograd import HypergraphFunction
    c, rates, drv = c5
    say("case torch autograd")
    f = HypergraphFunction(drv, c.text)
    f.compile(rates)
    wmap = _weights(f.structure.edges().keys())
    sigs = [tuple(int(b) for b in f.structure.bits[f.structure.offsets[e]:f.structure.offsets[e + 1]])
            for e in range(len(f.structure))]
    w = torch.tensor([wmap[s] for s in sigs], dtype=torch.float64, device="cuda")
    r = torch.tensor(rates, dtype=torch.float64, device="cuda", requires_grad=True)
    q = f(r)
    assert np.array_equal(q.detach().cpu().numpy().view(np.uint64), f.structure.q.view(np.uint64))
    loss = torch.sum(w * torch.log(q / (1 - q)))
    loss.backward()
    _, g_q = _gpu_dl_dq(f.structure, wmap)
    expect = drv.rates_gradient(g_q)
    # torch differentiates log(q / (1 - q)) through the division: dL/dq agrees to rounding
    assert np.allclose(r.grad.cpu().numpy(), expect, rtol=1e-10, atol=0)


def test_torch_autograd_keeps_each_forward_rates(c5):
    """Two forward passes at different rates, then the backward of the first
    alone: its gradient is the one at the first rates (the backward does not
    use whatever rates the driver applied last). A compile of another circuit
    between forward and backward is refused."""
    torch = _cuda()
    from paper_2604_16613_amd.autograd import HypergraphFunction
    c, rates, drv = c5
    say("case autograd with two forwards")
    f = HypergraphFunction(drv, c.text)
    f.compile(rates)
    wmap = _weights(f.structure.edges().keys(), seed=4)
    sigs = [tuple(int(b) for b in f.structure.bits[f.structure.offsets[e]:f.structure.offsets[e + 1]])
            for e in range(len(f.structure))]
    w = torch.tensor([wmap[s] for s in sigs], dtype=torch.float64, device="cuda")
    r1 = torch.tensor(rates, dtype=torch.float64, device="cuda", requires_grad=True)
    r2 = torch.tensor(log_uniform_rates(c.n_channels, 5), dtype=torch.float64, device="cuda", requires_grad=True)
    q1 = f(r1)
    q2 = f(r2)
    torch.sum(w * torch.log(q1 / (1 - q1))).backward()
    hg1 = drv.refresh_rates(rates)
    _, g_q = _gpu_dl_dq(hg1, wmap)
    expect = drv.rates_gradient(g_q)
    assert np.allclose(r1.grad.cpu().numpy(), expect, rtol=1e-10, atol=0)
    assert r2.grad is None
    drv.compile_hypergraph(rotated_surface_code_memory(3, 3).text)
    with pytest.raises(RuntimeError):
        torch.sum(w * torch.log(q2 / (1 - q2))).backward()
