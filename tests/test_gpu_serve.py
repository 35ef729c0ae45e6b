"""GPU tests of the request server (continuous batching over two drivers):
every served result equals the same circuit compiled alone, bit for bit,
whatever it was batched with; failures stay with their own request; tickets,
time-outs and concurrent submitters behave as documented."""

import random
import sys
import threading
import time

import pytest

import oracle
from paper_2604_16613_amd import Driver, GpError, Server
from paper_2604_16613_amd import _gp
from workloads import iceberg_surface_batch, log_uniform_rates, rotated_surface_code_memory

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def same(a, b, label):
    ea, eb = a.edges(), b.edges()
    assert set(ea) == set(eb), f"{label}: hyperedge sets differ"
    for k in ea:
        assert ea[k] == eb[k], f"{label}: {k} {ea[k]!r} != {eb[k]!r}"


@pytest.fixture(scope="module")
def branches():
    return [c.text for c in iceberg_surface_batch(5, n_branches=40, seed=300)]


def test_served_results_equal_compiles_alone(branches):
    say("case served vs alone")
    with Server.for_circuits(branches, max_batch=12) as srv, Driver.from_batch(branches) as alone:
        rng = random.Random(5)
        tickets = []
        for t in branches:
            tickets.append(srv.submit(t))
            time.sleep(rng.random() * 2e-4)
        got = [srv.wait(k) for k in tickets]
        st = srv.stats()
        assert st["requests"] == len(branches) and 1 <= st["max_batch"] <= 12
        for i, (hg, lat) in enumerate(got):
            assert lat > 0
            same(hg, alone.compile_hypergraph(branches[i]), f"request {i}")
        for i in (0, 17, 39):
            ref = oracle.run(branches[i])
            e = got[i][0].edges()
            assert set(e) == set(ref.edges())
            for k, q in ref.edges().items():
                assert abs(e[k] - q) <= 1e-12 * q


def test_served_rates_and_concurrent_submitters():
    say("case served rates, threads")
    c = rotated_surface_code_memory(5, 5)
    rate_sets = [log_uniform_rates(c.n_channels, s) for s in range(24)]
    results = {}

    with Server.for_circuits([c.text] * 6) as srv, Driver.from_circuit(c.text) as alone:
        def submitter(lo, hi):
            for s in range(lo, hi):
                results[s] = srv.submit(c.text, rate_sets[s])

        th = [threading.Thread(target=submitter, args=(k * 6, k * 6 + 6)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for s, ticket in results.items():
            hg, _ = srv.wait(ticket)
            same(hg, alone.compile_hypergraph(c.text, rate_sets[s]), f"rates {s}")


def test_served_errors_stay_with_their_request(branches):
    say("case served errors")
    bad_parse = "CX 0\n"
    gauge = "R 0\nH 0\nM 0\nDETECTOR rec[-1]\n"
    too_big = rotated_surface_code_memory(9, 9).text
    with Server.for_circuits(branches[:4], max_batch=4) as srv, Driver.from_batch(branches[:4]) as alone:
        plan = [branches[0], bad_parse, branches[1], gauge, too_big, branches[2], branches[3]]
        tickets = [srv.submit(t) for t in plan]
        codes = {1: -2, 3: -5, 4: -4}
        for i, t in enumerate(tickets):
            if i in codes:
                with pytest.raises(GpError) as e:
                    srv.wait(t)
                assert e.value.code == codes[i], (i, e.value)
            else:
                hg, _ = srv.wait(t)
                same(hg, alone.compile_hypergraph(plan[i]), f"good request {i}")


def test_tickets_and_timeouts(branches):
    say("case tickets")
    with Server.for_circuits(branches[:2], max_batch=2) as srv:
        t = srv.submit(branches[0])
        try:
            srv.wait(t, timeout_us=0)
        except GpError as e:
            assert e.code == -10
            srv.wait(t)
        with pytest.raises(GpError) as e:
            srv.wait(t)
        assert e.value.code == -1
        with pytest.raises(GpError) as e:
            srv.wait(12345)
        assert e.value.code == -1
        # results nobody collects are freed with the server
        srv.submit(branches[1])


def test_admission_refuses_past_its_limits(branches):
    """Backpressure: past the limit of live (uncollected) requests, or of the
    host bytes they hold, a submission fails at once with GP_E_BUSY and is
    not queued; collecting a result frees room; a request is always admitted
    when nothing is live."""
    say("case admission")
    with Server.for_circuits(branches, max_batch=4) as srv, Driver.from_batch(branches) as alone:
        with pytest.raises(GpError) as e:
            srv.set_admission(0, 1 << 20)
        assert e.value.code == -1
        srv.set_admission(2, 1 << 30)
        a = srv.submit(branches[0])
        b = srv.submit(branches[1])
        with pytest.raises(GpError) as e:
            srv.submit(branches[2])
        assert e.value.code == -11 and e.value.name == "GP_E_BUSY"
        hg, _ = srv.wait(a)
        same(hg, alone.compile_hypergraph(branches[0]), "admitted request a")
        c = srv.submit(branches[2])
        for t, k in ((b, 1), (c, 2)):
            hg, _ = srv.wait(t)
            same(hg, alone.compile_hypergraph(branches[k]), f"request {k}")
        # bytes: the first request is admitted alone even over the limit, the
        # next one waits until it is collected
        srv.set_admission(100, len(branches[3]) // 2)
        d = srv.submit(branches[3])
        with pytest.raises(GpError) as e:
            srv.submit(branches[4])
        assert e.value.code == -11
        srv.wait(d)
        f = srv.submit(branches[4])
        hg, _ = srv.wait(f)
        same(hg, alone.compile_hypergraph(branches[4]), "request after the byte limit")
        assert srv.stats()["requests"] == 5


@pytest.mark.timeout(300)
def test_served_d10_workload_against_the_oracle():
    """The served workload of the benchmark (outer distance 10 branches,
    seeds 1000..), submitted back to back so that they batch: every result
    equals the branch compiled alone bit for bit, and two of them the oracle
    to 1e-12."""
    say("case served d10")
    texts = [c.text for c in iceberg_surface_batch(10, n_branches=8, seed=1000)]
    with Server.for_circuits(texts, max_batch=16) as srv, Driver.from_batch(texts) as alone:
        tickets = [srv.submit(t) for t in texts]
        got = [srv.wait(k)[0] for k in tickets]
        for i, hg in enumerate(got):
            same(hg, alone.compile_hypergraph(texts[i]), f"served d10 request {i}")
    for i in (0, 7):
        say(f"case served d10: request {i} against the oracle")
        ref = oracle.run(texts[i]).edges()
        e = got[i].edges()
        assert set(e) == set(ref)
        for k, q in ref.items():
            assert abs(e[k] - q) <= 1e-12 * q
