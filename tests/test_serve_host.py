"""Host logic of the serving loop on the CPU: the footprint predictor against exact counts,
and admission / continuous batching / latency accounting against a fake executor that
propagates with the CPU oracle (no GPU)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2505_03307_amd import serve, workloads as W

from _compare import oracle_arrays


@pytest.mark.parametrize("n", [4, 6, 9])
def test_predictor_matches_ansatz_counts(n):
    for L in (1, 2):
        c = W.c3_hea(seed=n, n=n, layers=L, eps=0.0)
        img, terms = serve.predict_terms(c)
        assert int(oracle.propagate(c).counts().sum()) == terms
        assert img >= terms


def test_predictor_bounds_other_circuits():
    c = W.c2_clifford_rz(seed=2, n=12, depth=40, n_rz=6)
    img, terms = serve.predict_terms(c)
    assert terms >= int(oracle.propagate(c).counts().sum())
    assert serve.predict_bytes(c) > 0


class FakeBatch:
    """Stands in for a qimax_batch: one pass per circuit layer, results from the oracle."""

    def __init__(self):
        self.next = 1
        self.live = {}
        self.finished = []
        self.steps = 0

    def submit(self, c):
        i = self.next
        self.next += 1
        self.live[i] = [c, len(c.layer_end)]
        return i

    def step(self):
        self.steps += 1
        for i in list(self.live):
            self.live[i][1] -= 1
            if self.live[i][1] == 0:
                self.finished.append(i)
        return len(self.live) - len(self.finished)

    def poll(self):
        out, self.finished = self.finished, []
        return out

    def circuit_updates(self, i):
        return 1

    def fetch(self, i):
        c, _ = self.live.pop(i)
        return oracle_arrays(oracle.propagate(c), c.n)

    def close(self):
        pass


def test_admission_respects_the_budget_and_arrival_order():
    circuits, gaps = W.c5_stream(seed=3, count=12, n_range=(4, 6))
    arrivals = np.cumsum(gaps) * 1e-4
    budget = max(serve.predict_bytes(c) for c in circuits) * 2
    fake = FakeBatch()
    results, srv = serve.serve_trace(circuits, arrivals, budget, batch=fake, keep_results=True)
    assert sorted(r.rid for r in results) == list(range(12))
    for r in results:
        assert r.finished >= r.admitted >= r.arrival - 1e-9
        want = oracle_arrays(oracle.propagate(circuits[r.rid]), circuits[r.rid].n)
        for a, b in zip(srv.outputs[r.rid], want):
            assert np.array_equal(a, b)
    # admission happened in arrival order: admission times never decrease along the trace
    by_rid = {r.rid: r for r in results}
    adm = [by_rid[i].admitted for i in np.argsort(arrivals, kind="stable")]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    assert srv.reserved == 0


def test_oversized_request_is_rejected():
    c = W.c3_hea(seed=1, n=8, layers=2)
    srv = serve.Server(budget_bytes=100, batch=FakeBatch())
    with pytest.raises(ValueError):
        srv.try_admit(0, c, 0.0, 0.0)


def test_summary():
    rs = [serve.Result(i, 0.0, 0.0, 0.001 * (i + 1), 10, 5) for i in range(100)]
    s = serve.summarize(rs, 1.0)
    assert s["requests"] == 100 and abs(s["p50_ms"] - 50.5) < 1e-9 and s["p99_ms"] > s["p50_ms"]


def test_two_lane_server_with_fake_executors():
    circuits, gaps = W.c5_stream(seed=4, count=16, n_range=(4, 7))
    arrivals = np.cumsum(gaps) * 1e-4
    results, outputs = serve.serve_trace_lanes(circuits, arrivals, budget_bytes=10 ** 12, split_bytes=20000,
                                               keep_results=True, batch_factory=FakeBatch)
    assert sorted(r.rid for r in results) == list(range(16))
    for r in results:
        assert r.finished >= r.admitted >= r.arrival - 1e-9
        want = oracle_arrays(oracle.propagate(circuits[r.rid]), circuits[r.rid].n)
        for a, b in zip(outputs[r.rid], want):
            assert np.array_equal(a, b)


class FakeRunner:
    """Stands in for the large lane's single-circuit executor: results from the oracle."""

    def __init__(self):
        self.ran = []
        self.closed = False

    def run(self, c):
        self.ran.append(c.name)
        return oracle_arrays(oracle.propagate(c), c.n), 1

    def close(self):
        self.closed = True


def test_two_lane_server_with_a_single_circuit_large_lane():
    circuits, gaps = W.c5_stream(seed=6, count=16, n_range=(4, 7))
    arrivals = np.cumsum(gaps) * 1e-4
    cls = serve.key_class(max(c.n for c in circuits))
    need = sorted(serve.predict_bytes(c, 32, cls) for c in circuits)
    split = need[len(need) // 2]  # about half of the requests in each lane
    runner = FakeRunner()
    results, outputs = serve.serve_trace_lanes(circuits, arrivals, budget_bytes=10 ** 12, split_bytes=split,
                                               keep_results=True, batch_factory=FakeBatch, large_runner=runner)
    assert sorted(r.rid for r in results) == list(range(16))
    large = [i for i, c in enumerate(circuits) if serve.predict_bytes(c, 32, cls) >= split]
    assert large and len(large) < 16  # both lanes take part
    assert sorted(runner.ran) == sorted(circuits[i].name for i in large) and runner.closed
    for r in results:
        assert r.finished >= r.admitted >= r.arrival - 1e-9
        want = oracle_arrays(oracle.propagate(circuits[r.rid]), circuits[r.rid].n)
        for a, b in zip(outputs[r.rid], want):
            assert np.array_equal(a, b)
    # the large lane ran its requests one at a time, in arrival order
    big = sorted((r for r in results if r.rid in large), key=lambda r: r.admitted)
    assert [r.rid for r in big] == sorted(large, key=lambda i: (arrivals[i], i))
    assert all(a.finished <= b.admitted for a, b in zip(big, big[1:]))

