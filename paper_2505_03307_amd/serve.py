"""Serving loop: circuits arrive over time and are propagated with continuous batching.

Requests (workloads.Circuit) arrive at given times. The server keeps one batch
(qimax_batch) on the GPU; between steps it admits arrived requests in arrival order while
their predicted device footprint fits the memory budget, runs one step (every admitted
circuit advances one pass, all in one set of launches), and hands finished results back
with their latency (arrival -> result on the host). The sequential reference serves the
same trace one circuit at a time on a single-circuit context.

The footprint predictor follows the paper's feasibility bound (Sec. IV: the number of
Pauli strings a run can hold is limited by memory / (bytes per string)): predicted bytes =
peak images in flight x bytes per image + terms x bytes per term + 1 MiB of buffers of
fixed size, with the peak image
count taken from the closed form of the hardware-efficient ansatz when the circuit is of
that family (3n terms after one layer; 3^(n+1) + 9n - 21 after two, from 4*3^n + 9n - 12
images), and otherwise from the bound min(4^n - 1, 2^(#non-Clifford gates)) per generator.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import workloads as W
from .qimax import Batch, Simulator

_NON_CLIFFORD = W.NON_CLIFFORD


def _hea_layers(c: W.Circuit):
    """Number of layers if c is the Rx/Ry/Rz + CX-ladder ansatz, else None."""
    n = c.n
    per = 3 * n + (n - 1)
    if c.m == 0 or c.m % per:
        return None
    L = c.m // per
    g = c.gate.reshape(L, per)
    want = np.array([W.Gate.RX, W.Gate.RY, W.Gate.RZ] * n + [W.Gate.CX] * (n - 1), dtype=np.uint8)
    return L if np.all(g == want[None, :]) else None


def predict_terms(c: W.Circuit):
    """(peak images of one pass, final terms), upper bounds, for admission."""
    n = c.n
    L = _hea_layers(c)
    if L == 1:
        return 3 * n, 3 * n
    if L == 2:
        return 4 * 3 ** n + 9 * n - 12, 3 ** (n + 1) + 9 * n - 21
    k = int(np.isin(c.gate, np.array(_NON_CLIFFORD, dtype=np.uint8)).sum())
    per_gen = min(4 ** n - 1, 2 ** min(k, 62))
    return 3 * n * per_gen, n * per_gen


def key_class(n: int) -> int:
    """Qubit limit of the key class a circuit of n qubits needs (16, 32 or 64)."""
    return 16 if n <= 16 else (32 if n <= 32 else 64)


_FIXED_BYTES = 1 << 20


def predict_bytes(c: W.Circuit, precision: int = 32, batch_max_n: int | None = None) -> int:
    cls = batch_max_n or key_class(c.n)
    kb = 4 if cls <= 16 else (8 if cls <= 32 else 16)
    wb = 8 if precision == 64 else 4
    img, terms = predict_terms(c)
    # the library's buffers for a round of `img` images (each grown with 25% headroom): two
    # key/weight image buffers for the sort, and three term arrays sized by the images (the
    # generators and the two output slots a call alternates between); per input term its A-chain
    # key, sign byte and 8-byte image offset; plus a round's buffers of fixed size (tilings,
    # look-back status words, chain tables, staging: 0.1-0.2 MB for the small ansatz circuits)
    return int(1.25 * (5 * img * (kb + wb) + terms * (kb + 9))) + _FIXED_BYTES


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    terms: int
    updates: int

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Server:
    """Continuous batching over one qimax_batch with admission by predicted memory."""

    def __init__(self, budget_bytes: int, precision: int = 32, max_n: int = 32, keep_results: bool = False,
                 batch=None):
        # batch: anything with submit/step/poll/fetch/circuit_updates/close (default: a qimax_batch)
        self.batch = batch if batch is not None else Batch(precision=precision, max_n=max_n)
        self.precision = precision
        self.max_n = max_n
        self.budget = int(budget_bytes)
        self.in_flight = {}   # batch id -> (rid, arrival, admitted, predicted bytes)
        self.reserved = 0
        self.keep_results = keep_results
        self.outputs = {}

    def close(self):
        self.batch.close()

    def try_admit(self, rid: int, circuit: W.Circuit, arrival: float, now: float) -> bool:
        need = predict_bytes(circuit, self.precision, self.max_n)
        if need > self.budget:
            raise ValueError(f"request {rid} needs {need} bytes, more than the whole budget")
        if self.in_flight and self.reserved + need > self.budget:
            return False
        bid = self.batch.submit(circuit)
        self.in_flight[bid] = (rid, arrival, now, need)
        self.reserved += need
        return True

    def step(self, clock) -> list[Result]:
        if not self.in_flight:
            return []
        self.batch.step()
        out = []
        for bid in self.batch.poll():
            rid, arrival, admitted, need = self.in_flight.pop(bid)
            updates = self.batch.circuit_updates(bid)
            res = self.batch.fetch(bid)
            self.reserved -= need
            if self.keep_results:
                self.outputs[rid] = res
            out.append(Result(rid, arrival, admitted, clock(), int(res[0][-1]), updates))
        return out


def serve_trace(circuits, arrivals, budget_bytes: int, precision: int = 32, keep_results: bool = False,
                batch=None):
    """Serve the trace in real time with continuous batching. Returns (results, server)."""
    order = np.argsort(arrivals, kind="stable")
    srv = Server(budget_bytes, precision, max_n=key_class(max(c.n for c in circuits)),
                 keep_results=keep_results, batch=batch)
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0  # noqa: E731
    pending = list(order)
    results = []
    while pending or srv.in_flight:
        now = clock()
        # admit arrived requests in arrival order while their footprint fits
        while pending and arrivals[pending[0]] <= now:
            i = pending[0]
            if not srv.try_admit(int(i), circuits[i], float(arrivals[i]), now):
                break
            pending.pop(0)
        if srv.in_flight:
            results.extend(srv.step(clock))
        elif pending:
            wait = arrivals[pending[0]] - clock()
            if wait > 0:
                time.sleep(min(wait, 0.01))
    return results, srv


def serve_sequential(circuits, arrivals, precision: int = 32, keep_results: bool = False, progress=None):
    """The plain path on the same trace: one circuit at a time, FIFO, in real time.
    progress(n), if given, is called after each result with the number of results so far."""
    order = np.argsort(arrivals, kind="stable")
    t0 = time.perf_counter()
    results, outputs = [], {}
    sims = {}
    for i in order:
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        c = circuits[i]
        start = time.perf_counter() - t0
        key = (c.n, float(c.eps))
        if key not in sims:
            sims[key] = Simulator(c.n, precision=precision, prune_eps=c.eps)
        s = sims[key]
        s.reset()
        u0 = s.stats()["term_updates"]
        s.run(c)
        res = s.generators()
        done = time.perf_counter() - t0
        if keep_results:
            outputs[int(i)] = res
        results.append(Result(int(i), float(arrivals[i]), start, done, int(res[0][-1]),
                              s.stats()["term_updates"] - u0))
        if progress:
            progress(len(results))
    for s in sims.values():
        s.close()
    return results, outputs


def summarize(results, wall: float) -> dict:
    lat = np.array([r.latency for r in results])
    upd = float(sum(r.updates for r in results))
    return {"requests": len(results), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "mean_ms": round(float(lat.mean()) * 1e3, 3), "wall_s": round(wall, 3),
            "requests_per_s": round(len(results) / wall, 2), "term_updates_per_s": round(upd / wall, 1)}


class _Budget:
    """Device bytes reserved by admitted requests, shared by the lanes."""

    def __init__(self, total: int):
        import threading
        self.total = int(total)
        self.used = 0
        self.lock = threading.Lock()

    def try_reserve(self, need: int, force: bool) -> bool:
        with self.lock:
            if force or self.used + need <= self.total:
                self.used += need
                return True
            return False

    def release(self, need: int):
        with self.lock:
            self.used -= need


class SimRunner:
    """Runs one circuit at a time through the single-circuit API, one warm context per
    (n, eps) kept for later requests: the large lane's executor."""

    def __init__(self, precision: int = 32):
        self.precision = precision
        self.sims = {}

    def run(self, c: W.Circuit):
        """(generators, term updates) of circuit c."""
        key = (c.n, float(c.eps))
        if key not in self.sims:
            self.sims[key] = Simulator(c.n, precision=self.precision, prune_eps=c.eps)
        s = self.sims[key]
        s.reset()
        u0 = s.stats()["term_updates"]
        s.run(c)
        res = s.generators()
        return res, s.stats()["term_updates"] - u0

    def close(self):
        for s in self.sims.values():
            s.close()
        self.sims = {}


def serve_trace_lanes(circuits, arrivals, budget_bytes: int, precision: int = 32, split_bytes: int = 256 << 20,
                      large_in_flight: int = 1, keep_results: bool = False, batch_factory=None, progress=None,
                      large_runner=None):
    """Two lanes, each driven by its own host thread on its own HIP stream: requests predicted
    to need less than split_bytes are continuously batched in one lane, so small requests do
    not wait behind the rounds of large ones. The large lane runs its requests one at a time
    through large_runner (an object with run(circuit) -> (generators, updates) and close();
    by default a SimRunner: large requests already fill the device, and the single-circuit API
    plans all of a circuit's rounds in one call) or, when large_runner is None and a
    batch_factory is given, as a second batch with at most large_in_flight requests in
    flight. Admission in arrival order per lane, against one shared memory budget (a lane
    with nothing in flight may always admit its next request). progress(n), if given, is
    called with the number of requests the trace has handed to the lanes (every 100).
    Returns (results, outputs)."""
    import collections
    import threading

    if large_runner is None and batch_factory is None:
        large_runner = SimRunner(precision)

    order = np.argsort(arrivals, kind="stable")
    max_n = key_class(max(c.n for c in circuits))
    budget = _Budget(budget_bytes)
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0  # noqa: E731

    class Lane:
        def __init__(self, cap, runner=None):
            self.cap = cap
            self.runner = runner
            self.batch = None if runner else (batch_factory() if batch_factory else Batch(precision=precision, max_n=max_n))
            self.queue = collections.deque()
            self.cv = threading.Condition()
            self.closed = False
            self.in_flight = {}
            self.results = []
            self.outputs = {}
            self.error = None

    lanes = [Lane(None), Lane(large_in_flight, large_runner)]

    def run_single(lane):
        # one request at a time: wait for the next, reserve its footprint, run it to the end
        while True:
            with lane.cv:
                while not lane.queue and not lane.closed:
                    lane.cv.wait(timeout=0.01)
                if not lane.queue:
                    return
                rid, need = lane.queue.popleft()
            budget.try_reserve(need, force=True)
            adm = clock()
            res, upd = lane.runner.run(circuits[rid])
            budget.release(need)
            if keep_results:
                lane.outputs[rid] = res
            lane.results.append(Result(rid, float(arrivals[rid]), adm, clock(), int(res[0][-1]), upd))

    def work(lane):
        try:
            if lane.runner is not None:
                run_single(lane)
                return
            while True:
                with lane.cv:
                    while not lane.queue and not lane.in_flight and not lane.closed:
                        lane.cv.wait(timeout=0.01)
                    if lane.closed and not lane.queue and not lane.in_flight:
                        return
                    admitted = []
                    while lane.queue:
                        if lane.cap is not None and len(lane.in_flight) + len(admitted) >= lane.cap:
                            break
                        rid, need = lane.queue[0]
                        if not budget.try_reserve(need, force=not lane.in_flight and not admitted):
                            break
                        lane.queue.popleft()
                        admitted.append((rid, need))
                now = clock()
                for rid, need in admitted:
                    bid = lane.batch.submit(circuits[rid])
                    lane.in_flight[bid] = (rid, float(arrivals[rid]), now, need)
                if lane.in_flight:
                    lane.batch.step()
                    for bid in lane.batch.poll():
                        rid, arr, adm, need = lane.in_flight.pop(bid)
                        upd = lane.batch.circuit_updates(bid)
                        res = lane.batch.fetch(bid)
                        budget.release(need)
                        if keep_results:
                            lane.outputs[rid] = res
                        lane.results.append(Result(rid, arr, adm, clock(), int(res[0][-1]), upd))
        except Exception as e:  # surfaced by the caller
            lane.error = e

    threads = [threading.Thread(target=work, args=(ln,), daemon=True) for ln in lanes]
    for t in threads:
        t.start()
    for n_handed, i in enumerate(order, 1):
        wait = arrivals[i] - clock()
        if wait > 0:
            time.sleep(wait)
        if progress and n_handed % 100 == 0:
            progress(n_handed)
        need = predict_bytes(circuits[i], precision, max_n)
        if need > budget.total:
            raise ValueError(f"request {i} needs {need} bytes, more than the whole budget")
        lane = lanes[0] if need < split_bytes else lanes[1]
        with lane.cv:
            lane.queue.append((int(i), need))
            lane.cv.notify()
    for ln in lanes:
        with ln.cv:
            ln.closed = True
            ln.cv.notify()
    for t in threads:
        t.join()
    results, outputs = [], {}
    for ln in lanes:
        if ln.error:
            raise ln.error
        results += ln.results
        outputs.update(ln.outputs)
        if ln.runner is not None:
            ln.runner.close()
        else:
            ln.batch.close()
    return results, outputs
