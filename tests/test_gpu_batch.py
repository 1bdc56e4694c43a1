"""Batches of circuits (one qimax_batch): every result equals the single-circuit result
bit for bit and matches the oracle; circuits can join a running batch."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2505_03307_amd import workloads as W
from paper_2505_03307_amd.qimax import Batch, QimaxError, Simulator

from _compare import compare_fp64, oracle_arrays

pytestmark = pytest.mark.gpu


def say(*a):
    print("[batch]", *a, file=sys.stderr, flush=True)


def mixed_circuits():
    cs = [W.c1_random_hst(s) for s in range(3)]
    cs += [W.c2_clifford_rz(seed=s, n=n, depth=d, n_rz=k) for s, (n, d, k) in enumerate([(16, 60, 10), (24, 80, 14), (32, 120, 18)])]
    cs += [W.c3_hea(seed=s, n=n, layers=2, eps=e) for s, (n, e) in enumerate([(4, 0.0), (7, 1e-3), (9, 1e-9)])]
    cs += [W.random_layered(7, 5, layers=3, gates_per_layer=30)]
    cs += [W.random_circuit(8, 6, 0)]  # empty circuit
    return cs


def alone(c, **kw):
    with Simulator(c.n, prune_eps=c.eps, **kw) as s:
        s.run(c)
        return s.generators()


@pytest.mark.parametrize("precision", [64, 32])
def test_batch_equals_alone_bit_for_bit(precision):
    cs = mixed_circuits()
    say("batch of", len(cs), "precision", precision)
    with Batch(precision=precision) as b:
        ids = [b.submit(c) for c in cs]
        b.run()
        done = set(b.poll())
        assert done == set(ids)
        for c, cid in zip(cs, ids):
            got = b.fetch(cid)
            ref = alone(c, precision=precision)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), c.name


def test_batch_matches_oracle():
    cs = mixed_circuits()
    with Batch() as b:
        ids = [b.submit(c) for c in cs]
        b.run()
        for c, cid in zip(cs, ids):
            compare_fp64(b.fetch(cid), oracle_arrays(oracle.propagate(c), c.n), label=c.name)


def test_circuits_join_a_running_batch():
    cs = mixed_circuits()
    with Batch() as b:
        first = [b.submit(c) for c in cs[:4]]
        b.step()
        b.step()
        later = [b.submit(c) for c in cs[4:]]
        steps = 0
        while b.step():
            steps += 1
            assert steps < 10000
        for c, cid in zip(cs, first + later):
            got = b.fetch(cid)
            ref = alone(c)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), c.name
        info = b.info()
        assert info["active"] == 0 and info["queued"] == 0 and info["terms"] == 0


def test_batch_rejects_bad_circuits():
    with Batch() as b:
        bad = W.random_circuit(1, 40, 10)
        with pytest.raises(QimaxError, match="ETOOLARGE"):
            b.submit(bad)
        c = W.c1_random_hst(0)
        c.q0 = c.q0.copy()
        c.q0[3] = 99
        with pytest.raises(QimaxError, match="EINVAL"):
            b.submit(c)


def test_wide_batch_of_the_n8_to_48_family():
    """Circuits of the 256-circuit batch recipe (n from 8 to 48) in a 64-qubit-class batch:
    every result equals the single-circuit result bit for bit."""
    cs = [c for c in W.c4_batch(count=24, depth_range=(30, 80), rz_range=(3, 10))]
    say("wide batch", [c.n for c in cs])
    with Batch(max_n=64) as b:
        ids = [b.submit(c) for c in cs]
        b.run()
        for c, cid in zip(cs, ids):
            got = b.fetch(cid)
            ref = alone(c)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), c.name


def test_status_buffers_regrown_between_circuits():
    """Circuits of growing size on one reused context: the look-back status buffers grow
    between them (possibly at the same address) and must not keep stale words. The n=26
    circuit of the 256-circuit recipe exposed this."""
    cs = W.c4_batch(count=64)
    for i in (53, 0, 16, 48):
        c = cs[i]
        if c.n > 32:
            continue
        say("regrow", i, c.n)
        with Simulator(c.n) as s:
            for small in (W.c2_clifford_rz(seed=9, n=c.n, depth=20, n_rz=2), c):
                s.reset()
                s.run(small)
            got = s.generators()
        compare_fp64(got, oracle_arrays(oracle.propagate(c), c.n), label=c.name)


def test_served_results_equal_alone():
    """A Poisson trace through the two-lane continuous-batching server: every request's
    generators are bit-identical to the same circuit run alone."""
    from paper_2505_03307_amd import serve
    circuits, gaps = W.c5_stream(seed=5, count=24, n_range=(6, 11))
    arrivals = np.cumsum(gaps) * 2e-3
    results, outputs = serve.serve_trace_lanes(circuits, arrivals, budget_bytes=8 << 30, split_bytes=1 << 20,
                                               keep_results=True)
    assert sorted(r.rid for r in results) == list(range(24))
    for r in results:
        c = circuits[r.rid]
        ref = alone(c, precision=32)
        for x, y in zip(outputs[r.rid], ref):
            assert np.array_equal(x, y), c.name


@pytest.mark.parametrize("variant", [("QIMAX_HOST_TILING", "1"), ("QIMAX_SORT_CLASSIC", "1"),
                                     ("QIMAX_LOCAL_SORT", "0"), ("QIMAX_LOCAL_SORT_M", "0"),
                                     ("QIMAX_LOCAL_SORT_M", "1"), ("QIMAX_XCD_RANGES", "0"),
                                     ("QIMAX_SMALL_ROUNDS", "0"), ("QIMAX_FUSED_EXPAND", "0"),
                                     ("QIMAX_CHUNK_TILE", "2048"), ("QIMAX_CHUNK_TILE", "4096"),
                                     ("QIMAX_DEFER_SPINS", "100000"), ("QIMAX_CLASSIC_PASSES", "1"),
                                     ("QIMAX_SMALL_GROUPS", "0")])
def test_tiling_and_sort_variants_bit_identical(variant, monkeypatch):
    """Image tilings built on the device from the fan-out bound (the default for rounds whose
    bound is small) or on the host after reading the image count back; the classic
    multi-launch sort; every digit by global passes, or the top 0 / 1 digits followed by
    chunk-local sorts (0 makes every segment above a chunk fall back to global passes); small
    rounds (one block per segment) or the general path for them; the count and the expansion
    in one launch or in two; fixed nominal chunks of 2048 or 4096 images; chunks that wait for
    their predecessors' offsets instead of deferring: all are stable sorts of the same images,
    hence identical sums, so the results must agree bit for bit, alone and batched."""
    name, value = variant
    cs = mixed_circuits()
    with Batch(precision=64) as b:
        ids = [b.submit(c) for c in cs]
        b.run()
        ref = [b.fetch(i) for i in ids]
    ref_alone = [alone(c) for c in cs[3:6]]
    monkeypatch.setenv(name, value)
    say("variant", name, value)
    with Batch(precision=64) as b:
        ids = [b.submit(c) for c in cs]
        b.run()
        for c, cid, r in zip(cs, ids, ref):
            for x, y in zip(b.fetch(cid), r):
                assert np.array_equal(x, y), (name, value, c.name)
    for c, r in zip(cs[3:6], ref_alone):
        for x, y in zip(alone(c), r):
            assert np.array_equal(x, y), (name, value, c.name)


def test_chunk_overflow_sorts_again(monkeypatch):
    """With no top-digit pass forced, a segment larger than a chunk cannot be sorted
    chunk-locally: the round is sorted again with global passes (counted in sort_redos) and
    the result equals the oracle's and the default path's."""
    c = W.c2_clifford_rz(seed=3, n=24, depth=150, n_rz=24)  # largest generator: 37,825 terms
    ref = alone(c)
    monkeypatch.setenv("QIMAX_LOCAL_SORT_M", "0")
    with Simulator(c.n, prune_eps=c.eps) as s:
        s.run(c)
        got = s.generators()
        redos = s.stats()["sort_redos"]
    say("redos", redos, "terms", int(got[0][-1]))
    assert redos > 0
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)
    compare_fp64(got, oracle_arrays(oracle.propagate(c), c.n), label=c.name)


def test_autotuner_settles_and_keeps_results(monkeypatch):
    """The sort variant is chosen per size class of rounds from measured times: after a few
    runs of the same circuit every explored class is fixed, and every run gives the same
    generators bit for bit (the variants are the same stable sort). Small rounds (one block
    per segment, no sort variants) are turned off so that this circuit's rounds are tuned."""
    monkeypatch.setenv("QIMAX_SMALL_ROUNDS", "0")
    c = W.c2_clifford_rz(seed=1, n=24, depth=100, n_rz=20)
    with Simulator(c.n, prune_eps=c.eps) as s:
        runs = []
        for _ in range(11):
            s.reset()
            s.run(c)
            runs.append(s.generators())
        st = s.stats()
        tun = s.tuning()
    say("tuned classes", st["tuned_classes"], tun)
    assert st["tuned_classes"] > 0
    # qimax_get_tuning: one entry per class; a fixed class chose its fastest candidate
    fixed = [t for t in tun if t["best"] >= 0]
    assert len(fixed) == st["tuned_classes"]
    for t in fixed:
        assert t["key_bytes"] == 8 and t["weight_bits"] == 64 and t["tried"] >= 3
        assert t["ms"][t["best"]] == min(t["ms"])
    for r in runs[1:]:
        for x, y in zip(r, runs[0]):
            assert np.array_equal(x, y)


def test_batch_with_more_segments_than_a_tiling_block_holds():
    """More than 2048 generators in one batch: the round tilings are then built by a single
    block reading its segment offsets from global memory instead of LDS. Every result equals
    the single-circuit result bit for bit."""
    cs = [W.c2_clifford_rz(seed=100 + i, n=48, depth=12, n_rz=2) for i in range(45)]
    say("segments", sum(c.n for c in cs))
    assert sum(c.n for c in cs) > 2048
    with Batch(max_n=64) as b:
        ids = [b.submit(c) for c in cs]
        b.run()
        for c, cid in zip(cs, ids):
            got = b.fetch(cid)
            ref = alone(c)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), c.name


@pytest.mark.parametrize("case", ["hea12_1", "hea12_2", "hea16_1", "hea14_2", "c2_24"])
def test_predicted_footprint_covers_device_memory(case):
    """The server admits a request by serve.predict_bytes: for circuits of the served family
    (and one Clifford+Rz circuit), the device memory a batch grows by while it runs that one
    request alone stays below the prediction."""
    from paper_2505_03307_amd import serve
    c = {"hea12_1": lambda: W.c3_hea(seed=11, n=12, layers=1),
         "hea12_2": lambda: W.c3_hea(seed=12, n=12, layers=2),
         "hea16_1": lambda: W.c3_hea(seed=13, n=16, layers=1),
         "hea14_2": lambda: W.c3_hea(seed=14, n=14, layers=2),
         "c2_24": lambda: W.c2_clifford_rz(seed=15, n=24, depth=120, n_rz=14)}[case]()
    cls = serve.key_class(c.n)
    with Batch(precision=32, max_n=cls) as b:
        a0 = b.info()["alloc_bytes"]
        b.submit(c)
        b.run()
        peak = b.info()["peak_bytes"]
    need = serve.predict_bytes(c, 32, cls)
    say("footprint", case, "grew", peak - a0, "predicted", need)
    assert peak - a0 <= need


def test_wide_offset_paths_bit_identical(monkeypatch):
    """The count's 64-bit in-tile image offsets (taken by a tile of 2^32 images or more) and
    the expansion's parent search in global memory (taken by a round of 2^31 images or more),
    forced at small sizes with the count and the expansion as separate launches: the same
    images in the same order, hence bit-identical results."""
    cs = mixed_circuits()
    ref = [alone(c) for c in cs]
    monkeypatch.setenv("QIMAX_FUSED_EXPAND", "0")
    monkeypatch.setenv("QIMAX_WIDE_OFFSETS", "1")
    for c, r in zip(cs, ref):
        say("wide offsets", c.name)
        for x, y in zip(alone(c), r):
            assert np.array_equal(x, y), c.name
