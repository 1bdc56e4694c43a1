"""A recorded step replayed as one HIP graph (qimax_graph_record / qimax_graph_launch),
through the C ABI: every replay leaves the same generators, bit for bit, as the eager step
(with eager work and synchronisations between the replays), counts the same term updates,
and is refused once the context's buffers have changed."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2505_03307_amd import workloads as W
from paper_2505_03307_amd.qimax import QimaxError, Simulator

pytestmark = pytest.mark.gpu


def say(*a):
    print("[graph]", *a, file=sys.stderr, flush=True)


def _eager(s, c):
    s.reset()
    s.run(c)
    s.flush()
    return s.generators()


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("case", ["clifford_rz", "ansatz", "layered_fp32"])
def test_replay_equals_eager(case):
    c = {"clifford_rz": lambda: W.c2_clifford_rz(seed=3, n=24, depth=100, n_rz=18),
         "ansatz": lambda: W.c3_hea(seed=2, n=10, layers=2, eps=1e-9),
         "layered_fp32": lambda: W.random_layered(4, 12, layers=3, gates_per_layer=80, p_nonclifford=0.1)}[case]()
    say("case", case, c.name)
    prec = 32 if case == "layered_fp32" else 64
    with Simulator(c.n, precision=prec, prune_eps=c.eps) as s:
        # eager steps until the autotuner has timed every candidate of the step's size classes
        # (an exploring step may allocate buffers the recording did not use, and a replay is
        # refused once the buffers change), which also grows every buffer the step needs
        for _ in range(11):
            want = _eager(s, c)
        u0 = s.stats()["term_updates"]
        want2 = _eager(s, c)
        step_upd = s.stats()["term_updates"] - u0
        assert _same(want, want2)
        g = s.record_step(c)
        try:
            assert _same(s.generators(), want)  # the recording run computed the step
            for rep in range(3):
                u1 = s.stats()["term_updates"]
                g.launch()
                s.sync()
                assert s.stats()["term_updates"] - u1 == step_upd
                got = s.generators()
                assert _same(got, want), f"replay {rep} differs"
                # eager work between replays: the same step again (no buffer changes)
                assert _same(_eager(s, c), want)
        finally:
            g.close()


def test_replay_refused_after_buffers_change():
    small = W.c2_clifford_rz(seed=1, n=16, depth=40, n_rz=6)
    big = W.c2_clifford_rz(seed=2, n=16, depth=120, n_rz=30)
    with Simulator(16) as s:
        want = _eager(s, small)
        g = s.record_step(small)
        try:
            g.launch()
            assert _same(s.generators(), want)
            _eager(s, big)  # grows the buffers
            with pytest.raises(QimaxError, match="ESTATE"):
                g.launch()
        finally:
            g.close()
    # a fresh context: the record call sizes its buffers with a first run of the step
    with Simulator(16) as ref:
        want_big = _eager(ref, big)
    with Simulator(16) as s2:
        g2 = s2.record_step(big)
        try:
            assert _same(s2.generators(), want_big)
            g2.launch()
            assert _same(s2.generators(), want_big)
        finally:
            g2.close()
