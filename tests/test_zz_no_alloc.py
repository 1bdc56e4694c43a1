"""qimax_compare_noalloc (the comparison for callers that cannot allocate device memory)
against qimax_compare on the same contexts: two calls in a row, the second on smaller
inputs, through the C ABI; plus its refusal of deferred operators."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2505_03307_amd import workloads as W
from paper_2505_03307_amd.qimax import QimaxError, Simulator

pytestmark = pytest.mark.gpu


def say(*a):
    print("[no-alloc]", *a, file=sys.stderr, flush=True)


def _pair(c):
    s64 = Simulator(c.n, prune_eps=c.eps)
    s32 = Simulator(c.n, precision=32, prune_eps=c.eps)
    for s in (s64, s32):
        s.run(c)
        s.flush()
    return s32, s64


def test_noalloc_equals_compare_twice_smaller_second():
    big = W.c3_hea(seed=4, n=12, layers=2, eps=1e-9)                  # 1.6M terms
    small = W.c2_clifford_rz(seed=1, n=12, depth=40, n_rz=8)           # a few hundred terms
    for c in (big, small):
        say("case", c.name)
        s32, s64 = _pair(c)
        want = s32.compare(s64, tau=1e-6)
        got = s32.compare(s64, tau=1e-6, no_alloc=True)
        s32.close()
        s64.close()
        d0, r0, k0 = want
        d1, r1, k1 = got
        # the per-tile sums reach the accumulators in any order: equal up to rounding
        assert np.allclose(d1, d0, rtol=1e-12, atol=1e-300)
        assert np.allclose(r1, r0, rtol=1e-12, atol=0.0)
        assert np.array_equal(k1, k0)
        assert float(np.max(d1 / r1)) <= 5e-6


def test_noalloc_refuses_deferred_operators():
    c = W.c2_clifford_rz(seed=2, n=10, depth=20, n_rz=3)
    # a call of Clifford gates only: the library keeps its operators back until readout or flush
    cl = W.random_circuit(5, 10, 40, gates=[W.Gate.H, W.Gate.S, W.Gate.CX])
    with Simulator(c.n) as a, Simulator(c.n, precision=32) as b:
        for s in (a, b):
            s.run(c)
            s.run(cl)
        with pytest.raises(QimaxError, match="ESTATE"):
            a.compare(b, no_alloc=True)
        a.flush()
        b.flush()
        d, r, k = a.compare(b, no_alloc=True)
        d0, r0, k0 = a.compare(b)
        assert np.allclose(d, d0, rtol=1e-12, atol=1e-300) and np.array_equal(k, k0)
        assert np.all(r > 0)
