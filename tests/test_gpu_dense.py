"""Dense accumulation instead of the sort (the v2-style fixed-size weight array, one slot per
Pauli string of a generator, 4^n slots, n <= 12) through the C ABI: against the oracle and the
sort path within the FP64 tolerance, deterministic from run to run (fixed-point sums commute),
FP32 within 5e-6 of FP64, the prune threshold, and the autotuner's choice between the two."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2505_03307_amd import workloads as W
from paper_2505_03307_amd.qimax import Simulator

from _compare import compare_fp64, fp32_relative_errors, oracle_arrays

pytestmark = pytest.mark.gpu


def say(*a):
    print("[dense]", *a, file=sys.stderr, flush=True)


def _run(c, monkeypatch, mode, **kw):
    if mode is None:
        monkeypatch.delenv("QIMAX_DENSE", raising=False)
    else:
        monkeypatch.setenv("QIMAX_DENSE", mode)
    with Simulator(c.n, prune_eps=c.eps, **kw) as s:
        s.run(c)
        g = s.generators()
        st = s.stats()
    return g, st


@pytest.mark.parametrize("case", ["hea8", "random10", "c1", "hea10_eps"])
def test_dense_matches_oracle_and_sort(case, monkeypatch):
    c = {"hea8": lambda: W.c3_hea(seed=3, n=8, layers=2, eps=0.0),
         "random10": lambda: W.random_layered(21, 10, layers=2, gates_per_layer=120, p_nonclifford=0.25),
         "c1": lambda: W.c1_random_hst(seed=4),
         "hea10_eps": lambda: W.c3_hea(seed=5, n=10, layers=2, eps=1e-4)}[case]()
    say("case", c.name)
    dense, _ = _run(c, monkeypatch, "1")
    again, _ = _run(c, monkeypatch, "1")
    for x, y in zip(dense, again):  # integer sums: the same result every run
        assert np.array_equal(x, y)
    ref = oracle_arrays(oracle.propagate(c), c.n)
    compare_fp64(dense, ref, label=f"dense {c.name}")
    srt, _ = _run(c, monkeypatch, None)
    compare_fp64(dense, srt, tau=1e-12, tol=1e-13, label=f"dense vs sort {c.name}")
    if c.eps > 0:
        assert np.all(np.abs(dense[2]) > c.eps)


def test_dense_fp32(monkeypatch):
    c = W.c3_hea(seed=7, n=9, layers=2, eps=0.0)
    g32, _ = _run(c, monkeypatch, "1", precision=32)
    g64, _ = _run(c, monkeypatch, None)
    rel, mx = fp32_relative_errors(g32, g64)
    say("dense fp32 rel", float(rel.max()))
    assert float(rel.max()) <= 5e-6


def test_autotuner_chooses_between_dense_and_sort(monkeypatch):
    c = W.random_layered(30, 9, layers=2, gates_per_layer=150, p_nonclifford=0.3)
    monkeypatch.setenv("QIMAX_DENSE", "auto")
    monkeypatch.setenv("QIMAX_SMALL_ROUNDS", "0")
    with Simulator(c.n) as s:
        outs = []
        for _ in range(13):
            s.reset()
            s.run(c)
            outs.append(s.generators())
        st = s.stats()
    say("tuned classes", st["tuned_classes"])
    assert st["tuned_classes"] > 0
    ref = oracle_arrays(oracle.propagate(c), c.n)
    for g in outs:
        compare_fp64(g, ref, label="auto")
