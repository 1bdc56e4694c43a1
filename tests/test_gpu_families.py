"""The paper's benchmark families (Sec. V) on the GPU through the C ABI: GHZ and graph states
(stabilizer rank 1, equal to the tableau at sizes the oracle cannot reach quickly), parity of
all three families with the oracle at small #Repeats, closed-form counts of |XYZ + chain>, and
the grouping of a circuit of millions of gates into one U and one V run per layer."""
from __future__ import annotations

import sys
import time

import numpy as np
import pytest

import oracle
from paper_2505_03307_amd import workloads as W
from paper_2505_03307_amd.qimax import Simulator

from _compare import compare_fp64, oracle_arrays
from _keys import xz_to_index
from _tableau import Tableau

pytestmark = pytest.mark.gpu


def say(*a):
    print("[families]", *a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("case", ["ghz20", "graph24", "xyz8"])
def test_families_match_oracle(case):
    c = {"ghz20": lambda: W.ghz(20, repeats=50, layers=2),
         "graph24": lambda: W.graph_state(5, 24, repeats=20, layers=2),
         "xyz8": lambda: W.xyz_chain(seed=3, n=8, repeats=100, layers=2)}[case]()
    say("case", c.name, "m", c.m)
    with Simulator(c.n, prune_eps=c.eps) as s:
        s.run(c)
        g = s.generators()
    o = oracle.propagate(c, threads=16)
    compare_fp64(g, oracle_arrays(o, c.n), raw_exact=case != "xyz8", tol=1e-11, label=c.name)


@pytest.mark.parametrize("family,n,reps", [("ghz", 64, 1000), ("graph", 48, 200), ("ghz", 33, 5000)])
def test_rank_one_at_scale(family, n, reps):
    """Every generator a single Pauli string of weight +-1 (rank 1), equal to the tableau row."""
    c = W.ghz(n, repeats=reps) if family == "ghz" else W.graph_state(11, n, repeats=reps)
    say("rank one", c.name, "m", c.m)
    with Simulator(n) as s:
        s.run(c)
        off, keys, w = s.generators()
    assert np.diff(off.astype(np.int64)).tolist() == [1] * n
    assert np.all(np.abs(w) == 1.0)
    rows = Tableau(n).run(c).rows()
    for j in range(n):
        x, z, sign = rows[j]
        want = xz_to_index(np.array([x], dtype=np.uint64), np.array([z], dtype=np.uint64), n)[0]
        assert np.array_equal(keys[j], want)
        assert float(w[j]) == sign


@pytest.mark.parametrize("n,reps", [(12, 1000), (14, 10000)])
def test_xyz_chain_counts(n, reps):
    """Closed-form counts at any #Repeats: 3n after one layer, 3^(n+1) + 9n - 21 after two,
    and the norm of every generator 1."""
    c = W.xyz_chain(seed=n, n=n, repeats=reps, layers=2)
    say("xyz counts", c.name, "m", c.m)
    with Simulator(n) as s:
        s.run(c.prefix_layers(1))
        assert s.num_terms() == 3 * n
        s.apply_circuit(c.layer(1))
        off, keys, w = s.generators()
    assert int(off[-1]) == 3 ** (n + 1) + 9 * n - 21
    for j in range(n):
        ww = w[int(off[j]):int(off[j + 1])]
        assert abs(float(np.sum(ww * ww)) - 1.0) < 1e-10


def test_grouping_of_a_million_gate_layer():
    """#Repeats = 10^5 on 15 qubits (4.5 million gates per layer): one U run and one V run;
    each wire's composed transfer matrix equals the product of its 300,000 gate matrices, and
    the grouping stays fast."""
    c = W.xyz_chain(seed=1, n=15, repeats=100_000, layers=1)
    with Simulator(c.n) as s:
        s.group(W.xyz_chain(seed=2, n=15, repeats=10, layers=1))  # warm-up
        t0 = time.perf_counter()
        ops, K, Kp = s.group(c)
        dt = time.perf_counter() - t0
    say("grouping of", c.m, "gates:", round(dt * 1e3, 1), "ms")
    assert (K, Kp) == (1, 1)
    assert len(ops) == 15 + 14
    for q in (0, 7, 14):
        sel = np.flatnonzero((c.q0 == q) & (c.gate != W.Gate.CX))
        M = np.eye(4)
        for i in sel.tolist():
            M = oracle.gate_ptm(int(c.gate[i]), float(c.theta[i])) @ M
        qs, R = ops[q]
        assert qs == (q,)
        assert np.max(np.abs(R - M)) < 1e-9
    assert dt < 5.0
