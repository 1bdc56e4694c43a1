"""Term updates counted by the library (qimax_stats.term_updates) against their definition
(tests/_updates.py: one output image of one grouped operator, each group once), on circuits
where the pass planner splits Clifford groups around the expanding operator."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2505_03307_amd import workloads as W
from paper_2505_03307_amd.qimax import Simulator
from _updates import definition_updates

pytestmark = pytest.mark.gpu


def say(*a):
    print("[counts]", *a, file=sys.stderr, flush=True)


def library_updates(c):
    with Simulator(c.n, prune_eps=c.eps) as s:
        s.run(c)
        s.generators()  # applies any deferred operators
        return s.generator_updates(), s.stats()["term_updates"]


def _layered_no_t(seed, n, layers, gates_per_layer):
    """A layered random circuit over every gate but T / T^dagger: products of their 1/sqrt(2)
    entries cancel exactly in one summation order and leave a 1e-17 residue in another, which
    changes later term counts (and so the update count) between two correct implementations;
    rotations by random angles do not cancel."""
    gates = [g for g in W.Gate if g not in (W.Gate.T, W.Gate.TDG)]
    c = W.random_circuit(seed, n, layers * gates_per_layer, p_nonclifford=0.1, gates=gates)
    ends = np.linspace(0, c.m, layers + 1).astype(np.int64)[1:]
    return W.Circuit(n, c.gate, c.q0, c.q1, c.theta, np.unique(ends), 0.0, f"layered-no-T(seed={seed},n={n})")


@pytest.mark.parametrize("case", ["c2_small", "c2_mid", "hea8", "layered12", "clifford"])
def test_updates_match_definition(case):
    c = {"c2_small": lambda: W.c2_clifford_rz(seed=2, n=16, depth=60, n_rz=10),
         "c2_mid": lambda: W.c2_clifford_rz(seed=4, n=24, depth=120, n_rz=20),
         "hea8": lambda: W.c3_hea(seed=3, n=8, layers=2, eps=0.0),
         "layered12": lambda: _layered_no_t(7, 12, layers=3, gates_per_layer=60),
         "clifford": lambda: W.random_circuit(8, 10, 200, p_nonclifford=0.0)}[case]()
    say("case", case, c.name)
    per_gen, total = library_updates(c)
    want = definition_updates(c, threads=16)
    assert per_gen.tolist() == want.tolist()
    assert total == int(want.sum())


def test_updates_c2_full_size():
    """The benchmarked n=32 Clifford+Rz workload, seed 0: 1,078,842,236 updates per run."""
    c = W.c2_clifford_rz(seed=0)
    per_gen, total = library_updates(c)
    want = definition_updates(c, threads=16)
    say("c2 full updates", total, int(want.sum()))
    assert per_gen.tolist() == want.tolist()
    assert total == 1_078_842_236
