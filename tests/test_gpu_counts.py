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


@pytest.mark.parametrize("case", ["c2_small", "c2_mid", "hea8", "layered12", "clifford"])
def test_updates_match_definition(case):
    c = {"c2_small": lambda: W.c2_clifford_rz(seed=2, n=16, depth=60, n_rz=10),
         "c2_mid": lambda: W.c2_clifford_rz(seed=4, n=24, depth=120, n_rz=20),
         "hea8": lambda: W.c3_hea(seed=3, n=8, layers=2, eps=0.0),
         "layered12": lambda: W.random_layered(7, 12, layers=3, gates_per_layer=60, p_nonclifford=0.1),
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
