"""Readout on the device: keys as x/z words, <P> and every p_{k,0} from a device statevector
(against dense statevectors built from the gates' unitaries), the batched GF(2) path, and the
per-generator comparison of two results (against the host's)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_2505_03307_amd import workloads as W
from paper_2505_03307_amd.qimax import QimaxError, Simulator
from paper_2505_03307_amd.workloads import Gate

import _dense as D
from _compare import fp32_relative_errors
from _keys import LETTER, xz_to_index

pytestmark = pytest.mark.gpu


def say(*a):
    print("[readout]", *a, file=sys.stderr, flush=True)


def test_generators_xz_matches_index_words():
    for c in (W.c1_random_hst(seed=1), W.random_circuit(31, 40, 300, p_nonclifford=0.05),
              W.c3_hea(seed=2, n=6, layers=2, eps=0.0)):
        say("xz", c.name)
        with Simulator(c.n, precision=32 if c.n == 6 else 64) as s:
            s.run(c)
            off, keys, w = s.generators()
            off2, x, z, w2 = s.generators_xz()
        assert np.array_equal(off, off2)
        assert np.array_equal(xz_to_index(x, z, c.n), keys)
        assert np.array_equal(w, w2)


@pytest.mark.parametrize("which", ["hea12_fp32", "random24", "random40"])
def test_exported_generators_at_size(which):
    """Results large enough to leave through the device-side export (64 Ki terms or more;
    the ansatz in more than one chunk through the image buffers), with 32-, 64- and 128-bit
    keys: the index words and FP64 weights agree with the separate x/z readout, and the
    ansatz count with its closed form."""
    c, prec = {"hea12_fp32": lambda: (W.c3_hea(seed=3, n=12, layers=2, eps=0.0), 32),
               "random24": lambda: (W.c2_clifford_rz(seed=4, n=24, depth=60, n_rz=24), 64),
               "random40": lambda: (W.c2_clifford_rz(seed=3, n=40, depth=60, n_rz=30), 64)}[which]()
    say("export", c.name)
    with Simulator(c.n, precision=prec) as s:
        s.run(c)
        off, keys, w = s.generators()
        off2, x, z, w2 = s.generators_xz()
    assert keys.shape[0] >= 1 << 16
    if which == "hea12_fp32":
        assert keys.shape[0] == 3 ** 13 + 9 * 12 - 21
    assert np.array_equal(off, off2)
    assert np.array_equal(xz_to_index(x, z, c.n), keys)
    assert np.array_equal(w, w2)
    for j in range(c.n):  # ascending keys within every generator
        kj = keys[int(off[j]):int(off[j + 1])]
        if c.n > 32:
            assert np.all((kj[1:, 1] > kj[:-1, 1]) | ((kj[1:, 1] == kj[:-1, 1]) & (kj[1:, 0] > kj[:-1, 0])))
        else:
            assert np.all(kj[1:, 0] > kj[:-1, 0])


def _want(psi, n, p):
    return float(np.real(np.vdot(psi, D.apply_pauli_state(psi.copy(), n, [LETTER.index(ch) for ch in p]))))


@pytest.mark.parametrize("which", ["hst8", "random6", "hea10", "random12"])
def test_device_expectations_match_statevector(which):
    c = {"hst8": lambda: W.c1_random_hst(seed=6),
         "random6": lambda: W.random_circuit(22, 6, 80, p_nonclifford=0.3),
         "hea10": lambda: W.c3_hea(seed=5, n=10, layers=2, eps=0.0),
         "random12": lambda: W.random_circuit(23, 12, 150, p_nonclifford=0.2)}[which]()
    say("expect", c.name)
    rng = np.random.default_rng(5)
    psi = D.statevector(c)
    n = c.n
    probes = ["".join(LETTER[int(d)] for d in rng.integers(0, 4, n)) for _ in range(8)]
    probes += ["".join("Z" if q == k else "I" for q in range(n)) for k in range(n)]
    with Simulator(n) as s:
        s.run(c)
        got = s.expect_many(probes)
        p0 = s.prob_zero_all()
        one = s.expect(probes[0])
    want = np.array([_want(psi, n, p) for p in probes])
    assert np.max(np.abs(got - want)) < 1e-9
    assert abs(one - want[0]) < 1e-9
    pz = np.array([float(np.sum(np.abs(psi.reshape([2] * n).take(0, axis=k)) ** 2)) for k in range(n)])
    assert np.max(np.abs(p0 - pz)) < 1e-9


def test_clifford_batched_gf2_path():
    gates = [Gate.H, Gate.S, Gate.SDG, Gate.SX, Gate.X, Gate.Y, Gate.Z, Gate.CX, Gate.CZ]
    c = W.random_circuit(41, 10, 300, gates=gates)
    psi = D.statevector(c)
    rng = np.random.default_rng(9)
    with Simulator(c.n) as s:
        s.run(c)
        off, keys, w = s.generators()
        probes = ["".join(LETTER[int(d)] for d in rng.integers(0, 4, c.n)) for _ in range(20)]
        for j in range(c.n):  # the generators' own strings: <G_j> = sign
            k = int(keys[int(off[j]), 0])
            probes.append("".join(LETTER[(k >> (2 * (c.n - 1 - q))) & 3] for q in range(c.n)))
        got = s.expect_many(probes)
        p0 = s.prob_zero_all()
    want = np.array([_want(psi, c.n, p) for p in probes])
    assert np.max(np.abs(got - want)) < 1e-12
    pz = np.array([float(np.sum(np.abs(psi.reshape([2] * c.n).take(0, axis=k)) ** 2)) for k in range(c.n)])
    assert np.max(np.abs(p0 - pz)) < 1e-12


def test_device_expectation_n22():
    """A non-Clifford state of 22 qubits (4M amplitudes), a few Rz gates in a Clifford circuit."""
    c = W.c2_clifford_rz(seed=3, n=22, depth=30, n_rz=4)
    psi = D.statevector(c)
    rng = np.random.default_rng(2)
    probes = ["".join(LETTER[int(d)] for d in rng.integers(0, 4, c.n)) for _ in range(4)]
    with Simulator(c.n) as s:
        s.run(c)
        off, keys, w = s.generators()
        for j in range(3):  # strings with large expectation values: the generators' leading terms
            k = int(keys[int(off[j]) + int(np.argmax(np.abs(w[int(off[j]):int(off[j + 1])]))), 0])
            probes.append("".join(LETTER[(k >> (2 * (c.n - 1 - q))) & 3] for q in range(c.n)))
        got = s.expect_many(probes)
    want = np.array([_want(psi, c.n, p) for p in probes])
    say("n22 expectations", got.tolist())
    assert np.max(np.abs(got - want)) < 1e-9


def test_expect_rejects_too_large():
    c = W.c2_clifford_rz(seed=1, n=33, depth=10, n_rz=3)
    with Simulator(c.n) as s:
        s.run(c)
        with pytest.raises(QimaxError, match="ETOOLARGE"):
            s.expect("Z" * c.n)


def test_compare_matches_host():
    c = W.c3_hea(seed=4, n=10, layers=2, eps=1e-9)
    with Simulator(c.n, prune_eps=c.eps) as s64, Simulator(c.n, precision=32, prune_eps=c.eps) as s32:
        s64.run(c)
        s32.run(c)
        d, r, k = s32.compare(s64, tau=1e-6)
        rel_host, _ = fp32_relative_errors(s32.generators(), s64.generators())
        g64 = s64.generators()
        d0, r0, k0 = s64.compare(s64, tau=1e-6)
    assert np.allclose(d / r, rel_host, rtol=1e-6, atol=1e-13)
    nrm = np.array([np.linalg.norm(g64[2][int(g64[0][j]):int(g64[0][j + 1])]) for j in range(c.n)])
    assert np.allclose(r, nrm, rtol=1e-12)
    assert np.all(d0 == 0.0) and np.all(k0 == 0)
