"""Parity of the HIP path (through the C ABI) with the CPU oracle, plus the library's
edge cases and failure paths. Needs an MI355X and the built library."""
from __future__ import annotations

import math
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2505_03307_amd import workloads as W
from paper_2505_03307_amd.qimax import QimaxError, Simulator
from paper_2505_03307_amd.workloads import Gate

import _dense as D
from _compare import compare_fp64, fp32_contract, fp32_relative_errors, oracle_arrays
from _keys import LETTER, string_to_index

pytestmark = pytest.mark.gpu


def say(*a):
    print("[parity]", *a, file=sys.stderr, flush=True)


def run_gpu(circuit, **kw):
    s = Simulator(circuit.n, prune_eps=circuit.eps, **kw)
    s.run(circuit)
    return s


def run_both(circuit, gens=None, threads=0, **kw):
    say("case", circuit.name, "m", circuit.m, kw)
    s = run_gpu(circuit, **kw)
    g = s.generators()
    o = oracle.propagate(circuit, gens=gens, threads=threads)
    return s, g, oracle_arrays(o, circuit.n)


# ------------------------------------------------------------------------------ init

@pytest.mark.parametrize("n", [1, 5, 16, 17, 32])
def test_initial_generators(n):
    say("init n", n)
    with Simulator(n) as s:
        off, keys, w = s.generators()
    assert off.tolist() == list(range(n + 1))
    assert keys[:, 0].tolist() == [3 * 4 ** (n - 1 - j) for j in range(n)]
    assert w.tolist() == [1.0] * n


# ------------------------------------------------------------------------- parity

@pytest.mark.parametrize("seed", range(4))
def test_c1_every_layer(seed):
    """n=8 {H,S,T}+CX workload, compared after every layer."""
    c = W.c1_random_hst(seed)
    say("c1 every layer seed", seed)
    s = Simulator(c.n)
    for li in range(len(c.layer_end)):
        lay = c.layer(li)
        s.apply_circuit(lay)
        o = oracle.propagate(c.prefix_layers(li + 1))
        compare_fp64(s.generators(), oracle_arrays(o, c.n), label=f"layer {li}")
    s.close()


@pytest.mark.parametrize("seed", range(12))
def test_random_full_gate_set(seed):
    n = 1 + seed
    # (with the two-qubit rotations in the mix, 0.2 would give n = 12 about 1.8e8 terms)
    c = W.random_layered(seed, n, layers=3, gates_per_layer=8 * n, p_nonclifford=0.2 if n <= 9 else 0.1)
    _, g, r = run_both(c)
    compare_fp64(g, r, label=c.name)


@pytest.mark.parametrize("n", [4, 7, 10, 13])
def test_hea_closed_form_and_parity(n):
    c = W.c3_hea(seed=n, n=n, layers=2, eps=0.0)
    s, g, r = run_both(c)
    counts = np.diff(g[0].astype(np.int64)).tolist()
    want = [3 ** n + 3] + [3 ** (n - j) + 3 ** (n + 1 - j) + 9 for j in range(1, n - 1)] + [12]
    assert counts == want
    compare_fp64(g, r, raw_exact=True, label=c.name)


def test_hea_prune_eps():
    c = W.c3_hea(seed=2, n=9, layers=2, eps=1e-3)
    _, g, r = run_both(c)
    assert np.all(np.abs(g[2]) > 1e-3)
    compare_fp64(g, r, label=c.name)


@pytest.mark.parametrize("n,depth,rz", [(16, 60, 12), (24, 100, 20), (32, 200, 30)])
def test_c2_family_reduced(n, depth, rz):
    c = W.c2_clifford_rz(seed=1, n=n, depth=depth, n_rz=rz)
    _, g, r = run_both(c)
    compare_fp64(g, r, label=c.name)


def test_c2_full_size_seed0():
    """The full n=32, depth-200, 40-Rz workload (the benchmarked configuration), FP64,
    every term of every generator against the oracle."""
    c = W.c2_clifford_rz(seed=0)
    t0 = time.time()
    _, g, r = run_both(c, threads=16)
    say("c2 full: terms", int(g[0][-1]), "oracle+gpu s", round(time.time() - t0, 1))
    assert int(g[0][-1]) == 44474186
    info = compare_fp64(g, r, label="c2 seed 0")
    say("c2 full residues", info)


def test_hea_full_size_every_generator():
    """n=16, two layers, eps=0 at full size (129,140,286 terms): every generator's count
    against the closed form, and every term of every generator against the oracle (raw key
    sets identical, weights within 1e-12), plus the norm invariant."""
    c = W.c3_hea(seed=0, n=16, layers=2, eps=0.0)
    say("hea full n=16 L=2, all generators")
    t0 = time.time()
    s = run_gpu(c)
    g = s.generators()
    s.close()
    counts = np.diff(g[0].astype(np.int64)).tolist()
    want = [3 ** 16 + 3] + [3 ** (16 - j) + 3 ** (17 - j) + 9 for j in range(1, 15)] + [12]
    assert counts == want and sum(counts) == 129_140_286
    for j in range(16):
        w = g[2][int(g[0][j]):int(g[0][j + 1])]
        assert abs(float(np.sum(w * w)) - 1.0) < 1e-10
    o = oracle.propagate(c, threads=16)
    say("hea full: oracle done", round(time.time() - t0, 1), "s")
    info = compare_fp64(g, oracle_arrays(o, 16), raw_exact=True, label="hea n=16 full")
    say("hea full: compared", info, round(time.time() - t0, 1), "s")


def test_clifford_only_is_exact():
    gates = [Gate.H, Gate.S, Gate.SDG, Gate.SX, Gate.X, Gate.Y, Gate.Z, Gate.CX, Gate.CZ]
    c = W.random_circuit(9, 32, 600, gates=gates)
    _, g, r = run_both(c)
    compare_fp64(g, r, raw_exact=True, label="clifford")
    assert np.all(np.abs(g[2]) == 1.0)
    assert np.diff(g[0].astype(np.int64)).tolist() == [1] * 32


def test_mirror_circuit():
    c = W.c1_random_hst(seed=5).as_single_layer()
    m = c.concat(c.inverse())
    m.layer_end = np.array([m.m])
    s = run_gpu(m)
    off, keys, w = s.generators()
    for j in range(8):
        k = keys[int(off[j]):int(off[j + 1]), 0]
        ww = w[int(off[j]):int(off[j + 1])]
        zj = 3 * 4 ** (7 - j)
        assert abs(ww[k == zj][0] - 1.0) < 1e-12
        assert np.all(np.abs(ww[k != zj]) < 1e-12)


def test_empty_and_single_qubit():
    with Simulator(3) as s:
        s.apply_circuit((np.zeros(0, np.uint8), np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0)))
        assert s.generators()[0].tolist() == [0, 1, 2, 3]
    c = W.random_circuit(3, 1, 50, p_nonclifford=0.5)
    _, g, r = run_both(c)
    compare_fp64(g, r, label="n=1")


# ------------------------------------------------------------------- apply_layer (PTMs)

def _rand_unitary(rng, d):
    A = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    Q, R = np.linalg.qr(A)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


def test_apply_layer_generic_unitaries():
    """Dense non-Clifford one- and two-qubit operators (16x16 PTMs with many nonzeros)."""
    rng = np.random.default_rng(3)
    n = 6
    ops = []
    for k in range(6):
        if k % 2 == 0:
            q = int(rng.integers(n))
            ops.append(((q,), D.ptm_from_unitary(_rand_unitary(rng, 2))))
        else:
            a, b = rng.choice(n, 2, replace=False).tolist()
            ops.append(((a, b), D.ptm_from_unitary(_rand_unitary(rng, 4))))
    say("apply_layer generic")
    s = Simulator(n)
    o = oracle.Oracle(n)
    for qs, R in ops:
        s.apply_layer([(qs, R)])
        if len(qs) == 1:
            o.ptm1(qs[0], R)
        else:
            o.ptm2(qs[0], qs[1], R)
    compare_fp64(s.generators(), oracle_arrays(o, n), tol=1e-11, label="generic")


def test_example1_through_the_abi():
    """Example 1 (Sec. III-B) replayed with non-orthogonal maps (validate = 0): a two-qubit
    map first turns generator 0 (ZI) into 2 XZ + IY, then the example's one-qubit maps give
    6YZ + 8ZZ + IX + IZ (flat indices 11, 15, 1, 3)."""
    def idx(s):
        return 4 * LETTER.index(s[0]) + LETTER.index(s[1])
    M2 = np.eye(16)
    M2[:, idx("ZI")] = 0.0
    M2[idx("XZ"), idx("ZI")] = 2.0
    M2[idx("IY"), idx("ZI")] = 1.0
    M0 = np.eye(4); M0[:, 1] = 0; M0[2, 1] = 3.0; M0[3, 1] = 4.0
    M1 = np.eye(4); M1[:, 2] = 0; M1[1, 2] = 1.0; M1[3, 2] = 1.0
    with Simulator(2, validate=False) as s:
        s.apply_layer([((0, 1), M2)])
        s.apply_layer([((0,), M0), ((1,), M1)])
        off, keys, w = s.generators()
    got = dict(zip(keys[int(off[0]):int(off[1]), 0].tolist(), w[int(off[0]):int(off[1])].tolist()))
    assert got == {string_to_index("YZ"): 6.0, string_to_index("ZZ"): 8.0, string_to_index("IX"): 1.0,
                   string_to_index("IZ"): 1.0}
    assert sorted(got) == [1, 3, 11, 15]


# --------------------------------------------------------------------- failure paths

def test_invalid_inputs_leave_state_unchanged():
    c = W.c3_hea(seed=1, n=5, layers=1, eps=0.0)
    with Simulator(5) as s:
        s.run(c)
        before = s.generators()
        bad = W.Circuit(5, np.array([Gate.H], np.uint8), np.array([7], np.uint32), np.array([7], np.uint32),
                        np.zeros(1), np.array([1]), 0.0)
        with pytest.raises(QimaxError, match="EINVAL"):
            s.apply_circuit(bad)
        bad2 = W.Circuit(5, np.array([99], np.uint8), np.array([0], np.uint32), np.array([0], np.uint32),
                         np.zeros(1), np.array([1]), 0.0)
        with pytest.raises(QimaxError, match="EINVAL"):
            s.apply_circuit(bad2)
        with pytest.raises(QimaxError, match="EINVAL"):
            s.apply_layer([((0,), np.full((4, 4), 0.5))])  # not a PTM of a unitary
        with pytest.raises(QimaxError, match="EINVAL"):
            s.apply_layer([((1, 1), np.eye(16))])
        with pytest.raises(QimaxError, match="EINVAL"):
            s.expect("XYZ")
        after = s.generators()
        for a, b in zip(before, after):
            assert np.array_equal(a, b)


def test_memory_cap_gives_enomem_and_keeps_state():
    c = W.c3_hea(seed=1, n=10, layers=2, eps=0.0)
    with Simulator(10, mem_cap_bytes=2_000_000) as s:
        s.run(c.prefix_layers(1))
        before = s.generators()
        with pytest.raises(QimaxError, match="ENOMEM"):
            s.apply_circuit(c.layer(1))
        after = s.generators()
        for a, b in zip(before, after):
            assert np.array_equal(a, b)
        assert np.diff(after[0].astype(np.int64)).tolist() == [3] * 10


def test_create_rejects_bad_arguments():
    with pytest.raises(QimaxError, match="ETOOLARGE"):
        Simulator(65)
    with pytest.raises(QimaxError, match="EINVAL"):
        Simulator(0)
    with pytest.raises(QimaxError, match="EINVAL"):
        Simulator(4, precision=16)


# ----------------------------------------------------------------------- grouping pass

def test_grouping_matches_the_paper_partition():
    c = W.c1_random_hst(seed=2).as_single_layer()
    with Simulator(c.n) as s:
        ops, K, Kp = s.group(c)
    arity = [2 if g in (Gate.CX, Gate.CZ) else 1 for g in c.gate.tolist()]
    runs = 1 + sum(1 for i in range(1, len(arity)) if arity[i] != arity[i - 1])
    assert K + Kp == runs and abs(K - Kp) <= 1
    # every one-qubit operator is the product of its gates' transfer matrices (Alg. 1)
    pos = 0
    gi = 0
    while gi < c.m:
        two = arity[gi] == 2
        gj = gi
        while gj < c.m and (arity[gj] == 2) == two:
            gj += 1
        if two:
            for i in range(gi, gj):
                qs, R = ops[pos]
                pos += 1
                assert qs == (int(c.q0[i]), int(c.q1[i]))
                assert np.array_equal(R, oracle.gate_ptm(int(c.gate[i])))
        else:
            for q in range(c.n):
                sel = [i for i in range(gi, gj) if int(c.q0[i]) == q]
                if not sel:
                    continue
                M = np.eye(4)
                for i in sel:
                    M = oracle.gate_ptm(int(c.gate[i]), float(c.theta[i])) @ M
                if np.array_equal(M, np.eye(4)):
                    continue
                qs, R = ops[pos]
                pos += 1
                assert qs == (q,)
                assert np.max(np.abs(R - M)) < 1e-14
        gi = gj
    assert pos == len(ops)


# --------------------------------------------------------------------------- precision

@pytest.fixture(scope="module")
def hea16_fp64():
    """The n=16 two-layer ansatz at its stated precision setting (eps = 1e-9), FP64 on the GPU."""
    c = W.c3_hea(seed=0, n=16, layers=2, eps=1e-9)
    s = run_gpu(c)
    yield c, s
    s.close()


@pytest.mark.parametrize("merge", [0, 1])
def test_hea_full_size_fp32_contract(hea16_fp64, merge):
    """The ansatz at full size in FP32 (compensated FP32 sums, or FP64 accumulation), eps =
    1e-9, against FP64 on the GPU: per generator ||w32 - w64|| / ||w64|| <= 5e-6, keys on
    K_tau (tau = 1e-6) identical up to counted straddlers; the library's own per-generator
    error (qimax_compare) agrees with the host's."""
    c, s64 = hea16_fp64
    say("hea fp32 merge", merge)
    s32 = run_gpu(c, precision=32, fp32_merge=merge)
    d, r, kdiff = s32.compare(s64, tau=1e-6)
    rel_lib = d / np.where(r > 0, r, 1.0)
    rel, strad, mx = fp32_contract(s32.generators(), s64.generators(), eps=1e-9)
    say("hea fp32 merge", merge, "rel max", float(rel.max()), "lib", float(rel_lib.max()), "straddlers", strad,
        "max |dw|", mx)
    assert np.allclose(rel_lib, rel, rtol=1e-6, atol=1e-12)
    assert int(kdiff.sum()) == strad
    assert float(rel_lib.max()) <= 5e-6
    s32.close()


@pytest.mark.parametrize("merge", [0, 1])
def test_c2_full_size_fp32_contract(merge):
    """The n=32 Clifford+Rz workload at full size in FP32 against FP64 (eps = 0)."""
    c = W.c2_clifford_rz(seed=0)
    say("c2 fp32 merge", merge)
    s64 = run_gpu(c)
    s32 = run_gpu(c, precision=32, fp32_merge=merge)
    d, r, kdiff = s32.compare(s64, tau=1e-6)
    rel, strad, mx = fp32_contract(s32.generators(), s64.generators(), eps=0.0)
    say("c2 fp32 merge", merge, "rel max", float(rel.max()), "straddlers", strad, "max |dw|", mx)
    assert np.allclose(d / r, rel, rtol=1e-6, atol=1e-12)
    assert int(kdiff.sum()) == strad
    s32.close()
    s64.close()


@pytest.mark.parametrize("merge", [0, 1])
def test_fp32_within_5e6_of_fp64(merge):
    for c in (W.c2_clifford_rz(seed=3, n=24, depth=120, n_rz=24), W.c3_hea(seed=4, n=10, layers=2, eps=1e-9)):
        say("fp32", c.name, "merge", merge)
        g64 = run_gpu(c).generators()
        g32 = run_gpu(c, precision=32, fp32_merge=merge).generators()
        rel, mx = fp32_relative_errors(g32, g64)
        say("fp32 rel max", float(rel.max()), "max |dw|", mx)
        assert float(rel.max()) <= 5e-6


# --------------------------------------------------------------------------- readout

def test_expect_matches_statevector():
    rng = np.random.default_rng(11)
    for c in (W.random_circuit(21, 8, 120, gates=[Gate.H, Gate.S, Gate.CX, Gate.CZ, Gate.SX]),
              W.c1_random_hst(seed=6), W.random_circuit(22, 6, 80, p_nonclifford=0.3)):
        say("expect", c.name)
        psi = D.statevector(c)
        with Simulator(c.n) as s:
            s.run(c)
            off, keys, w = s.generators()
            probes = ["".join(LETTER[int(d)] for d in rng.integers(0, 4, c.n)) for _ in range(6)]
            probes += ["".join("Z" if q == k else "I" for q in range(c.n)) for k in range(c.n)]
            # each generator's own leading Pauli string
            for j in range(c.n):
                k = int(keys[int(off[j]), 0])
                probes.append("".join(LETTER[(k >> (2 * (c.n - 1 - q))) & 3] for q in range(c.n)))
            for p in probes:
                want = float(np.real(np.vdot(psi, D.apply_pauli_state(psi.copy(), c.n,
                                                                     [LETTER.index(ch) for ch in p]))))
                assert abs(s.expect(p) - want) < 1e-9, p


# -------------------------------------------------------------- 128-bit keys (32 < n <= 64)

@pytest.mark.parametrize("n", [33, 40, 48, 64])
def test_wide_keys_random(n):
    c = W.random_layered(n, n, layers=2, gates_per_layer=6 * n, p_nonclifford=0.05)
    _, g, r = run_both(c)
    assert g[1].shape[1] == 2
    compare_fp64(g, r, label=c.name)


def test_wide_keys_clifford_rz():
    c = W.c2_clifford_rz(seed=5, n=48, depth=150, n_rz=22)
    _, g, r = run_both(c)
    compare_fp64(g, r, label=c.name)


def test_wide_keys_initial_and_expect():
    n = 48
    with Simulator(n) as s:
        off, keys, w = s.generators()
        for j in range(n):
            v = int(keys[j, 0]) | (int(keys[j, 1]) << 64)
            assert v == 3 << (2 * (n - 1 - j))
        assert s.expect("Z" + "I" * (n - 1)) == 1.0
        assert s.expect("X" + "I" * (n - 1)) == 0.0


def test_dense_two_qubit_operators_at_n12():
    """Dense non-Clifford two-qubit operators (15 images per non-identity local Pauli) on
    twelve qubits after a Clifford spread, against the oracle: 16x16 expansions on the general
    path with many images per term."""
    rng = np.random.default_rng(11)
    n = 12
    c = W.random_circuit(17, n, 60, gates=[W.Gate.H, W.Gate.S, W.Gate.CX])
    s = Simulator(n)
    o = oracle.Oracle(n)
    s.run(c)
    o.gates(c.gate, c.q0, c.q1, c.theta)
    for k in range(4):
        a, b = rng.choice(n, 2, replace=False).tolist()
        R = D.ptm_from_unitary(_rand_unitary(rng, 4))
        s.apply_layer([((a, b), R)])
        o.ptm2(a, b, R)
    say("dense 2q n12 terms", s.num_terms())
    compare_fp64(s.generators(), oracle_arrays(o, n), tol=1e-11, label="dense 2q n12")
