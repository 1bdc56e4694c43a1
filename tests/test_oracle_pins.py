"""Pins of the CPU oracle against facts that do not come from the oracle itself:
values the paper prints, the gates' unitaries, dense brute force, a stabilizer
tableau, closed-form counts and invariants. No GPU needed."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

import oracle
from paper_2505_03307_amd import workloads as W
from paper_2505_03307_amd.workloads import Gate

import _dense as D
from _keys import (LETTER, oracle_generator_dict, string_to_xz, xz_to_index, xz_to_strings,
                   string_to_index)
from _tableau import Tableau

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ---------------------------------------------------------------- gate tables

def test_cx_matches_paper_rules():
    """CX conjugation rules and look-up tables of Sec. III-C-2."""
    lines = _read("cx_rules.txt")
    R = oracle.gate_ptm(Gate.CX)
    seen = set()
    luts = {}
    for ln in lines:
        parts = ln.split()
        if parts[0].startswith("LUT"):
            luts[parts[0]] = np.array([int(v) for v in parts[1:]]).reshape(4, 4)
            continue
        src, dst, sign = parts[0], parts[1], float(parts[2])
        i = 4 * LETTER.index(src[0]) + LETTER.index(src[1])
        o = 4 * LETTER.index(dst[0]) + LETTER.index(dst[1])
        col = R[:, i]
        assert col[o] == sign, (src, dst)
        assert np.count_nonzero(col) == 1
        seen.add(src)
    assert len(seen) == 16
    for pc in range(4):
        for pt in range(4):
            col = R[:, 4 * pc + pt]
            o = int(np.flatnonzero(col)[0])
            assert o >> 2 == luts["LUT_c"][pc, pt]
            assert o & 3 == luts["LUT_t"][pc, pt]
            assert col[o] == luts["LUT_sign"][pc, pt]


def test_cx_propagation_matches_paper_rules():
    """The same 16 rules through the oracle's propagation, control on qubit 0."""
    for ln in _read("cx_rules.txt"):
        parts = ln.split()
        if parts[0].startswith("LUT") or parts[0] == "II":
            continue
        x, z = string_to_xz(parts[0])
        o = oracle.Oracle.from_terms(2, [[(x, z, 1.0)]])
        o.gate(Gate.CX, 0, 1)
        assert oracle_generator_dict(o, 0) == {parts[1]: float(parts[2])}


@pytest.mark.parametrize("code", [g for g in Gate if g not in W.TWO_QUBIT])
@pytest.mark.parametrize("theta", [0.0, 0.3, 1.234, -2.5, math.pi / 2])
def test_1q_ptm_matches_unitary(code, theta):
    R = oracle.gate_ptm(code, theta)
    ref = D.ptm_from_unitary(D.unitary_1q(code, theta))
    assert np.max(np.abs(R - ref)) < 1e-14


@pytest.mark.parametrize("code", [Gate.CX, Gate.CZ, Gate.ISWAP])
def test_2q_ptm_matches_unitary(code):
    R = oracle.gate_ptm(code)
    ref = D.ptm_from_unitary(D.unitary_2q(code))
    assert np.max(np.abs(R - ref)) < 1e-14
    assert set(np.unique(R).tolist()) <= {-1.0, 0.0, 1.0}


@pytest.mark.parametrize("code", [Gate.RXX, Gate.RYY, Gate.RZZ])
@pytest.mark.parametrize("theta", [0.0, 0.3, 1.234, -2.5, math.pi / 2])
def test_2q_rotation_ptm_matches_unitary(code, theta):
    """exp(-i theta P P / 2): Paulis commuting with PP stay, the others rotate into -i PP Q."""
    R = oracle.gate_ptm(code, theta)
    ref = D.ptm_from_unitary(D.unitary_2q(code, theta))
    assert np.max(np.abs(R - ref)) < 1e-14
    # every column has one or two nonzeros (fan-out at most 2)
    assert set(((R != 0).sum(axis=0)).tolist()) <= {1, 2}


def test_sx_maps_z_to_minus_y():
    R = oracle.gate_ptm(Gate.SX)
    assert R[2, 3] == -1.0 and np.count_nonzero(R[:, 3]) == 1


# ---------------------------------------------------------------- worked examples

def test_example1_flatten():
    """Example 1 (Sec. III-B): 2(3Y+4Z)Z + I(X+Z) -> 6YZ + 8ZZ + IX + IZ."""
    lines = _read("example1.txt")
    n = int(lines[0].split()[1])
    terms, maps, expect = [], {}, {}
    for ln in lines[1:]:
        p = ln.split()
        if p[0] == "input":
            x, z = string_to_xz(p[1])
            terms.append((x, z, float(p[2])))
        elif p[0] == "map":
            q = int(p[1])
            M = maps.setdefault(q, np.eye(4))
            col = LETTER.index(p[2])
            M[:, col] = 0.0
            for item in p[3:]:
                out, v = item.split(":")
                M[LETTER.index(out), col] = float(v)
        elif p[0] == "output":
            expect[p[1]] = (float(p[2]), int(p[3]))
    o = oracle.Oracle.from_terms(n, [terms])
    for q, M in sorted(maps.items()):
        o.ptm1(q, M)
    got = oracle_generator_dict(o, 0)
    assert got == {k: v[0] for k, v in expect.items()}
    x, z, _ = o.read(0)
    idx = xz_to_index(x, z, n)[:, 0].tolist()
    assert sorted(idx) == sorted(v[1] for v in expect.values())
    for k, (_, i) in expect.items():
        assert string_to_index(k) == i


def _parse_gens(text):
    gens = []
    for part in text.split(";"):
        tok = part.split()
        d = {}
        if len(tok) == 1:
            s = tok[0]
            sign = -1.0 if s.startswith("-") else 1.0
            d[s.lstrip("+-")] = sign
        else:
            for i in range(0, len(tok), 2):
                d[tok[i + 1]] = float(tok[i])
        gens.append(d)
    return gens


@pytest.mark.parametrize("reading", ["printed_pi_over_6", "pi_over_3"])
def test_example_sx_rz_cx(reading):
    lines = _read("example_sx_rz_cx.txt")
    n = int(lines[0].split()[1])
    o = oracle.Oracle(n)
    theta = math.pi / 6 if reading == "printed_pi_over_6" else math.pi / 3
    for ln in lines[1:]:
        head, body = ln.split("|")
        h = head.split()
        if h[1] == "SX":
            o.gate(Gate.SX, int(h[2]))
        elif h[1] == "RZ":
            o.gate(Gate.RZ, int(h[2]), theta=theta)
        elif h[1] == "CX":
            o.gate(Gate.CX, int(h[2]), int(h[3]))
        want = _parse_gens(body)
        if reading == "pi_over_3":
            # (1/2, -sqrt3/2) -> (sqrt3/2, -1/2): sin and cos exchange at t = pi/3
            for d in want:
                if len(d) == 2:
                    (k1, v1), (k2, v2) = d.items()
                    d[k1], d[k2] = -v2, -v1
        for g in range(n):
            got = oracle_generator_dict(o, g)
            assert set(got) == set(want[g])
            for k in got:
                assert abs(got[k] - want[g][k]) < 1e-15


@pytest.mark.parametrize("t1,t2", [(0.3, 1.1), (2.0, -0.7), (4.0, 5.5)])
def test_example_ry_rx(t1, t2):
    env = {"cos": math.cos, "sin": math.sin, "t1": t1, "t2": t2}
    want = {}
    for ln in _read("example_ry_rx.txt"):
        p, expr = ln.split(maxsplit=1)
        want[p] = eval(expr, {"__builtins__": {}}, env)
    o = oracle.Oracle(1)
    o.gate(Gate.H, 0)
    o.gate(Gate.RY, 0, theta=t1)
    o.gate(Gate.RX, 0, theta=t2)
    got = oracle_generator_dict(o, 0)
    for k, v in want.items():
        assert abs(got.get(k, 0.0) - v) < 1e-15


def test_initial_generators():
    n = 5
    o = oracle.Oracle(n)
    for j in range(n):
        x, z, w = o.read(j)
        assert w.tolist() == [1.0]
        assert xz_to_index(x, z, n)[0, 0] == 3 * 4 ** (n - 1 - j)


# ---------------------------------------------------------------- dense brute force

def _dense_generators(circuit):
    n = circuit.n
    U = D.full_unitary(circuit)
    out = []
    for j in range(n):
        Zj = D.pauli_string_matrix([3 if q == j else 0 for q in range(n)])
        c = D.pauli_decompose(U @ Zj @ U.conj().T, n)
        assert np.max(np.abs(c.imag)) < 1e-12
        out.append(c.real)
    return out


def _assert_matches_dense(circuit, tol=1e-12):
    o = oracle.propagate(circuit)
    dense = _dense_generators(circuit)
    for j in range(circuit.n):
        x, z, w = o.read(j)
        idx = xz_to_index(x, z, circuit.n)[:, 0].astype(np.int64)
        ref = dense[j]
        sig = np.flatnonzero(np.abs(ref) > tol)
        mine = {int(i): float(v) for i, v in zip(idx, w) if abs(v) > tol}
        assert sorted(mine) == sig.tolist()
        for i in sig.tolist():
            assert abs(mine[i] - ref[i]) < tol
        assert 0 not in mine  # no identity term


@pytest.mark.parametrize("seed", range(6))
def test_oracle_vs_dense_unitary_random(seed):
    n = 1 + seed % 5
    _assert_matches_dense(W.random_circuit(seed, n, 30 + 10 * n, p_nonclifford=0.25))


def test_oracle_vs_dense_unitary_c1():
    """The whole of the n=8 random {H,S,T}+CX workload, every weight."""
    _assert_matches_dense(W.c1_random_hst(seed=0))


def test_oracle_vs_dense_hea():
    _assert_matches_dense(W.c3_hea(seed=3, n=5, layers=2, eps=0.0))


def _random_unitary(rng, d):
    A = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    Q, R = np.linalg.qr(A)
    return Q * (np.diag(R) / np.abs(np.diag(R)))


def test_generic_ptm_ops_vs_dense():
    """Arbitrary one- and two-qubit unitaries given as transfer matrices."""
    rng = np.random.default_rng(7)
    n = 4
    ops = [("1", 2, None, _random_unitary(rng, 2)), ("2", 0, 3, _random_unitary(rng, 4)),
           ("2", 2, 1, _random_unitary(rng, 4)), ("1", 0, None, _random_unitary(rng, 2))]
    o = oracle.Oracle(n)
    Ufull = np.eye(2 ** n, dtype=complex)
    for kind, a, b, U in ops:
        if kind == "1":
            o.ptm1(a, D.ptm_from_unitary(U))
            cols = [D._apply_1q_state(Ufull[:, k].copy(), n, a, U) for k in range(2 ** n)]
        else:
            o.ptm2(a, b, D.ptm_from_unitary(U))
            cols = [D._apply_2q_state(Ufull[:, k].copy(), n, a, b, U) for k in range(2 ** n)]
        Ufull = np.stack(cols, axis=1)
    for j in range(n):
        Zj = D.pauli_string_matrix([3 if q == j else 0 for q in range(n)])
        ref = D.pauli_decompose(Ufull @ Zj @ Ufull.conj().T, n).real
        x, z, w = o.read(j)
        idx = xz_to_index(x, z, n)[:, 0].astype(np.int64)
        got = np.zeros(4 ** n)
        got[idx] = w
        assert np.max(np.abs(got - ref)) < 1e-12


# ---------------------------------------------------------------- statevector semantics

@pytest.mark.parametrize("seed", range(4))
def test_stabilizer_relation(seed):
    """G_j |psi> = |psi> for every propagated generator (n <= 10)."""
    n = 6 + seed
    # one-qubit gates with CX and CZ: the two-qubit rotations are covered by the dense pins
    gates = [g for g in Gate if g not in (Gate.ISWAP, Gate.RXX, Gate.RYY, Gate.RZZ)]
    c = W.random_circuit(100 + seed, n, 12 * n, p_nonclifford=0.2, gates=gates)
    psi = D.statevector(c)
    o = oracle.propagate(c)
    for j in range(n):
        x, z, w = o.read(j)
        strings = xz_to_strings(x, z, n)
        acc = np.zeros_like(psi)
        for s, wt in zip(strings, w):
            acc += wt * D.apply_pauli_state(psi.copy(), n, [LETTER.index(ch) for ch in s])
        assert np.max(np.abs(acc - psi)) < 1e-10


def test_density_operator_product():
    """rho = 2^-n prod_j (I + G_j) equals |psi><psi| (eq. (2))."""
    c = W.random_circuit(5, 4, 40, p_nonclifford=0.3)
    n = c.n
    psi = D.statevector(c)
    o = oracle.propagate(c)
    rho = np.eye(2 ** n, dtype=complex)
    for j in range(n):
        x, z, w = o.read(j)
        G = np.zeros((2 ** n, 2 ** n), dtype=complex)
        for s, wt in zip(xz_to_strings(x, z, n), w):
            G += wt * D.pauli_string_matrix([LETTER.index(ch) for ch in s])
        rho = rho @ (np.eye(2 ** n) + G)
    rho /= 2 ** n
    assert np.max(np.abs(rho - np.outer(psi, psi.conj()))) < 1e-10


# ---------------------------------------------------------------- Clifford special case

@pytest.mark.parametrize("n", [5, 17, 32, 48])
def test_clifford_matches_tableau(n):
    gates = [Gate.H, Gate.S, Gate.SDG, Gate.SX, Gate.X, Gate.Y, Gate.Z, Gate.CX, Gate.CZ, Gate.ISWAP]
    c = W.random_circuit(n, n, 20 * n, gates=gates)
    o = oracle.propagate(c)
    rows = Tableau(n).run(c).rows()
    for j in range(n):
        x, z, w = o.read(j)
        assert len(w) == 1 and abs(w[0]) == 1.0
        assert (int(x[0]), int(z[0]), float(w[0])) == rows[j]


def test_c2_without_rz_matches_tableau():
    c = W.c2_clifford_rz(seed=2)
    keep = c.gate != Gate.RZ
    cl = W.Circuit(c.n, c.gate[keep], c.q0[keep], c.q1[keep], c.theta[keep],
                   np.array([int(keep.sum())]), 0.0, "c2-clifford")
    o = oracle.propagate(cl)
    rows = Tableau(c.n).run(cl).rows()
    for j in range(c.n):
        x, z, w = o.read(j)
        assert (int(x[0]), int(z[0]), float(w[0])) == rows[j]


# ---------------------------------------------------------------- invariants and counts

@pytest.mark.parametrize("seed", range(5))
def test_norm_invariant(seed):
    """sum_a w_a^2 = 1: conjugation by a unitary preserves the Pauli-basis norm."""
    c = W.c1_random_hst(seed) if seed < 3 else W.c3_hea(seed, n=6, layers=2, eps=0.0)
    o = oracle.propagate(c)
    for j in range(c.n):
        _, _, w = o.read(j)
        assert abs(np.sum(w * w) - 1.0) < 1e-12
        assert np.max(np.abs(w)) <= 1.0 + 1e-12


@pytest.mark.parametrize("n", range(3, 10))
def test_hea_closed_form_counts(n):
    """Term counts of the Rx/Ry/Rz + CX-ladder ansatz at eps = 0 and generic angles:
    3n after one layer and 3^(n+1) + 9n - 21 after two; generator 0 holds 3^n + 3,
    generator j in [1, n-2] holds 3^(n-j) + 3^(n+1-j) + 9, the last holds 12."""
    c = W.c3_hea(seed=n, n=n, layers=2, eps=0.0)
    o1 = oracle.propagate(c.prefix_layers(1))
    assert o1.counts().tolist() == [3] * n
    counts = oracle.propagate(c).counts().tolist()
    want = [3 ** n + 3] + [3 ** (n - j) + 3 ** (n + 1 - j) + 9 for j in range(1, n - 1)] + [12]
    assert counts == want
    assert sum(counts) == 3 ** (n + 1) + 9 * n - 21


def test_mirror_circuit_returns_to_z():
    c = W.c1_random_hst(seed=4)
    mirror = c.as_single_layer().concat(c.inverse())
    mirror.layer_end = np.array([mirror.m])
    o = oracle.propagate(mirror)
    for j in range(c.n):
        d = oracle_generator_dict(o, j)
        zj = "".join("Z" if q == j else "I" for q in range(c.n))
        assert abs(d[zj] - 1.0) < 1e-12
        assert all(abs(v) < 1e-12 for k, v in d.items() if k != zj)


def test_prune_at_layer_end():
    c = W.c3_hea(seed=1, n=6, layers=2, eps=0.0)
    full = oracle.propagate(c)
    eps = 0.05
    c2 = W.c3_hea(seed=1, n=6, layers=2, eps=eps)
    pruned = oracle.propagate(c2)
    # replay by hand: layer 1, prune, layer 2, prune
    o = oracle.Oracle(6)
    for li in range(2):
        lay = c.layer(li)
        for i in range(lay.m):
            o.gate(int(lay.gate[i]), int(lay.q0[i]), int(lay.q1[i]), float(lay.theta[i]))
        o.prune(eps)
    for j in range(6):
        a = pruned.read(j)
        b = o.read(j)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
        assert np.all(np.abs(a[2]) > eps)
    assert pruned.counts().sum() < full.counts().sum()


def test_subset_equals_full():
    c = W.c2_clifford_rz(seed=0, n_rz=12, depth=60, n=16)
    full = oracle.propagate(c)
    sub = oracle.propagate(c, gens=[3, 11])
    for slot, j in enumerate([3, 11]):
        a, b = full.read(j), sub.read(slot)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


def test_exact_cancellation_is_dropped():
    """Rz(t) then Rz(-t) on X: the Y coefficient cos(t)sin(t) - sin(t)cos(t) is an exact zero
    in floating point and must not be stored (only non-zero weights are kept, Sec. III-B)."""
    o = oracle.Oracle(1)
    o.gate(Gate.H, 0)
    o.gate(Gate.RZ, 0, theta=0.7)
    o.gate(Gate.RZ, 0, theta=-0.7)
    d = oracle_generator_dict(o, 0)
    assert list(d) == ["X"] and abs(d["X"] - 1.0) < 1e-15


def test_prune_drops_weights_equal_to_eps():
    """The prune keeps |w| > eps: a weight exactly equal to eps is dropped."""
    R = np.eye(4)
    R[:, 3] = 0.0
    R[1, 3] = 0.5     # Z -> 0.5 X + 0.25 Y (a linear map, not a unitary)
    R[2, 3] = 0.25
    o = oracle.Oracle(1)
    o.ptm1(0, R)
    o.prune(0.25)
    assert oracle_generator_dict(o, 0) == {"X": 0.5}
