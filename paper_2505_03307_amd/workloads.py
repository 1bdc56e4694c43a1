"""Seeded synthetic circuits: the inputs shared by the HIP path and the CPU oracle.

This module holds only the input format and the random circuit recipes. It
contains none of the method's arithmetic (no Pauli algebra, no transfer
matrices, no merging): both sides receive the same instruction arrays and each
computes from them on its own.

Instruction format (the paper's instruction tuple {g, w, theta}, Sec. III-A):
one gate per row, stored as four parallel arrays

    gate  : uint8   gate code (see ``Gate``)
    q0    : uint32  first wire (the control for CX)
    q1    : uint32  second wire for two-qubit gates, else equal to q0
    theta : float64 rotation angle; 0 for gates without a parameter

Two-qubit gates: CX (q0 = control), CZ, ISWAP, and the rotations RXX, RYY, RZZ
(exp(-i theta P P / 2) for P = X, Y, Z on both wires).

``layer_end`` lists, for every circuit layer, the index one past its last
instruction. A layer is what one call of the propagation API receives; the
prune of small weights runs once at the end of each layer.
"""
from __future__ import annotations

import dataclasses
import enum
import math

import numpy as np


class Gate(enum.IntEnum):
    """Gate codes of the instruction arrays (input format, identical on both sides)."""
    H = 0
    S = 1
    SDG = 2
    T = 3
    TDG = 4
    SX = 5
    X = 6
    Y = 7
    Z = 8
    RX = 9
    RY = 10
    RZ = 11
    CX = 12
    CZ = 13
    ISWAP = 14
    RXX = 15
    RYY = 16
    RZZ = 17


TWO_QUBIT = (Gate.CX, Gate.CZ, Gate.ISWAP, Gate.RXX, Gate.RYY, Gate.RZZ)
CLIFFORD_1Q = (Gate.H, Gate.S, Gate.SDG, Gate.SX, Gate.X, Gate.Y, Gate.Z)
ROTATIONS = (Gate.RX, Gate.RY, Gate.RZ, Gate.RXX, Gate.RYY, Gate.RZZ)
NON_CLIFFORD = (Gate.T, Gate.TDG) + ROTATIONS


@dataclasses.dataclass
class Circuit:
    n: int
    gate: np.ndarray
    q0: np.ndarray
    q1: np.ndarray
    theta: np.ndarray
    layer_end: np.ndarray
    eps: float = 0.0
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.gate.shape[0])

    def layers(self):
        """Yield (start, stop) instruction ranges, one per layer."""
        start = 0
        for stop in self.layer_end.tolist():
            yield start, int(stop)
            start = int(stop)

    def layer(self, i: int) -> "Circuit":
        bounds = list(self.layers())
        a, b = bounds[i]
        return Circuit(self.n, self.gate[a:b], self.q0[a:b], self.q1[a:b], self.theta[a:b],
                       np.array([b - a], dtype=np.int64), self.eps, f"{self.name}[layer {i}]")

    def prefix_layers(self, k: int) -> "Circuit":
        """The first k layers as a circuit of their own."""
        stop = int(self.layer_end[k - 1]) if k > 0 else 0
        return Circuit(self.n, self.gate[:stop], self.q0[:stop], self.q1[:stop], self.theta[:stop],
                       self.layer_end[:k].copy(), self.eps, f"{self.name}[:{k} layers]")

    def as_single_layer(self) -> "Circuit":
        return Circuit(self.n, self.gate, self.q0, self.q1, self.theta,
                       np.array([self.m], dtype=np.int64), self.eps, self.name)

    def inverse(self) -> "Circuit":
        """U^dagger as instructions: reversed order, each gate inverted."""
        inv = {Gate.S: Gate.SDG, Gate.SDG: Gate.S, Gate.T: Gate.TDG, Gate.TDG: Gate.T}
        g = self.gate[::-1].copy()
        th = -self.theta[::-1].copy()
        cube = []
        for i in range(g.shape[0]):
            code = Gate(int(g[i]))
            if code in (Gate.SX, Gate.ISWAP):
                cube.append(i)
            g[i] = int(inv.get(code, code))
            if code not in ROTATIONS:
                th[i] = 0.0
        q0 = self.q0[::-1].copy()
        q1 = self.q1[::-1].copy()
        if cube:  # SX^dagger = SX^3, ISWAP^dagger = ISWAP^3: expand in place
            cube = set(cube)
            rows = []
            for i in range(g.shape[0]):
                reps = 3 if i in cube else 1
                rows.extend([i] * reps)
            rows = np.array(rows)
            g, q0, q1, th = g[rows], q0[rows], q1[rows], th[rows]
        return Circuit(self.n, g, q0, q1, th, np.array([g.shape[0]], dtype=np.int64), self.eps,
                       f"inverse({self.name})")

    def concat(self, other: "Circuit") -> "Circuit":
        assert self.n == other.n
        return Circuit(self.n, np.concatenate([self.gate, other.gate]),
                       np.concatenate([self.q0, other.q0]), np.concatenate([self.q1, other.q1]),
                       np.concatenate([self.theta, other.theta]),
                       np.concatenate([self.layer_end, other.layer_end + self.m]), self.eps,
                       f"{self.name}+{other.name}")


class _Builder:
    def __init__(self, n: int):
        self.n = n
        self.g, self.a, self.b, self.t = [], [], [], []
        self.ends = []

    def add(self, code: Gate, q0: int, q1: int | None = None, theta: float = 0.0):
        if q1 is None:
            q1 = q0
        self.g.append(int(code)); self.a.append(int(q0)); self.b.append(int(q1)); self.t.append(float(theta))

    def end_layer(self):
        if not self.ends or self.ends[-1] != len(self.g):
            self.ends.append(len(self.g))

    def build(self, eps: float = 0.0, name: str = "") -> Circuit:
        self.end_layer()
        return Circuit(self.n, np.array(self.g, dtype=np.uint8), np.array(self.a, dtype=np.uint32),
                       np.array(self.b, dtype=np.uint32), np.array(self.t, dtype=np.float64),
                       np.array(self.ends, dtype=np.int64), eps, name)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def c1_random_hst(seed: int = 0, n: int = 8, layers: int = 20, p_t: float = 0.05) -> Circuit:
    """n=8 qubits, 20 layers; per layer one gate per qubit from {H, S, T} (T with
    probability 0.05, else H or S evenly), then CX on a random perfect matching with
    each orientation drawn by a fair coin. FP64, eps = 0."""
    rng = _rng(seed)
    b = _Builder(n)
    for _ in range(layers):
        for q in range(n):
            u = rng.random()
            b.add(Gate.T if u < p_t else (Gate.H if u < p_t + (1 - p_t) / 2 else Gate.S), q)
        perm = rng.permutation(n)
        for i in range(0, n - 1, 2):
            c, t = int(perm[i]), int(perm[i + 1])
            if rng.random() < 0.5:
                c, t = t, c
            b.add(Gate.CX, c, t)
        b.end_layer()
    return b.build(0.0, f"c1(seed={seed},n={n},L={layers})")


def _clifford_rz_moments(rng: np.random.Generator, n: int, depth: int, n_rz: int, b: _Builder,
                         layer_per_moment: bool):
    """Random Clifford moments (each unused qubit draws H, S or CX uniformly; a CX
    pairs with the next unused qubit of the walk and takes a random orientation;
    the last qubit falls back to H or S), with n_rz Rz gates at distinct
    (moment, qubit) slots, each placed after that moment's Clifford gates."""
    n_rz = min(n_rz, n * depth)
    slots = rng.choice(n * depth, size=n_rz, replace=False)
    slot_set = {}
    for s in slots.tolist():
        slot_set.setdefault(s // n, []).append(s % n)
    for d in range(depth):
        perm = rng.permutation(n).tolist()
        one_q, two_q = [], []
        i = 0
        while i < n:
            q = perm[i]
            choice = int(rng.integers(3))
            if choice == 2 and i + 1 < n:
                p = perm[i + 1]
                if rng.random() < 0.5:
                    two_q.append((q, p))
                else:
                    two_q.append((p, q))
                i += 2
                continue
            if choice == 2:
                choice = int(rng.integers(2))
            one_q.append((Gate.H if choice == 0 else Gate.S, q))
            i += 1
        for code, q in one_q:
            b.add(code, q)
        for c, t in two_q:
            b.add(Gate.CX, c, t)
        for q in sorted(slot_set.get(d, [])):
            b.add(Gate.RZ, q, q, float(rng.uniform(0.0, 2.0 * math.pi)))
        if layer_per_moment:
            b.end_layer()


def c2_clifford_rz(seed: int = 0, n: int = 32, depth: int = 200, n_rz: int = 40,
                   layer_per_moment: bool = False) -> Circuit:
    """n=32, 200 random Clifford moments (H, S, CX uniform) with 40 Rz(theta),
    theta ~ U[0, 2pi), at random (moment, qubit) slots. eps = 0, so the layer split
    does not change the result; by default the whole circuit is one layer."""
    rng = _rng(seed)
    b = _Builder(n)
    _clifford_rz_moments(rng, n, depth, n_rz, b, layer_per_moment)
    return b.build(0.0, f"c2(seed={seed},n={n},D={depth},Rz={n_rz})")


def c3_hea(seed: int = 0, n: int = 16, layers: int = 2, eps: float = 1e-9) -> Circuit:
    """Hardware-efficient ansatz: per layer Rx, Ry, Rz on every qubit (angles
    U[0, 2pi)), then the CX ladder CX(0,1), CX(1,2), ..., CX(n-2, n-1)."""
    rng = _rng(seed)
    b = _Builder(n)
    for _ in range(layers):
        for q in range(n):
            for code in (Gate.RX, Gate.RY, Gate.RZ):
                b.add(code, q, q, float(rng.uniform(0.0, 2.0 * math.pi)))
        for q in range(n - 1):
            b.add(Gate.CX, q, q + 1)
        b.end_layer()
    return b.build(eps, f"c3(seed={seed},n={n},L={layers})")


def c4_batch(batch_seed: int = 0, count: int = 256, n_range=(8, 48), depth_range=(50, 400),
             rz_range=(5, 30)) -> list[Circuit]:
    """256 circuits: n ~ U{8..48}, depth ~ U{50..400}, 5..30 Rz each, built as the
    n=32 Clifford+Rz family; circuit i draws its gates from seed 1000 + i."""
    rng = _rng(batch_seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
        k = int(rng.integers(rz_range[0], rz_range[1] + 1))
        crng = _rng(1000 + i)
        b = _Builder(n)
        _clifford_rz_moments(crng, n, depth, k, b, False)
        out.append(b.build(0.0, f"c4[{i}](n={n},D={depth},Rz={k})"))
    return out


def c5_stream(seed: int = 0, count: int = 2000, n_range=(10, 16), layer_choices=(1, 2),
              eps: float = 1e-9):
    """Served stream: circuits from the hardware-efficient-ansatz family with fresh
    angles, n ~ U{10..16}, L ~ U{1, 2}. Returns (circuits, unit-rate exponential
    inter-arrival gaps); the caller scales the gaps to its arrival rate."""
    rng = _rng(seed)
    circuits, gaps = [], []
    for i in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        L = int(rng.choice(layer_choices))
        circuits.append(c3_hea(seed=10_000 + i, n=n, layers=L, eps=eps))
        gaps.append(float(rng.exponential(1.0)))
    return circuits, np.array(gaps)


def random_circuit(seed: int, n: int, m: int, p_nonclifford: float = 0.15,
                   gates=None) -> Circuit:
    """A small random circuit over the full gate set, for parity and pin tests."""
    rng = _rng(seed)
    if gates is None:
        gates = list(Gate)
    b = _Builder(n)
    for _ in range(m):
        code = Gate(int(rng.choice([int(g) for g in gates])))
        if code in NON_CLIFFORD and rng.random() > p_nonclifford * 4:
            code = Gate(int(rng.choice([int(g) for g in CLIFFORD_1Q if g in gates] or [int(Gate.H)])))
        th = float(rng.uniform(0, 2 * math.pi)) if code in ROTATIONS else 0.0
        if code in TWO_QUBIT:
            if n < 2:
                continue
            a, c = rng.choice(n, size=2, replace=False).tolist()
            b.add(code, a, c, th)
        else:
            q = int(rng.integers(n))
            b.add(code, q, q, th)
    return b.build(0.0, f"random(seed={seed},n={n},m={m})")


def random_layered(seed: int, n: int, layers: int, gates_per_layer: int, eps: float = 0.0,
                   p_nonclifford: float = 0.15) -> Circuit:
    """A random circuit split into several layers (prune points)."""
    c = random_circuit(seed, n, layers * gates_per_layer, p_nonclifford)
    m = c.m
    ends = np.linspace(0, m, layers + 1).astype(np.int64)[1:]
    ends[-1] = m
    ends = np.unique(ends)
    return Circuit(n, c.gate, c.q0, c.q1, c.theta, ends, eps, f"layered(seed={seed},n={n},L={layers})")


# ------------------------------------------------------------------------------------------
# The paper's benchmark families (Sec. V): GHZ, graph state and |XYZ + chain>. The paper's
# circuits came from a generator that is not available here; these are built from the
# paper's description of their structure: L layers, each with its component repeated
# #Repeats times (the gate count grows linearly with #Repeats and with n).

def _from_arrays(n: int, gate, q0, q1, theta, layer_end, eps: float, name: str) -> Circuit:
    return Circuit(n, np.asarray(gate, dtype=np.uint8), np.asarray(q0, dtype=np.uint32),
                   np.asarray(q1, dtype=np.uint32), np.asarray(theta, dtype=np.float64),
                   np.asarray(layer_end, dtype=np.int64), eps, name)


def _repeat_block(n: int, gate, q0, q1, repeats: int, layers: int, name: str) -> Circuit:
    """A parameter-free block repeated `repeats` times per layer, `layers` layers."""
    g = np.tile(np.asarray(gate, dtype=np.uint8), repeats * layers)
    a = np.tile(np.asarray(q0, dtype=np.uint32), repeats * layers)
    b = np.tile(np.asarray(q1, dtype=np.uint32), repeats * layers)
    per = len(gate) * repeats
    ends = np.arange(1, layers + 1, dtype=np.int64) * per
    return _from_arrays(n, g, a, b, np.zeros(g.shape[0]), ends, 0.0, name)


def ghz(n: int, repeats: int = 1, layers: int = 1) -> Circuit:
    """GHZ preparation (H on qubit 0, then CX(0,1), CX(1,2), ..., CX(n-2, n-1)) as the block,
    repeated `repeats` times in each of `layers` layers. A Clifford circuit: every generator
    stays a single Pauli string (stabilizer rank 1)."""
    gate = [Gate.H] + [Gate.CX] * (n - 1)
    q0 = [0] + list(range(n - 1))
    q1 = [0] + list(range(1, n))
    return _repeat_block(n, gate, q0, q1, repeats, layers, f"ghz(n={n},R={repeats},L={layers})")


def graph_state(seed: int, n: int, repeats: int = 1, layers: int = 1, p_edge: float = 0.5) -> Circuit:
    """Graph-state preparation on a seeded random graph G(n, p_edge): H on every qubit, then
    CZ on every edge (in lexicographic edge order); the block repeated `repeats` times in each
    of `layers` layers. Clifford: stabilizer rank 1."""
    rng = _rng(seed)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p_edge]
    gate = [Gate.H] * n + [Gate.CZ] * len(edges)
    q0 = list(range(n)) + [e[0] for e in edges]
    q1 = list(range(n)) + [e[1] for e in edges]
    return _repeat_block(n, gate, q0, q1, repeats, layers, f"graph(seed={seed},n={n},R={repeats},L={layers})")


def xyz_chain(seed: int, n: int, repeats: int, layers: int = 1, eps: float = 0.0) -> Circuit:
    """|XYZ + chain>: per layer, the XYZ component (Rx, Ry, Rz on every qubit, angles
    U[0, 2pi)) repeated `repeats` times, then the chain CX(0,1), CX(1,2), ..., CX(n-2, n-1).
    Each layer is one prune point. Built with array operations, so that #Repeats = 10^5
    (millions of gates) is cheap."""
    rng = _rng(seed)
    per_rep = 3 * n
    g1 = np.tile(np.array([Gate.RX, Gate.RY, Gate.RZ], dtype=np.uint8), n * repeats)
    w1 = np.tile(np.repeat(np.arange(n, dtype=np.uint32), 3), repeats)
    gs, qa, qb, th, ends = [], [], [], [], []
    m = 0
    for _ in range(layers):
        angles = rng.uniform(0.0, 2.0 * math.pi, size=per_rep * repeats)
        gs += [g1, np.full(n - 1, Gate.CX, dtype=np.uint8)]
        qa += [w1, np.arange(n - 1, dtype=np.uint32)]
        qb += [w1, np.arange(1, n, dtype=np.uint32)]
        th += [angles, np.zeros(n - 1)]
        m += per_rep * repeats + n - 1
        ends.append(m)
    return _from_arrays(n, np.concatenate(gs), np.concatenate(qa), np.concatenate(qb), np.concatenate(th),
                        ends, eps, f"xyz_chain(seed={seed},n={n},R={repeats},L={layers})")
