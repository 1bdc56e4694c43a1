"""Stabilizer tableau for Clifford circuits (test helper).

Aaronson & Gottesman, "Improved simulation of stabilizer circuits" (2004): the n
stabilizer rows of U|0^n> are U Z_j U^dagger, each a signed Pauli string held as
(x bits, z bits, sign bit). Only H, S and CX are primitive here; every other
Clifford gate of the input format is composed from them.
"""
from __future__ import annotations

import numpy as np

from paper_2505_03307_amd.workloads import Gate


class Tableau:
    def __init__(self, n: int):
        self.n = n
        self.x = np.zeros((n, n), dtype=bool)
        self.z = np.eye(n, dtype=bool)
        self.r = np.zeros(n, dtype=bool)

    def h(self, q):
        self.r ^= self.x[:, q] & self.z[:, q]
        self.x[:, q], self.z[:, q] = self.z[:, q].copy(), self.x[:, q].copy()

    def s(self, q):
        self.r ^= self.x[:, q] & self.z[:, q]
        self.z[:, q] ^= self.x[:, q]

    def cx(self, c, t):
        self.r ^= self.x[:, c] & self.z[:, t] & ~(self.x[:, t] ^ self.z[:, c])
        self.x[:, t] ^= self.x[:, c]
        self.z[:, c] ^= self.z[:, t]

    def apply(self, code: int, a: int, b: int):
        g = Gate(code)
        if g == Gate.H:
            self.h(a)
        elif g == Gate.S:
            self.s(a)
        elif g == Gate.SDG:
            self.s(a); self.s(a); self.s(a)
        elif g == Gate.Z:
            self.s(a); self.s(a)
        elif g == Gate.X:
            self.h(a); self.s(a); self.s(a); self.h(a)
        elif g == Gate.Y:
            # Y = i X Z: conjugation by Y equals conjugation by X then Z
            self.h(a); self.s(a); self.s(a); self.h(a)
            self.s(a); self.s(a)
        elif g == Gate.SX:
            self.h(a); self.s(a); self.h(a)
        elif g == Gate.CX:
            self.cx(a, b)
        elif g == Gate.CZ:
            self.h(b); self.cx(a, b); self.h(b)
        elif g == Gate.ISWAP:
            # ISWAP = CX(a,b) CX(b,a) S(b) CX(a,b) in time order, up to a global phase
            self.cx(a, b); self.s(b); self.cx(b, a); self.cx(a, b)
        else:
            raise ValueError(f"not a Clifford gate: {g!r}")

    def run(self, circuit):
        for i in range(circuit.m):
            self.apply(int(circuit.gate[i]), int(circuit.q0[i]), int(circuit.q1[i]))
        return self

    def rows(self):
        """[(x_word, z_word, sign)] per generator (n <= 64)."""
        out = []
        w = (1 << np.arange(self.n, dtype=np.uint64)).astype(np.uint64)
        for j in range(self.n):
            xw = int(np.sum(w[self.x[j]], dtype=np.uint64)) if self.x[j].any() else 0
            zw = int(np.sum(w[self.z[j]], dtype=np.uint64)) if self.z[j].any() else 0
            out.append((xw, zw, -1.0 if self.r[j] else 1.0))
        return out
