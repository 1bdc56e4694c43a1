"""Term updates by their definition (test helper, drives the CPU oracle).

One term update is one output image of one grouped operator of the circuit, each operator
group counted once: the circuit is cut into the paper's alternating runs of one-qubit gates
(U_k) and two-qubit gates (V_k) (Sec. III-A, Alg. 2); a U_k with a non-Clifford wire
contributes, for every term it acts on, the product over its wires of the number of nonzero
entries in that wire's composed transfer-matrix column for the term's Pauli on the wire
(the "combinations" of the flatten in Sec. IV); every other group contributes one update per
term it acts on. The term counts come from the oracle, run group by group. This count does
not depend on how the GPU path splits or orders its passes.
"""
from __future__ import annotations

import numpy as np

import oracle

TWO_Q = (12, 13)  # CX, CZ


def _is_signed_perm(M: np.ndarray) -> bool:
    nz = M != 0.0
    return bool(np.all(nz.sum(axis=0) == 1) and np.all(np.abs(M[nz]) == 1.0))


def definition_updates(circuit, threads: int = 0) -> np.ndarray:
    """Per generator term updates of the whole circuit (every layer, prune at layer ends)."""
    n = circuit.n
    o = oracle.Oracle(n)
    upd = np.zeros(n, dtype=np.uint64)
    g, q0, q1, th = circuit.gate, circuit.q0, circuit.q1, circuit.theta
    for a, b in circuit.layers():
        i = a
        while i < b:
            two = int(g[i]) in TWO_Q
            j = i
            while j < b and (int(g[j]) in TWO_Q) == two:
                j += 1
            if two:
                upd += o.counts().astype(np.uint64)
            else:
                wires, nnz, perm = [], [], True
                for q in sorted(set(int(x) for x in q0[i:j])):
                    M = np.eye(4)
                    for k in range(i, j):
                        if int(q0[k]) == q:
                            M = oracle.gate_ptm(int(g[k]), float(th[k])) @ M
                    if np.array_equal(M, np.eye(4)):
                        continue  # an identity chain is no operator
                    wires.append(q)
                    nnz.append((M != 0.0).sum(axis=0))
                    perm &= _is_signed_perm(M)
                if wires:
                    if perm:
                        upd += o.counts().astype(np.uint64)
                    else:
                        upd += o.fanout_sum(wires, np.array(nnz, dtype=np.uint8))
            o.gates(g[i:j], q0[i:j], q1[i:j], th[i:j], threads)
            i = j
        o.prune(circuit.eps)
    o.close()
    return upd
