"""Term updates by their definition (test helper, drives the CPU oracle).

One term update is one output image of one grouped operator of the circuit, each operator
group counted once: the circuit is cut into the paper's alternating runs of one-qubit gates
(U_k) and two-qubit gates (V_k) (Sec. III-A, Alg. 2); a U_k with a non-Clifford wire
contributes, for every term it acts on, the product over its wires of the number of nonzero
entries in that wire's composed transfer-matrix column for the term's Pauli on the wire
(the "combinations" of the flatten in Sec. IV). A V_k's operators are its two-qubit gates,
consecutive gates on the same pair of wires fused into one (no gate of the run touching
either wire in between); a V_k with a non-Clifford operator contributes, for each such
operator in order, the nonzero count of its transfer-matrix column for every term it acts
on. Every other group contributes one update per term it acts on. The term counts come from
the oracle, run group by group. This count does not depend on how the GPU path splits or
orders its passes.
"""
from __future__ import annotations

import numpy as np

import oracle

TWO_Q = (12, 13, 14, 15, 16, 17)  # CX, CZ, ISWAP, RXX, RYY, RZZ


def _is_signed_perm(M: np.ndarray) -> bool:
    nz = M != 0.0
    return bool(np.all(nz.sum(axis=0) == 1) and np.all(np.abs(M[nz]) == 1.0))


def _swap_wires(R: np.ndarray) -> np.ndarray:
    """A 16x16 operator on (q0, q1) written for the wires in the other order."""
    idx = [4 * (k & 3) + (k >> 2) for k in range(16)]
    return R[np.ix_(idx, idx)]


def _pair_blocks(g, q0, q1, th, i, j):
    """The operators of the V_k run g[i:j]: [(wire a, wire b, R, member gate indices)],
    consecutive gates on one pair fused (the later gate acting on the earlier's images)."""
    blocks, last = [], {}
    for k in range(i, j):
        a, b = int(q0[k]), int(q1[k])
        R = oracle.gate_ptm(int(g[k]), float(th[k]))
        if a in last and b in last and last[a] == last[b]:
            a0, b0, R0, members = blocks[last[a]]
            blocks[last[a]] = (a0, b0, (R if a == a0 else _swap_wires(R)) @ R0, members + [k])
            continue
        last[a] = last[b] = len(blocks)
        blocks.append((a, b, R, [k]))
    return blocks


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
                blocks = _pair_blocks(g, q0, q1, th, i, j)
                if all(_is_signed_perm(R) for _, _, R, _m in blocks):
                    upd += o.counts().astype(np.uint64)
                    o.gates(g[i:j], q0[i:j], q1[i:j], th[i:j], threads)
                else:
                    # operator by operator (operators on disjoint wires commute, so this order
                    # gives the run's result); a non-Clifford one counts its images
                    for a2, b2, R, members in blocks:
                        if not _is_signed_perm(R):
                            upd += o.fanout_sum2(a2, b2, (R != 0.0).sum(axis=0).astype(np.uint8))
                        k = np.array(members)
                        o.gates(g[k], q0[k], q1[k], th[k], threads)
                i = j
                continue
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
