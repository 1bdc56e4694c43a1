"""The term-update count by its definition (tests/_updates.py), pinned by hand counts on small
circuits (no GPU). One update = one output image of one grouped operator, each group once."""
import math

import numpy as np

from paper_2505_03307_amd.workloads import Circuit, Gate
from _updates import definition_updates


def _circ(n, rows, layer_end=None, eps=0.0):
    g = np.array([int(r[0]) for r in rows], np.uint8)
    a = np.array([r[1] for r in rows], np.uint32)
    b = np.array([r[2] if len(r) > 2 else r[1] for r in rows], np.uint32)
    t = np.array([r[3] if len(r) > 3 else 0.0 for r in rows])
    ends = np.array(layer_end or [len(rows)], np.int64)
    return Circuit(n, g, a, b, t, ends, eps, "hand")


def test_hand_count_expanding_then_clifford_groups():
    # U_0 = Rz(0.3) H on qubit 0: column Z of the composed matrix has two nonzeros, so Z_0
    # gives 2 images and Z_1 (identity on qubit 0) gives 1. V_0 = CX(0,1) sees 2 and 1 terms,
    # U_1 = H(1) (Clifford) sees 2 and 1 terms again: 6 and 3.
    c = _circ(2, [(Gate.H, 0), (Gate.RZ, 0, 0, 0.3), (Gate.CX, 0, 1), (Gate.H, 1)])
    assert definition_updates(c).tolist() == [6, 3]


def test_hand_count_two_wires_one_group():
    # one U_0 with Rx on qubit 0 and Ry on qubit 1: each Z_j meets one rotation whose Z column
    # has two nonzeros (the other wire holds I): 2 images each, once for the whole group
    c = _circ(2, [(Gate.RX, 0, 0, 0.4), (Gate.RY, 1, 1, 1.1)])
    assert definition_updates(c).tolist() == [2, 2]


def test_hand_count_identity_chain_is_no_operator():
    # S then S^dagger on qubit 0 compose to the identity: no operator, no updates; the CX
    # group then sees one term per generator
    c = _circ(2, [(Gate.S, 0), (Gate.SDG, 0), (Gate.CX, 0, 1)])
    assert definition_updates(c).tolist() == [1, 1]


def test_hand_count_layers_and_ansatz_closed_form():
    # the ansatz layer (Rx, Ry, Rz per qubit, then a CX ladder) on n qubits: layer 1 gives 3
    # images per generator, the ladder sees 3 terms each: 6n updates
    n = 5
    rows = []
    for q in range(n):
        rows += [(Gate.RX, q, q, 0.3 + q), (Gate.RY, q, q, 0.7 + q), (Gate.RZ, q, q, 1.3 + q)]
    rows += [(Gate.CX, q, q + 1) for q in range(n - 1)]
    c = _circ(n, rows)
    assert definition_updates(c).tolist() == [6] * n
    assert math.isclose(float(definition_updates(c).sum()), 6 * n)


def test_hand_count_two_qubit_rotations_and_fusion():
    # V_0 = RZZ(0,1) then RXX(0,1): one fused operator. Z_0 (ZI) commutes with ZZ and
    # anticommutes with XX: the fused column of ZI holds 2 nonzeros; Z_1 (IZ) likewise: 2 and 2.
    # Then U_1 = H(0) (Clifford) sees 2 terms each: 4 and 4.
    c = _circ(2, [(Gate.RZZ, 0, 1, 0.7), (Gate.RXX, 1, 0, 0.2), (Gate.H, 0)])
    assert definition_updates(c).tolist() == [4, 4]


def test_hand_count_rotations_on_other_pairs_count_one_by_one():
    # V_0 = RZZ(0,1), ISWAP(1,2), RXX(1,2): the ISWAP and the RXX fuse into one operator on
    # (1, 2); the group is non-Clifford, so each of its two operators counts its images.
    # Z_0: RZZ keeps it (1 image), and it holds I on (1, 2) (1 image): 2. Z_1: RZZ keeps it
    # (1); the ISWAP moves its Z to wire 2, where it anticommutes with XX (2 images): 3.
    # Z_2: 1, then the ISWAP moves its Z to wire 1 (2 images): 3.
    c = _circ(3, [(Gate.RZZ, 0, 1, 0.7), (Gate.ISWAP, 1, 2), (Gate.RXX, 1, 2, 0.4)])
    assert definition_updates(c).tolist() == [2, 3, 3]
