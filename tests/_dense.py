"""Dense reference computations for small n (test helper, numpy only).

Built from the gates' unitary matrices, independently of the oracle: the full
unitary U of a circuit, the statevector U|0^n>, the Pauli decomposition
w_a = 2^-n Tr(P_a M) of a matrix, and Pauli strings applied to a statevector.
Qubit 0 is the leftmost tensor factor (the most significant bit of a basis index).
"""
from __future__ import annotations

import math

import numpy as np

from paper_2505_03307_amd.workloads import TWO_QUBIT, Gate

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
PAULI = [I2, PX, PY, PZ]  # codes I=0, X=1, Y=2, Z=3


def unitary_1q(code: int, theta: float = 0.0) -> np.ndarray:
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    g = Gate(code)
    if g == Gate.H:
        return np.array([[1, 1], [1, -1]], dtype=complex) / math.sqrt(2)
    if g == Gate.S:
        return np.diag([1, 1j])
    if g == Gate.SDG:
        return np.diag([1, -1j])
    if g == Gate.T:
        return np.diag([1, np.exp(1j * math.pi / 4)])
    if g == Gate.TDG:
        return np.diag([1, np.exp(-1j * math.pi / 4)])
    if g == Gate.SX:
        return 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]])
    if g == Gate.X:
        return PX.copy()
    if g == Gate.Y:
        return PY.copy()
    if g == Gate.Z:
        return PZ.copy()
    if g == Gate.RX:
        return np.array([[c, -1j * s], [-1j * s, c]])
    if g == Gate.RY:
        return np.array([[c, -s], [s, c]], dtype=complex)
    if g == Gate.RZ:
        return np.diag([np.exp(-1j * theta / 2), np.exp(1j * theta / 2)])
    raise ValueError(code)


def unitary_2q(code: int, theta: float = 0.0) -> np.ndarray:
    """4x4 unitary on (q0, q1), basis |q0 q1>, q0 the more significant bit."""
    g = Gate(code)
    if g == Gate.CX:
        return np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
    if g == Gate.CZ:
        return np.diag([1, 1, 1, -1]).astype(complex)
    if g == Gate.ISWAP:
        return np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]], dtype=complex)
    if g in (Gate.RXX, Gate.RYY, Gate.RZZ):
        P = {Gate.RXX: PX, Gate.RYY: PY, Gate.RZZ: PZ}[g]
        return math.cos(theta / 2) * np.eye(4) - 1j * math.sin(theta / 2) * np.kron(P, P)
    raise ValueError(code)


def ptm_from_unitary(U: np.ndarray) -> np.ndarray:
    """R[a][b] = (1/d) Tr(P_a U P_b U^dagger) over the Pauli basis of 1 or 2 qubits."""
    d = U.shape[0]
    k = int(round(math.log2(d)))
    basis = []
    for idx in range(4 ** k):
        digits = [(idx >> (2 * (k - 1 - i))) & 3 for i in range(k)]
        M = np.array([[1.0 + 0j]])
        for dg in digits:
            M = np.kron(M, PAULI[dg])
        basis.append(M)
    R = np.zeros((4 ** k, 4 ** k))
    for b, Pb in enumerate(basis):
        img = U @ Pb @ U.conj().T
        for a, Pa in enumerate(basis):
            R[a, b] = np.real(np.trace(Pa @ img)) / d
    return R


def _apply_1q_state(psi: np.ndarray, n: int, q: int, U: np.ndarray) -> np.ndarray:
    t = psi.reshape([2] * n)
    t = np.moveaxis(np.tensordot(U, t, axes=([1], [q])), 0, q)
    return t.reshape(-1)


def _apply_2q_state(psi: np.ndarray, n: int, a: int, b: int, U: np.ndarray) -> np.ndarray:
    t = psi.reshape([2] * n)
    U4 = U.reshape(2, 2, 2, 2)
    t = np.tensordot(U4, t, axes=([2, 3], [a, b]))
    t = np.moveaxis(t, [0, 1], [a, b])
    return t.reshape(-1)


def apply_circuit_state(circuit, psi: np.ndarray) -> np.ndarray:
    n = circuit.n
    for i in range(circuit.m):
        code = int(circuit.gate[i])
        a, b, th = int(circuit.q0[i]), int(circuit.q1[i]), float(circuit.theta[i])
        if Gate(code) in TWO_QUBIT:
            psi = _apply_2q_state(psi, n, a, b, unitary_2q(code, th))
        else:
            psi = _apply_1q_state(psi, n, a, unitary_1q(code, th))
    return psi


def statevector(circuit) -> np.ndarray:
    psi = np.zeros(2 ** circuit.n, dtype=complex)
    psi[0] = 1.0
    return apply_circuit_state(circuit, psi)


def full_unitary(circuit) -> np.ndarray:
    n = circuit.n
    D = 2 ** n
    cols = np.eye(D, dtype=complex)
    out = np.empty((D, D), dtype=complex)
    for j in range(D):
        out[:, j] = apply_circuit_state(circuit, cols[:, j].copy())
    return out


def pauli_string_matrix(digits) -> np.ndarray:
    M = np.array([[1.0 + 0j]])
    for dg in digits:
        M = np.kron(M, PAULI[dg])
    return M


def pauli_decompose(M: np.ndarray, n: int) -> np.ndarray:
    """c[idx] = 2^-n Tr(P_idx M), idx the base-4 index with qubit 0 most significant."""
    t = M.reshape([2] * (2 * n))  # axes: i_0..i_{n-1}, j_0..j_{n-1}
    # S[a, j, i] = (P_a)_{j i}; contracting Tr(P M) = sum_{i,j} (P)_{j i} M_{i j}
    S = np.stack(PAULI)  # (4, 2, 2) indexed [a, row, col]
    for q in range(n):
        # current layout: (done digits a_0..a_{q-1}, i_q..i_{n-1}, j_q..j_{n-1})
        nq = n - q
        iq_axis = q
        jq_axis = q + nq
        t = np.tensordot(t, S, axes=([iq_axis, jq_axis], [2, 1]))
        # new axis a_q is last; move it to position q
        t = np.moveaxis(t, -1, q)
    return (t.reshape(-1) / 2 ** n)


def apply_pauli_state(psi: np.ndarray, n: int, digits) -> np.ndarray:
    for q, dg in enumerate(digits):
        if dg:
            psi = _apply_1q_state(psi, n, q, PAULI[dg])
    return psi


def index_to_digits(idx: int, n: int):
    return [(idx >> (2 * (n - 1 - q))) & 3 for q in range(n)]
