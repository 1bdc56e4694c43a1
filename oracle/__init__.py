"""CPU oracle for generator propagation -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package. The product path (``paper_2505_03307_amd``) never does,
and the two share no code: this wrapper only marshals arrays into the plain C++
oracle in ``oracle.cpp`` (see its header for what is computed and from which
passages of the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QIMAX_ORACLE_LIB may name another build of oracle.cpp (used to check that the pins reject
# deliberately broken copies of the oracle).
LIB_PATH = os.environ.get("QIMAX_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.cpp")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with the host compiler (no GPU code)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC_PATH]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    u64p = ctypes.POINTER(ctypes.c_uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_new.restype = P
    lib.oracle_new.argtypes = [ctypes.c_int]
    lib.oracle_new_subset.restype = P
    lib.oracle_new_subset.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.oracle_new_terms.restype = P
    lib.oracle_new_terms.argtypes = [ctypes.c_int, ctypes.c_int, u64p, u64p, u64p, dp]
    lib.oracle_free.argtypes = [P]
    lib.oracle_num_gens.argtypes = [P]
    lib.oracle_gate.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.oracle_ptm1.argtypes = [P, ctypes.c_int, dp]
    lib.oracle_ptm2.argtypes = [P, ctypes.c_int, ctypes.c_int, dp]
    lib.oracle_prune.argtypes = [P, ctypes.c_double]
    lib.oracle_run.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint8),
                               ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32), dp,
                               ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64), ctypes.c_double,
                               ctypes.c_int]
    lib.oracle_gates.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint32),
                                 ctypes.POINTER(ctypes.c_uint32), dp, ctypes.c_int]
    lib.oracle_fanout_sum.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_uint8),
                                      u64p]
    lib.oracle_fanout_sum.restype = None
    lib.oracle_fanout_sum2.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8), u64p]
    lib.oracle_fanout_sum2.restype = None
    lib.oracle_count.restype = ctypes.c_size_t
    lib.oracle_count.argtypes = [P, ctypes.c_int]
    lib.oracle_gen_id.argtypes = [P, ctypes.c_int]
    lib.oracle_read.argtypes = [P, ctypes.c_int, u64p, u64p, dp]
    lib.oracle_gate_ptm.argtypes = [ctypes.c_int, ctypes.c_double, dp]
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class OracleError(RuntimeError):
    pass


class Oracle:
    """Generators of |0^n> (or a subset of them, or arbitrary start terms)."""

    def __init__(self, n: int, gens=None, *, _handle=None):
        lib = _load()
        self.n = n
        if _handle is not None:
            h = _handle
        elif gens is None:
            h = lib.oracle_new(n)
        else:
            g = np.ascontiguousarray(gens, dtype=np.int32)
            h = lib.oracle_new_subset(n, int(g.size), _ptr(g, ctypes.c_int))
        if not h:
            raise OracleError(f"oracle_new failed for n={n}")
        self._h = ctypes.c_void_p(h)

    @classmethod
    def from_terms(cls, n: int, terms_per_gen):
        """terms_per_gen: list (one per generator) of lists of (x, z, w)."""
        off = [0]
        xs, zs, ws = [], [], []
        for terms in terms_per_gen:
            for x, z, w in terms:
                xs.append(x); zs.append(z); ws.append(w)
            off.append(len(xs))
        off = np.array(off, dtype=np.uint64)
        xs = np.array(xs, dtype=np.uint64); zs = np.array(zs, dtype=np.uint64)
        ws = np.array(ws, dtype=np.float64)
        lib = _load()
        h = lib.oracle_new_terms(n, len(terms_per_gen), _ptr(off, ctypes.c_uint64),
                                 _ptr(xs, ctypes.c_uint64), _ptr(zs, ctypes.c_uint64),
                                 _ptr(ws, ctypes.c_double))
        return cls(n, _handle=h)

    def close(self):
        if self._h:
            _load().oracle_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_gens(self) -> int:
        return _load().oracle_num_gens(self._h)

    def gate(self, code: int, q0: int, q1: int | None = None, theta: float = 0.0):
        if q1 is None:
            q1 = q0
        if _load().oracle_gate(self._h, int(code), int(q0), int(q1), float(theta)) != 0:
            raise OracleError("invalid gate")

    def ptm1(self, q: int, R: np.ndarray):
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(4, 4)
        if _load().oracle_ptm1(self._h, int(q), _ptr(R, ctypes.c_double)) != 0:
            raise OracleError("invalid ptm1")

    def ptm2(self, q0: int, q1: int, R: np.ndarray):
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(16, 16)
        if _load().oracle_ptm2(self._h, int(q0), int(q1), _ptr(R, ctypes.c_double)) != 0:
            raise OracleError("invalid ptm2")

    def prune(self, eps: float):
        _load().oracle_prune(self._h, float(eps))

    def run(self, circuit, threads: int = 0):
        """Propagate through every layer of a workloads.Circuit (prune at each layer end)."""
        g = np.ascontiguousarray(circuit.gate, dtype=np.uint8)
        a = np.ascontiguousarray(circuit.q0, dtype=np.uint32)
        b = np.ascontiguousarray(circuit.q1, dtype=np.uint32)
        t = np.ascontiguousarray(circuit.theta, dtype=np.float64)
        ends = np.ascontiguousarray(circuit.layer_end, dtype=np.int64)
        rc = _load().oracle_run(self._h, g.size, _ptr(g, ctypes.c_uint8), _ptr(a, ctypes.c_uint32),
                                _ptr(b, ctypes.c_uint32), _ptr(t, ctypes.c_double), ends.size,
                                _ptr(ends, ctypes.c_int64), float(circuit.eps), int(threads))
        if rc != 0:
            raise OracleError("oracle_run rejected the circuit")
        return self

    def gates(self, gate, q0, q1, theta, threads: int = 0):
        """Apply a list of gates to every generator in order (no prune)."""
        g = np.ascontiguousarray(gate, dtype=np.uint8)
        a = np.ascontiguousarray(q0, dtype=np.uint32)
        b = np.ascontiguousarray(q1, dtype=np.uint32)
        t = np.ascontiguousarray(theta, dtype=np.float64)
        if _load().oracle_gates(self._h, g.size, _ptr(g, ctypes.c_uint8), _ptr(a, ctypes.c_uint32),
                                _ptr(b, ctypes.c_uint32), _ptr(t, ctypes.c_double), int(threads)) != 0:
            raise OracleError("oracle_gates rejected the gates")
        return self

    def fanout_sum(self, wires, nnz) -> np.ndarray:
        """Per generator: sum over terms of prod_i nnz[i][Pauli of the term on wires[i]]."""
        w = np.ascontiguousarray(wires, dtype=np.int32)
        z = np.ascontiguousarray(nnz, dtype=np.uint8).reshape(-1)
        assert z.size == 4 * w.size
        out = np.zeros(self.num_gens, dtype=np.uint64)
        _load().oracle_fanout_sum(self._h, int(w.size), _ptr(w, ctypes.c_int), _ptr(z, ctypes.c_uint8),
                                  _ptr(out, ctypes.c_uint64))
        return out

    def fanout_sum2(self, a: int, b: int, nnz16) -> np.ndarray:
        """Per generator: sum over terms of nnz16[4 p_a + p_b] (a two-qubit operator's columns)."""
        z = np.ascontiguousarray(nnz16, dtype=np.uint8).reshape(-1)
        assert z.size == 16
        out = np.zeros(self.num_gens, dtype=np.uint64)
        _load().oracle_fanout_sum2(self._h, int(a), int(b), _ptr(z, ctypes.c_uint8), _ptr(out, ctypes.c_uint64))
        return out

    def count(self, g: int) -> int:
        return int(_load().oracle_count(self._h, int(g)))

    def counts(self) -> np.ndarray:
        return np.array([self.count(g) for g in range(self.num_gens)], dtype=np.int64)

    def gen_id(self, g: int) -> int:
        return int(_load().oracle_gen_id(self._h, int(g)))

    def read(self, g: int):
        """(x, z, w) of generator slot g, ascending by the paper's base-4 index."""
        c = self.count(g)
        x = np.empty(c, dtype=np.uint64); z = np.empty(c, dtype=np.uint64)
        w = np.empty(c, dtype=np.float64)
        _load().oracle_read(self._h, int(g), _ptr(x, ctypes.c_uint64), _ptr(z, ctypes.c_uint64),
                            _ptr(w, ctypes.c_double))
        return x, z, w


def gate_ptm(code: int, theta: float = 0.0) -> np.ndarray:
    """The oracle's transfer matrix for a gate, R[out][in] (4x4 or 16x16)."""
    R = np.zeros(256, dtype=np.float64)
    d = _load().oracle_gate_ptm(int(code), float(theta), _ptr(R, ctypes.c_double))
    if d == 0:
        raise OracleError(f"unknown gate {code}")
    return R[: d * d].reshape(d, d).copy()


def propagate(circuit, gens=None, threads: int = 0) -> Oracle:
    """Convenience: the oracle state after the whole circuit."""
    o = Oracle(circuit.n, gens)
    o.run(circuit, threads)
    return o
