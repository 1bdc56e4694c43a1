"""Thin Python binding of libqimax.so (argument marshalling only).

Every step of the propagation runs in the HIP library; this module converts numpy
arrays to pointers and status codes to exceptions. It never falls back to any other
implementation: if the library is not built, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# QIMAX_LIB may name another build of the library (experiments with build variants)
LIB_PATH = os.environ.get("QIMAX_LIB") or os.path.join(_HERE, "libqimax.so")

STATUS = {0: "QIMAX_OK", -1: "QIMAX_EINVAL", -2: "QIMAX_ENOMEM", -3: "QIMAX_EDEVICE",
          -4: "QIMAX_ETOOLARGE", -5: "QIMAX_ESTATE"}


class QimaxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("fp32_merge", ctypes.c_int), ("prune_eps", ctypes.c_double),
                ("mem_cap_bytes", ctypes.c_size_t), ("hip_stream", ctypes.c_void_p), ("validate", ctypes.c_int),
                ("device", ctypes.c_int)]


class Op(ctypes.Structure):
    _fields_ = [("arity", ctypes.c_uint32), ("q", ctypes.c_uint32 * 2), ("ptm", ctypes.POINTER(ctypes.c_double))]


class Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("terms", "passes", "term_updates", "images", "sort_elems", "peak_bytes", "alloc_bytes")] + \
               [("host_wait_ms", ctypes.c_double), ("host_busy_ms", ctypes.c_double), ("syncs", ctypes.c_uint64),
                ("sort_redos", ctypes.c_uint64), ("tuned_classes", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("alg_bytes", ctypes.c_double)]


class TuneEntry(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint32) for k in ("key_bytes", "weight_bits", "log2_images", "dense_candidate")] + \
               [("best", ctypes.c_int32), ("tried", ctypes.c_uint32), ("ms", ctypes.c_float * 6)]


class CircuitC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("gate", ctypes.POINTER(ctypes.c_uint8)), ("q0", ctypes.POINTER(ctypes.c_uint32)),
                ("q1", ctypes.POINTER(ctypes.c_uint32)), ("theta", ctypes.POINTER(ctypes.c_double)),
                ("m", ctypes.c_size_t), ("layer_end", ctypes.POINTER(ctypes.c_uint64)), ("n_layers", ctypes.c_size_t),
                ("prune_eps", ctypes.c_double)]


class StepGraph:
    """A recorded step (qimax_graph): launch() replays it on the simulator's stream."""

    def __init__(self, sim: "Simulator", handle):
        self.sim = sim
        self._g = handle

    def launch(self):
        self.sim._check(load().qimax_graph_launch(self._g))
        return self

    def close(self):
        if self._g:
            load().qimax_graph_destroy(self._g)
            self._g = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class BatchInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in
                ("queued", "active", "finished", "rounds", "terms", "term_updates", "alloc_bytes", "peak_bytes")]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double)]


EXPORTS = ["qimax_batch_create", "qimax_batch_submit", "qimax_batch_step", "qimax_batch_run", "qimax_batch_poll",
           "qimax_batch_fetch", "qimax_batch_info", "qimax_batch_circuit_updates", "qimax_batch_context",
           "qimax_batch_last_error", "qimax_batch_destroy",
           "qimax_default_opts", "qimax_create", "qimax_reset", "qimax_flush", "qimax_graph_record", "qimax_graph_launch", "qimax_graph_destroy", "qimax_get_generator_updates", "qimax_apply_layer", "qimax_apply_circuit", "qimax_group_circuit",
           "qimax_num_terms", "qimax_get_generators", "qimax_get_generators_xz", "qimax_expect",
           "qimax_expect_many", "qimax_prob_zero_all", "qimax_compare", "qimax_compare_noalloc", "qimax_get_stats", "qimax_get_tuning", "qimax_sync",
           "qimax_profile", "qimax_profile_only", "qimax_profile_read", "qimax_copy_probe", "qimax_last_error", "qimax_destroy"]

_lib = None


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    szp = ctypes.POINTER(ctypes.c_size_t)
    lib.qimax_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.qimax_default_opts.restype = None
    lib.qimax_create.argtypes = [ctypes.c_uint32, ctypes.POINTER(Opts), ctypes.POINTER(P)]
    lib.qimax_reset.argtypes = [P]
    lib.qimax_flush.argtypes = [P]
    lib.qimax_graph_record.argtypes = [P, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint32),
                                       ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_double),
                                       ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64), ctypes.c_size_t,
                                       ctypes.POINTER(P)]
    lib.qimax_graph_launch.argtypes = [P]
    lib.qimax_graph_destroy.argtypes = [P]
    lib.qimax_graph_destroy.restype = None
    lib.qimax_get_generator_updates.argtypes = [P, u64p, ctypes.c_size_t]
    lib.qimax_apply_layer.argtypes = [P, ctypes.POINTER(Op), ctypes.c_size_t]
    lib.qimax_apply_circuit.argtypes = [P, u8p, u32p, u32p, dp, ctypes.c_size_t]
    lib.qimax_group_circuit.argtypes = [P, u8p, u32p, u32p, dp, ctypes.c_size_t, ctypes.POINTER(Op), dp,
                                        ctypes.c_size_t, szp, szp, szp]
    lib.qimax_num_terms.argtypes = [P, u64p]
    lib.qimax_get_generators.argtypes = [P, u64p, u64p, dp, ctypes.c_size_t, szp]
    lib.qimax_expect.argtypes = [P, ctypes.c_char_p, dp]
    lib.qimax_get_generators_xz.argtypes = [P, u64p, u64p, u64p, dp, ctypes.c_size_t, szp]
    lib.qimax_expect_many.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t, dp]
    lib.qimax_prob_zero_all.argtypes = [P, dp]
    lib.qimax_compare.argtypes = [P, P, ctypes.c_double, dp, dp, u64p]
    lib.qimax_compare_noalloc.argtypes = [P, P, ctypes.c_double, dp, dp, u64p]
    lib.qimax_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.qimax_get_tuning.argtypes = [P, ctypes.POINTER(TuneEntry), ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.qimax_sync.argtypes = [P]
    lib.qimax_profile.argtypes = [P, ctypes.c_int]
    lib.qimax_profile_read.argtypes = [P, ctypes.POINTER(KernelTime), ctypes.c_size_t, szp]
    lib.qimax_copy_probe.argtypes = [ctypes.c_size_t, ctypes.c_int, dp]
    lib.qimax_profile_only.argtypes = [P, ctypes.c_char_p]
    lib.qimax_last_error.argtypes = [P]
    lib.qimax_last_error.restype = ctypes.c_char_p
    lib.qimax_destroy.argtypes = [P]
    lib.qimax_destroy.restype = None
    lib.qimax_batch_create.argtypes = [ctypes.POINTER(Opts), ctypes.c_uint32, ctypes.POINTER(P)]
    lib.qimax_batch_submit.argtypes = [P, ctypes.POINTER(CircuitC), u64p]
    lib.qimax_batch_step.argtypes = [P, szp]
    lib.qimax_batch_run.argtypes = [P]
    lib.qimax_batch_poll.argtypes = [P, u64p, ctypes.c_size_t, szp]
    lib.qimax_batch_fetch.argtypes = [P, ctypes.c_uint64, u64p, u64p, dp, ctypes.c_size_t, szp]
    lib.qimax_batch_info.argtypes = [P, ctypes.POINTER(BatchInfo)]
    lib.qimax_batch_circuit_updates.argtypes = [P, ctypes.c_uint64, u64p]
    lib.qimax_batch_context.argtypes = [P]
    lib.qimax_batch_context.restype = P
    lib.qimax_batch_last_error.argtypes = [P]
    lib.qimax_batch_last_error.restype = ctypes.c_char_p
    lib.qimax_batch_destroy.argtypes = [P]
    lib.qimax_batch_destroy.restype = None
    for name in EXPORTS:
        if name not in ("qimax_default_opts", "qimax_last_error", "qimax_destroy", "qimax_batch_context",
                        "qimax_batch_last_error", "qimax_batch_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _instr(circuit_or_arrays):
    c = circuit_or_arrays
    if isinstance(c, tuple):
        g, a, b, t = c
    else:
        g, a, b, t = c.gate, c.q0, c.q1, c.theta
    return (np.ascontiguousarray(g, dtype=np.uint8), np.ascontiguousarray(a, dtype=np.uint32),
            np.ascontiguousarray(b, dtype=np.uint32), np.ascontiguousarray(t, dtype=np.float64))


class Simulator:
    """The n generators of |0^n> held on the GPU (one qimax context)."""

    def __init__(self, n: int, precision: int = 64, fp32_merge: int = 0, prune_eps: float = 0.0,
                 mem_cap_bytes: int = 0, stream: int | None = None, validate: bool = True, device: int = -1):
        lib = load()
        o = Opts()
        lib.qimax_default_opts(ctypes.byref(o))
        o.precision, o.fp32_merge, o.prune_eps = int(precision), int(fp32_merge), float(prune_eps)
        o.mem_cap_bytes, o.validate, o.device = int(mem_cap_bytes), int(bool(validate)), int(device)
        o.hip_stream = stream
        h = ctypes.c_void_p()
        st = lib.qimax_create(int(n), ctypes.byref(o), ctypes.byref(h))
        if st != 0:
            raise QimaxError(st, lib.qimax_last_error(None).decode())
        self._h = h
        self.n = n
        self.precision = precision

    # -------------------------------------------------------------------------- plumbing
    def _check(self, st: int):
        if st != 0:
            raise QimaxError(st, load().qimax_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            load().qimax_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------------ propagation
    def reset(self):
        """Back to Z_0 .. Z_{n-1}, keeping the device buffers."""
        self._check(load().qimax_reset(self._h))
        return self

    def flush(self):
        """Apply the operators kept back by calls that held only Clifford operators."""
        self._check(load().qimax_flush(self._h))
        return self

    def record_step(self, circuit) -> "StepGraph":
        """Record reset + every layer + flush of a workloads.Circuit as a replayable graph (the
        step runs once while it is recorded). Run the step once before recording."""
        g = np.ascontiguousarray(circuit.gate, dtype=np.uint8)
        a = np.ascontiguousarray(circuit.q0, dtype=np.uint32)
        b = np.ascontiguousarray(circuit.q1, dtype=np.uint32)
        t = np.ascontiguousarray(circuit.theta, dtype=np.float64)
        ends = np.ascontiguousarray(circuit.layer_end, dtype=np.uint64)
        h = ctypes.c_void_p()
        self._check(load().qimax_graph_record(self._h, _p(g, ctypes.c_uint8), _p(a, ctypes.c_uint32),
                                              _p(b, ctypes.c_uint32), _p(t, ctypes.c_double), g.size,
                                              _p(ends, ctypes.c_uint64), ends.size, ctypes.byref(h)))
        return StepGraph(self, h)

    def apply_circuit(self, circuit_or_arrays):
        g, a, b, t = _instr(circuit_or_arrays)
        self._check(load().qimax_apply_circuit(self._h, _p(g, ctypes.c_uint8), _p(a, ctypes.c_uint32),
                                               _p(b, ctypes.c_uint32), _p(t, ctypes.c_double), g.size))
        return self

    def run(self, circuit):
        """Every layer of a workloads.Circuit, one apply call per layer."""
        for a, b in circuit.layers():
            self.apply_circuit((circuit.gate[a:b], circuit.q0[a:b], circuit.q1[a:b], circuit.theta[a:b]))
        return self

    def apply_layer(self, ops):
        """ops: sequence of (qubits, R) with qubits an int or a pair and R 4x4 / 16x16 (R[out][in])."""
        arr = (Op * max(len(ops), 1))()
        keep = []
        for i, (qs, R) in enumerate(ops):
            qs = (qs,) if np.isscalar(qs) else tuple(qs)
            R = np.ascontiguousarray(R, dtype=np.float64)
            keep.append(R)
            arr[i].arity = len(qs)
            arr[i].q[0] = int(qs[0])
            arr[i].q[1] = int(qs[1]) if len(qs) > 1 else int(qs[0])
            arr[i].ptm = _p(R, ctypes.c_double)
        self._check(load().qimax_apply_layer(self._h, arr, len(ops)))
        return self

    def group_counts(self, circuit_or_arrays):
        """(number of grouped operators, K, K') of a circuit: the whole grouping pass runs, only
        the counts come back."""
        g, a, b, t = _instr(circuit_or_arrays)
        n_ops, nu, nv = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        self._check(load().qimax_group_circuit(self._h, _p(g, ctypes.c_uint8), _p(a, ctypes.c_uint32),
                                               _p(b, ctypes.c_uint32), _p(t, ctypes.c_double), g.size, None, None, 0,
                                               ctypes.byref(n_ops), ctypes.byref(nu), ctypes.byref(nv)))
        return n_ops.value, nu.value, nv.value

    def group(self, circuit_or_arrays):
        """The grouped operators (qubits, R) and (K, K') of a circuit, without applying it."""
        g, a, b, t = _instr(circuit_or_arrays)
        lib = load()
        n_ops, nu, nv = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        args = (self._h, _p(g, ctypes.c_uint8), _p(a, ctypes.c_uint32), _p(b, ctypes.c_uint32),
                _p(t, ctypes.c_double), g.size)
        self._check(lib.qimax_group_circuit(*args, None, None, 0, ctypes.byref(n_ops), ctypes.byref(nu),
                                            ctypes.byref(nv)))
        cap = n_ops.value
        ops = (Op * max(cap, 1))()
        buf = np.zeros(256 * max(cap, 1), dtype=np.float64)
        self._check(lib.qimax_group_circuit(*args, ops, _p(buf, ctypes.c_double), cap, ctypes.byref(n_ops),
                                            ctypes.byref(nu), ctypes.byref(nv)))
        out, off = [], 0
        for i in range(cap):
            d = 4 if ops[i].arity == 1 else 16
            R = buf[off:off + d * d].reshape(d, d).copy()
            off += d * d
            qs = (ops[i].q[0],) if ops[i].arity == 1 else (ops[i].q[0], ops[i].q[1])
            out.append((qs, R))
        return out, nu.value, nv.value

    # ---------------------------------------------------------------------------- readout
    def num_terms(self) -> int:
        T = ctypes.c_uint64()
        self._check(load().qimax_num_terms(self._h, ctypes.byref(T)))
        return T.value

    def generators(self):
        """(gen_off [n+1], keys [T, W] uint64 paper-index words, weights [T] float64)."""
        lib = load()
        T = ctypes.c_size_t()
        self._check(lib.qimax_get_generators(self._h, None, None, None, 0, ctypes.byref(T)))
        W = 1 if self.n <= 32 else 2
        off = np.zeros(self.n + 1, dtype=np.uint64)
        keys = np.zeros((max(T.value, 1), W), dtype=np.uint64)
        w = np.zeros(max(T.value, 1), dtype=np.float64)
        self._check(lib.qimax_get_generators(self._h, _p(off, ctypes.c_uint64), _p(keys, ctypes.c_uint64),
                                             _p(w, ctypes.c_double), T.value, ctypes.byref(T)))
        return off, keys[:T.value], w[:T.value]

    def generators_xz(self):
        """(gen_off [n+1], x [T], z [T] uint64 bit words (bit q: qubit q), weights [T] float64)."""
        lib = load()
        T = ctypes.c_size_t()
        off = np.zeros(self.n + 1, dtype=np.uint64)
        self._check(lib.qimax_get_generators_xz(self._h, _p(off, ctypes.c_uint64), None, None, None, 0,
                                                ctypes.byref(T)))
        x = np.zeros(max(T.value, 1), dtype=np.uint64)
        z = np.zeros(max(T.value, 1), dtype=np.uint64)
        w = np.zeros(max(T.value, 1), dtype=np.float64)
        self._check(lib.qimax_get_generators_xz(self._h, _p(off, ctypes.c_uint64), _p(x, ctypes.c_uint64),
                                                _p(z, ctypes.c_uint64), _p(w, ctypes.c_double), T.value,
                                                ctypes.byref(T)))
        return off, x[:T.value], z[:T.value], w[:T.value]

    def expect(self, pauli: str) -> float:
        out = ctypes.c_double()
        self._check(load().qimax_expect(self._h, pauli.encode(), ctypes.byref(out)))
        return out.value

    def expect_many(self, paulis) -> np.ndarray:
        paulis = list(paulis)
        out = np.zeros(max(len(paulis), 1), dtype=np.float64)
        buf = "".join(paulis).encode()
        self._check(load().qimax_expect_many(self._h, buf, len(paulis), _p(out, ctypes.c_double)))
        return out[:len(paulis)]

    def prob_zero_all(self) -> np.ndarray:
        """p_{k,0} = (1 + <Z_k>)/2 for every qubit k."""
        out = np.zeros(self.n, dtype=np.float64)
        self._check(load().qimax_prob_zero_all(self._h, _p(out, ctypes.c_double)))
        return out

    def compare(self, ref: "Simulator", tau: float = 1e-6, no_alloc: bool = False):
        """Per generator (||w_self - w_ref||_2, ||w_ref||_2, keys with |w| > tau on one side only).
        no_alloc: the variant that allocates no device memory (qimax_compare_noalloc)."""
        d = np.zeros(self.n, dtype=np.float64)
        r = np.zeros(self.n, dtype=np.float64)
        k = np.zeros(self.n, dtype=np.uint64)
        fn = load().qimax_compare_noalloc if no_alloc else load().qimax_compare
        self._check(fn(self._h, ref._h, float(tau), _p(d, ctypes.c_double), _p(r, ctypes.c_double),
                       _p(k, ctypes.c_uint64)))
        return d, r, k

    def tuning(self) -> list:
        """The autotuner's size classes and chosen candidates (qimax_get_tuning)."""
        lib = load()
        n = ctypes.c_size_t()
        self._check(lib.qimax_get_tuning(self._h, None, 0, ctypes.byref(n)))
        arr = (TuneEntry * max(n.value, 1))()
        self._check(lib.qimax_get_tuning(self._h, arr, n.value, ctypes.byref(n)))
        return [{"key_bytes": e.key_bytes, "weight_bits": e.weight_bits, "log2_images": e.log2_images,
                 "dense_candidate": bool(e.dense_candidate), "best": e.best, "tried": e.tried,
                 "ms": [round(float(x), 4) for x in e.ms[:5 + e.dense_candidate]]} for e in arr[:n.value]]

    def stats(self) -> dict:
        s = Stats()
        self._check(load().qimax_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def generator_updates(self) -> np.ndarray:
        out = np.zeros(self.n, dtype=np.uint64)
        self._check(load().qimax_get_generator_updates(self._h, _p(out, ctypes.c_uint64), self.n))
        return out

    def sync(self):
        self._check(load().qimax_sync(self._h))

    def profile(self, enable: bool):
        self._check(load().qimax_profile(self._h, int(bool(enable))))

    def profile_only(self, kernel: str | None):
        """Time only one kernel kind (None: all kinds)."""
        self._check(load().qimax_profile_only(self._h, kernel.encode() if kernel else None))

    def profile_read(self) -> dict:
        lib = load()
        arr = (KernelTime * 32)()
        n = ctypes.c_size_t()
        self._check(lib.qimax_profile_read(self._h, arr, 32, ctypes.byref(n)))
        return {arr[i].name.decode(): {"launches": int(arr[i].launches), "total_ms": float(arr[i].total_ms),
                                        "alg_bytes": float(arr[i].alg_bytes)} for i in range(n.value)}


class Batch:
    """Many circuits propagated together (one qimax_batch): every step advances each active
    circuit by one pass in one set of kernel launches; circuits may join at any step."""

    def __init__(self, precision: int = 64, fp32_merge: int = 0, mem_cap_bytes: int = 0, stream: int | None = None,
                 device: int = -1, max_n: int = 32):
        lib = load()
        o = Opts()
        lib.qimax_default_opts(ctypes.byref(o))
        o.precision, o.fp32_merge, o.mem_cap_bytes, o.device = int(precision), int(fp32_merge), int(mem_cap_bytes), int(device)
        o.hip_stream = stream
        h = ctypes.c_void_p()
        st = lib.qimax_batch_create(ctypes.byref(o), int(max_n), ctypes.byref(h))
        if st != 0:
            raise QimaxError(st, lib.qimax_last_error(None).decode())
        self._h = h
        self.precision = precision
        self._n = {}

    def _check(self, st: int):
        if st != 0:
            raise QimaxError(st, load().qimax_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            load().qimax_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, circuit) -> int:
        """Queue a workloads.Circuit (its layers and eps); returns its id."""
        g, a, b, t = _instr(circuit)
        ends = np.ascontiguousarray(circuit.layer_end, dtype=np.uint64)
        cc = CircuitC()
        cc.n = int(circuit.n)
        cc.gate, cc.q0, cc.q1, cc.theta = _p(g, ctypes.c_uint8), _p(a, ctypes.c_uint32), _p(b, ctypes.c_uint32), _p(t, ctypes.c_double)
        cc.m = g.size
        cc.layer_end = _p(ends, ctypes.c_uint64)
        cc.n_layers = ends.size
        cc.prune_eps = float(circuit.eps)
        cid = ctypes.c_uint64()
        self._check(load().qimax_batch_submit(self._h, ctypes.byref(cc), ctypes.byref(cid)))
        self._n[cid.value] = int(circuit.n)
        return cid.value

    def step(self) -> int:
        act = ctypes.c_size_t()
        self._check(load().qimax_batch_step(self._h, ctypes.byref(act)))
        return act.value

    def run(self):
        self._check(load().qimax_batch_run(self._h))
        return self

    def poll(self) -> list:
        lib = load()
        n = ctypes.c_size_t()
        self._check(lib.qimax_batch_poll(self._h, None, 0, ctypes.byref(n)))
        ids = np.zeros(max(n.value, 1), dtype=np.uint64)
        self._check(lib.qimax_batch_poll(self._h, _p(ids, ctypes.c_uint64), ids.size, ctypes.byref(n)))
        return [int(x) for x in ids[:n.value]]

    def fetch(self, cid: int):
        """(gen_off, keys [T, W], weights) of a finished circuit; releases it."""
        lib = load()
        T = ctypes.c_size_t()
        self._check(lib.qimax_batch_fetch(self._h, int(cid), None, None, None, 0, ctypes.byref(T)))
        n = self._n.pop(int(cid))
        off = np.zeros(n + 1, dtype=np.uint64)
        keys = np.zeros((max(T.value, 1), 1 if n <= 32 else 2), dtype=np.uint64)
        w = np.zeros(max(T.value, 1), dtype=np.float64)
        self._check(lib.qimax_batch_fetch(self._h, int(cid), _p(off, ctypes.c_uint64), _p(keys, ctypes.c_uint64),
                                          _p(w, ctypes.c_double), T.value, ctypes.byref(T)))
        return off, keys[:T.value], w[:T.value]

    def info(self) -> dict:
        s = BatchInfo()
        self._check(load().qimax_batch_info(self._h, ctypes.byref(s)))
        return {k: int(getattr(s, k)) for k, _ in BatchInfo._fields_}

    def circuit_updates(self, cid: int) -> int:
        u = ctypes.c_uint64()
        self._check(load().qimax_batch_circuit_updates(self._h, int(cid), ctypes.byref(u)))
        return u.value

    def _ctx(self):
        return load().qimax_batch_context(self._h)

    def sync(self):
        st = load().qimax_sync(self._ctx())
        if st != 0:
            raise QimaxError(st, "sync")

    def profile(self, enable: bool):
        load().qimax_profile(self._ctx(), int(bool(enable)))

    def profile_read(self) -> dict:
        lib = load()
        arr = (KernelTime * 32)()
        n = ctypes.c_size_t()
        lib.qimax_profile_read(self._ctx(), arr, 32, ctypes.byref(n))
        return {arr[i].name.decode(): {"launches": int(arr[i].launches), "total_ms": float(arr[i].total_ms),
                                        "alg_bytes": float(arr[i].alg_bytes)} for i in range(n.value)}


def copy_probe(nbytes: int, reps: int = 5) -> float:
    """Average ms of a plain device copy of nbytes (calibration of traffic counters)."""
    ms = ctypes.c_double()
    st = load().qimax_copy_probe(int(nbytes), int(reps), ctypes.byref(ms))
    if st != 0:
        raise QimaxError(st, "copy probe failed")
    return ms.value
