"""Key conversions used by the tests (test helper).

The external key format is the paper's base-4 index (Sec. III-B): digit d_j of
qubit j in {I=0, X=1, Y=2, Z=3}, index = sum_j d_j 4^(n-1-j). For n <= 32 it fits
one uint64 word; for 32 < n <= 64 it takes two words, word 0 the low 64 bits.
The oracle reports (x, z) bit words; these helpers put both sides in the same form.
"""
from __future__ import annotations

import numpy as np

LETTER = "IXYZ"


def words_for(n: int) -> int:
    return 1 if n <= 32 else 2


def xz_to_index(x: np.ndarray, z: np.ndarray, n: int) -> np.ndarray:
    """(x, z) bit words -> (T, W) uint64 paper-index words."""
    x = np.asarray(x, dtype=np.uint64)
    z = np.asarray(z, dtype=np.uint64)
    W = words_for(n)
    out = np.zeros((x.shape[0], W), dtype=np.uint64)
    one = np.uint64(1)
    for q in range(n):
        xb = (x >> np.uint64(q)) & one
        zb = (z >> np.uint64(q)) & one
        digit = (zb << one) | (xb ^ zb)  # I=0, X=1, Y=2, Z=3
        pos = 2 * (n - 1 - q)
        out[:, pos // 64] |= digit << np.uint64(pos % 64)
    return out


def string_to_xz(s: str):
    x = z = 0
    for q, ch in enumerate(s):
        d = LETTER.index(ch)
        if d in (1, 2):
            x |= 1 << q
        if d in (2, 3):
            z |= 1 << q
    return x, z


def string_to_index(s: str) -> int:
    idx = 0
    for ch in s:
        idx = idx * 4 + LETTER.index(ch)
    return idx


def index_words_to_int(words: np.ndarray) -> list[int]:
    words = np.asarray(words, dtype=np.uint64)
    if words.ndim == 1:
        words = words[:, None]
    out = []
    for row in words:
        v = 0
        for k, wd in enumerate(row.tolist()):
            v |= int(wd) << (64 * k)
        out.append(v)
    return out


def index_to_string(idx: int, n: int) -> str:
    return "".join(LETTER[(idx >> (2 * (n - 1 - q))) & 3] for q in range(n))


def xz_to_strings(x, z, n: int) -> list[str]:
    out = []
    for xv, zv in zip(np.asarray(x).tolist(), np.asarray(z).tolist()):
        s = []
        for q in range(n):
            xb, zb = (int(xv) >> q) & 1, (int(zv) >> q) & 1
            s.append("IXYZ"[(zb << 1) | (xb ^ zb)])
        out.append("".join(s))
    return out


def oracle_generator_dict(o, g: int) -> dict[str, float]:
    x, z, w = o.read(g)
    return dict(zip(xz_to_strings(x, z, o.n), w.tolist()))
