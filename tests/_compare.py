"""GPU-vs-oracle comparison contract (test helper).

FP64: on the significant set K_tau = {keys with |w| > tau}, tau = 1e-12, keys must match
bit for bit (and so must |K_tau|), weights within `tol`. Residue keys with |w| <= tau may
appear on either side (summation order differs between the two implementations); they are
counted. With raw_exact=True the complete key sets must be identical.
FP32 vs FP64: per generator ||w32 - w64||_2 / ||w64||_2 <= rel on the union of keys.
"""
from __future__ import annotations

import numpy as np

from _keys import xz_to_index


def oracle_arrays(o, n):
    """(gen_off, keys [T, W], w) from an oracle state, keys as paper-index words."""
    offs, ks, ws = [0], [], []
    for g in range(o.num_gens):
        x, z, w = o.read(g)
        ks.append(xz_to_index(x, z, n))
        ws.append(w)
        offs.append(offs[-1] + len(w))
    W = 1 if n <= 32 else 2
    keys = np.concatenate(ks) if ks else np.zeros((0, W), np.uint64)
    return np.array(offs, dtype=np.uint64), keys, (np.concatenate(ws) if ws else np.zeros(0))


def compare_fp64(gpu, ref, tau=1e-12, tol=1e-12, raw_exact=False, gens=None, label=""):
    """gpu, ref: (gen_off, keys, w). gens: generator ids of ref's slots (None = all)."""
    g_off, g_keys, g_w = gpu
    r_off, r_keys, r_w = ref
    n_ref = len(r_off) - 1
    gens = list(range(n_ref)) if gens is None else list(gens)
    residues = 0
    worst = 0.0
    for slot, j in enumerate(gens):
        ga, gb = int(g_off[j]), int(g_off[j + 1])
        ra, rb = int(r_off[slot]), int(r_off[slot + 1])
        gk, gw = g_keys[ga:gb], g_w[ga:gb]
        rk, rw = r_keys[ra:rb], r_w[ra:rb]
        if raw_exact:
            assert gk.shape == rk.shape, f"{label} gen {j}: {gk.shape[0]} vs {rk.shape[0]} terms"
            assert np.array_equal(gk, rk), f"{label} gen {j}: raw key sets differ"
        gm = np.abs(gw) > tau
        rm = np.abs(rw) > tau
        residues += int((~gm).sum() + (~rm).sum())
        gk_s, rk_s = gk[gm], rk[rm]
        assert gk_s.shape == rk_s.shape, f"{label} gen {j}: |K_tau| {gk_s.shape[0]} vs {rk_s.shape[0]}"
        assert np.array_equal(gk_s, rk_s), f"{label} gen {j}: significant keys differ"
        if gk_s.shape[0]:
            d = float(np.max(np.abs(gw[gm] - rw[rm])))
            worst = max(worst, d)
            assert d <= tol, f"{label} gen {j}: max |dw| = {d:.3e} > {tol:.1e}"
    return {"residues": residues, "max_abs_dw": worst}


def _key_rows(keys):
    """One comparable value per key row: the word itself for one-word keys (numeric order, fast
    set operations), else the row's bytes (an order of its own, consistent for set operations)."""
    k = np.ascontiguousarray(keys)
    if k.shape[1] == 1:
        return k[:, 0]
    return k.view(np.dtype((np.void, k.dtype.itemsize * k.shape[1]))).reshape(-1)


def _diff_sorted(a, wa, b, wb):
    """||wa - wb||_2^2 over the union of two ascending key arrays (a missing key weighs 0), and
    max |dw|, by searching a's keys in b."""
    if b.size == 0:
        return float(np.sum(wa * wa)), float(np.max(np.abs(wa), initial=0.0))
    pos = np.minimum(np.searchsorted(b, a), b.size - 1)
    hit = b[pos] == a
    dv = wa[hit] - wb[pos[hit]]
    hitb = np.zeros(b.size, dtype=bool)
    hitb[pos[hit]] = True
    only_a, only_b = wa[~hit], wb[~hitb]
    d2 = float(np.sum(dv * dv) + np.sum(only_a * only_a) + np.sum(only_b * only_b))
    mx = max(float(np.max(np.abs(dv), initial=0.0)), float(np.max(np.abs(only_a), initial=0.0)),
             float(np.max(np.abs(only_b), initial=0.0)))
    return d2, mx


def fp32_relative_errors(g32, g64):
    """Per generator ||w32 - w64||_2 / ||w64||_2 over the union of keys, and the max |dw|."""
    o32, k32, w32 = g32
    o64, k64, w64 = g64
    if k32.shape[1] == 1 and np.array_equal(o32, o64) and np.array_equal(k32, k64):
        # the same keys in the same order: per generator sums in one sweep
        starts = o64[:-1].astype(np.int64)
        d = w32 - w64
        nonempty = starts < o64[1:].astype(np.int64)
        d2 = np.zeros(len(starts)); r2 = np.zeros(len(starts))
        if d.size:
            d2[nonempty] = np.add.reduceat(d * d, starts[nonempty])
            r2[nonempty] = np.add.reduceat(w64 * w64, starts[nonempty])
        r = np.sqrt(r2)
        return np.sqrt(d2) / np.where(r > 0, r, 1.0), float(np.max(np.abs(d), initial=0.0))
    rel, mx = [], 0.0
    for j in range(len(o64) - 1):
        a = _key_rows(k32[int(o32[j]):int(o32[j + 1])]); wa = w32[int(o32[j]):int(o32[j + 1])]
        b = _key_rows(k64[int(o64[j]):int(o64[j + 1])]); wb = w64[int(o64[j]):int(o64[j + 1])]
        if a.dtype == np.uint64:  # one-word keys, ascending: search instead of a union
            d2, m = _diff_sorted(a, wa, b, wb)
            nrm = float(np.linalg.norm(wb))
            rel.append(d2 ** 0.5 / (nrm if nrm > 0 else 1.0))
            mx = max(mx, m)
            continue
        allk = np.union1d(a, b)
        va = np.zeros(allk.shape[0]); vb = np.zeros(allk.shape[0])
        va[np.searchsorted(allk, a)] = wa
        vb[np.searchsorted(allk, b)] = wb
        nrm = float(np.linalg.norm(vb))
        rel.append(float(np.linalg.norm(va - vb)) / (nrm if nrm > 0 else 1.0))
        if allk.shape[0]:
            mx = max(mx, float(np.max(np.abs(va - vb))))
    return np.array(rel), mx


def fp32_contract(g32, g64, eps, rel_tol=5e-6, tau_min=1e-6, delta=1e-9):
    """The FP32-vs-FP64 contract, per generator: ||w32 - w64||_2 / ||w64||_2 <= rel_tol over the
    union of keys; on K_tau = {|w| > tau}, tau = max(eps, tau_min), the key sets are equal
    except for straddlers, keys on one side only whose FP64 weight lies within delta of tau
    (rounding decides them). Returns (per-generator rel errors, straddlers, max |dw|)."""
    rel, mx = fp32_relative_errors(g32, g64)
    tau = max(eps, tau_min)
    o32, k32, w32 = g32
    o64, k64, w64 = g64
    straddlers = 0
    m32, m64 = np.abs(w32) > tau, np.abs(w64) > tau
    c32 = np.add.reduceat(m32, o32[:-1].astype(np.int64)) if m32.size else np.zeros(len(o32) - 1)
    c64 = np.add.reduceat(m64, o64[:-1].astype(np.int64)) if m64.size else np.zeros(len(o64) - 1)
    empty32, empty64 = o32[:-1] == o32[1:], o64[:-1] == o64[1:]
    c32 = np.where(empty32, 0, c32); c64 = np.where(empty64, 0, c64)
    if np.array_equal(c32, c64) and np.array_equal(k32[m32], k64[m64]):
        # K_tau identical for every generator: no straddlers
        assert float(rel.max(initial=0.0)) <= rel_tol, f"FP32 rel err {float(rel.max()):.3e} > {rel_tol}"
        return rel, 0, mx
    for j in range(len(o64) - 1):
        a32, b32 = int(o32[j]), int(o32[j + 1])
        a64, b64 = int(o64[j]), int(o64[j + 1])
        s32 = _key_rows(k32[a32:b32][np.abs(w32[a32:b32]) > tau])
        m64 = np.abs(w64[a64:b64]) > tau
        s64 = _key_rows(k64[a64:b64][m64])
        if s32.shape == s64.shape and np.array_equal(s32, s64):
            continue
        only = np.setxor1d(s32, s64, assume_unique=True)
        if only.size:
            allk = _key_rows(k64[a64:b64])
            order = np.argsort(allk, kind="stable")  # (byte order for two-word keys: not the numeric one)
            allk, wk = allk[order], w64[a64:b64][order]
            w_at = np.zeros(only.size)  # FP64 weight of each such key (0 when FP64 has no such key)
            if allk.size:
                pos = np.minimum(np.searchsorted(allk, only), allk.size - 1)
                hit = allk[pos] == only
                w_at[hit] = wk[pos[hit]]
            off = np.abs(np.abs(w_at) - tau)
            assert np.all(off <= delta), f"gen {j}: {int(np.sum(off > delta))} keys differ on K_tau beyond rounding"
            straddlers += int(only.size)
    assert float(rel.max(initial=0.0)) <= rel_tol, f"FP32 rel err {float(rel.max()):.3e} > {rel_tol}"
    return rel, straddlers, mx
