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
    k = np.ascontiguousarray(keys)
    return k.view(np.dtype((np.void, k.dtype.itemsize * k.shape[1]))).reshape(-1)


def fp32_relative_errors(g32, g64):
    """Per generator ||w32 - w64||_2 / ||w64||_2 over the union of keys, and the max |dw|."""
    o32, k32, w32 = g32
    o64, k64, w64 = g64
    rel, mx = [], 0.0
    for j in range(len(o64) - 1):
        a = _key_rows(k32[int(o32[j]):int(o32[j + 1])]); wa = w32[int(o32[j]):int(o32[j + 1])]
        b = _key_rows(k64[int(o64[j]):int(o64[j + 1])]); wb = w64[int(o64[j]):int(o64[j + 1])]
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
    for j in range(len(o64) - 1):
        a32, b32 = int(o32[j]), int(o32[j + 1])
        a64, b64 = int(o64[j]), int(o64[j + 1])
        s32 = _key_rows(k32[a32:b32][np.abs(w32[a32:b32]) > tau])
        m64 = np.abs(w64[a64:b64]) > tau
        s64 = _key_rows(k64[a64:b64][m64])
        only = np.setxor1d(s32, s64, assume_unique=True)
        if only.size:
            allk = _key_rows(k64[a64:b64])
            order = np.argsort(allk)  # byte order of the rows, which numeric order need not be
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
