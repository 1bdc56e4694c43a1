"""Benchmark: Pauli-term updates per second of generator propagation on one MI355X.

Headline workload (one step): the n=32 random Clifford circuit of 200 moments (H, S, CX
drawn uniformly per qubit) with 40 Rz(theta) gates at random slots, seed 0, FP64 weights,
prune eps = 0. A step resets the n generators to Z_j on the device, runs the grouping pass
and every propagation pass, and ends with the final generators resident in HBM (the
paper's timing window, Sec. V). One term update = one output image of one grouped operator
(U_k / V_k run), each group counted once (a Clifford group counts the terms it acts on).
Also measured: the same circuit in FP32, and the n=16 two-layer ansatz (the configuration
whose images merge) in FP64 and FP32 with eps = 1e-9.

Prints one JSON line. The roofline object covers the kernel with the largest share of
device time (found in the warm-up, where every kernel is timed), timed with HIP events on
the library's stream over the timed region, where only that kernel carries events; the
per-kernel breakdown comes from as many extra steps with every kernel timed. The
cpu_baseline object times the CPU oracle (test infrastructure) on a sample of the same
workload on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def traffic_for(kernel: str, workload: str = "c2"):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter summary, if
    it was taken on the current kernels."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        ent = data.get(workload, {}).get(kernel)
        if ent and ent.get("source_hash") == _kernel_source_hash():
            return ent.get("bytes_per_launch")
    except Exception:
        return None
    return None


def _kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "qimax_internal.h"):
        with open(os.path.join(ROOT, "paper_2505_03307_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bench_batch(log, count: int = 256):
    """The 256-circuit recipe (n 8..48, depth 50..400, 5..30 Rz): every circuit propagated
    one at a time on a single-circuit context (plain) vs all together in batches (one per
    key class), FP64 and FP32; FP32 error against FP64 per circuit."""
    from paper_2505_03307_amd import workloads as W
    from paper_2505_03307_amd.qimax import Batch, Simulator
    from paper_2505_03307_amd.serve import key_class

    circs = W.c4_batch(count=count)
    # both paths with the heuristic sort variants: the autotuner would still be timing
    # candidates in the measured repetition (its choices are the headline sections' subject)
    os.environ["QIMAX_AUTOTUNE"] = "0"
    classes = {}
    for i, c in enumerate(circs):
        classes.setdefault(key_class(c.n), []).append(i)
    out = {"circuits": len(circs), "n_range": [min(c.n for c in circs), max(c.n for c in circs)],
           "key_classes": {str(k): len(v) for k, v in sorted(classes.items())}}
    results = {}
    for precision in (64, 32):
        batches = {cls: Batch(precision=precision, max_n=cls, device=0) for cls in classes}
        sims = {}
        for rep in range(2):  # the first repetition grows the device buffers
            t0 = time.perf_counter()
            upd_b = 0
            res_b = {}
            for cls, idx in classes.items():
                bt = batches[cls]
                ids = [bt.submit(circs[i]) for i in idx]
                bt.run()
                for i, cid in zip(idx, ids):
                    upd_b += bt.circuit_updates(cid)
                    res_b[i] = bt.fetch(cid)
            t1 = time.perf_counter()
            upd_p = 0
            for i, c in enumerate(circs):
                s = sims.get(c.n)
                if s is None:
                    s = sims[c.n] = Simulator(c.n, precision=precision, device=0)
                s.reset()
                u0 = s.stats()["term_updates"]
                s.run(c)
                g = s.generators()
                upd_p += s.stats()["term_updates"] - u0
                if rep == 1 and precision == 64:
                    for x, y in zip(g, res_b[i]):
                        if not np.array_equal(x, y):
                            raise RuntimeError(f"batched result differs from plain for circuit {i}")
            t2 = time.perf_counter()
        for bt in batches.values():
            bt.close()
        for s in sims.values():
            s.close()
        results[precision] = res_b
        key = "fp64" if precision == 64 else "fp32"
        out[key] = {"batched_updates_per_s": round(upd_b / (t1 - t0), 1), "plain_updates_per_s": round(upd_p / (t2 - t1), 1),
                    "batched_s": round(t1 - t0, 4), "plain_s": round(t2 - t1, 4),
                    "speedup": round((t2 - t1) / (t1 - t0), 3), "term_updates": int(upd_b),
                    "final_terms": int(sum(int(r[0][-1]) for r in res_b.values()))}
        log("batch", key, out[key])
    # FP32 against FP64, stated per result: for each circuit the largest over its generators
    # of ||w32 - w64||_2 / ||w64||_2 over the union of keys
    per = []
    for i in results[64]:
        o64, k64, w64 = results[64][i]
        o32, k32, w32 = results[32][i]
        worst = 0.0
        for j in range(len(o64) - 1):
            a = {tuple(r): v for r, v in zip(k64[o64[j]:o64[j + 1]].tolist(), w64[o64[j]:o64[j + 1]].tolist())}
            bb = {tuple(r): v for r, v in zip(k32[o32[j]:o32[j + 1]].tolist(), w32[o32[j]:o32[j + 1]].tolist())}
            num = sum((a.get(k, 0.0) - bb.get(k, 0.0)) ** 2 for k in set(a) | set(bb)) ** 0.5
            den = sum(v * v for v in a.values()) ** 0.5
            worst = max(worst, num / (den or 1.0))
        per.append(worst)
    per = np.array(per)
    out["fp32_rel_err_vs_fp64_per_circuit"] = {"max": float(per.max()), "median": float(np.median(per)),
                                               "p99": float(np.quantile(per, 0.99)), "circuits": int(per.size)}
    out["fp32_within_5e-6"] = bool(per.max() <= 5e-6)
    os.environ.pop("QIMAX_AUTOTUNE", None)
    return out


def bench_serve(log, count: int = 200, budget_gb: float = 200.0, one_batch: bool = False):
    """Poisson arrivals of ansatz circuits (n 10..16, 1 or 2 layers, FP32, eps 1e-9) at 0.7x
    the measured sequential capacity: continuous batching vs the sequential plain path."""
    from paper_2505_03307_amd import workloads as W
    from paper_2505_03307_amd import serve

    circuits, gaps = W.c5_stream(seed=0, count=count)
    os.environ["QIMAX_AUTOTUNE"] = "0"  # both paths with the heuristic sort variants
    # sequential capacity, measured back to back on the first requests
    probe = min(60, count)
    res, _ = serve.serve_sequential(circuits[:probe], np.zeros(probe), precision=32)  # warm-up
    t0 = time.perf_counter()
    res, _ = serve.serve_sequential(circuits[:probe], np.zeros(probe), precision=32)
    cap = probe / (time.perf_counter() - t0)
    lam = 0.7 * cap
    arrivals = np.cumsum(gaps) / lam
    log("serve: sequential capacity", round(cap, 1), "req/s; arrival rate", round(lam, 1))
    t0 = time.perf_counter()
    seq, _ = serve.serve_sequential(circuits, arrivals, precision=32,
                                    progress=lambda k: k % 100 == 0 and log("serve: sequential", k, "done"))
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    srv_res, _ = serve.serve_trace_lanes(circuits, arrivals, int(budget_gb * 1e9), precision=32,
                                         progress=lambda k: log("serve: served", k, "arrived"))
    t_srv = time.perf_counter() - t0
    out = {"requests": count, "arrival_rate_per_s": round(lam, 2), "sequential_capacity_per_s": round(cap, 2),
           "budget_GB": budget_gb, "served": serve.summarize(srv_res, t_srv),
           "sequential": serve.summarize(seq, t_seq),
           "server": "two lanes split at 256 MB predicted footprint, one HIP stream and host thread each: "
                     "small requests continuously batched, large ones one at a time through the "
                     "single-circuit API"}
    if one_batch:
        t0 = time.perf_counter()
        one, srv = serve.serve_trace(circuits, arrivals, int(budget_gb * 1e9), precision=32)
        srv.close()
        out["served_one_batch"] = serve.summarize(one, time.perf_counter() - t0)
    log("serve", out)
    os.environ.pop("QIMAX_AUTOTUNE", None)
    return out


def bench_families(log, reps: int = 3):
    """The paper's families (Sec. V): GHZ, graph state and |XYZ + chain> at #Repeats from 10^2
    to 10^5. Per case: instructions m, grouped runs K + K', the grouping alone (median ms), a
    whole step (reset, grouping, propagation; median ms) and the average stabilizer rank
    (terms per generator). The paper's claim: cost follows K + K' and the rank, not m."""
    from paper_2505_03307_amd import workloads as W
    from paper_2505_03307_amd.qimax import Simulator

    cases = [("ghz", 64, r, 1) for r in (100, 1000, 10000)] + [("graph", 48, r, 1) for r in (100, 1000)] + \
            [("xyz_chain", 12, r, 2) for r in (100, 1000, 10000, 100000)]
    out = []
    for fam, n, r, L in cases:
        c = (W.ghz(n, repeats=r, layers=L) if fam == "ghz" else
             W.graph_state(0, n, repeats=r, layers=L) if fam == "graph" else W.xyz_chain(0, n, repeats=r, layers=L))
        with Simulator(n, device=0) as s:
            s.run(c)  # warm-up (buffers)
            s.sync()
            tg, ts = [], []
            for _ in range(reps):
                t0 = time.perf_counter()
                n_ops, K, Kp = s.group_counts(c)
                tg.append(time.perf_counter() - t0)
            for _ in range(reps):
                s.sync()
                t0 = time.perf_counter()
                s.reset()
                s.run(c)
                s.flush()
                s.sync()
                ts.append(time.perf_counter() - t0)
            terms = s.num_terms()
        ent = {"family": fam, "n": n, "repeats": r, "layers": L, "m": c.m, "runs_K_plus_Kp": K + Kp, "operators": n_ops,
               "grouping_ms": round(float(np.median(tg)) * 1e3, 3), "step_ms": round(float(np.median(ts)) * 1e3, 3),
               "avg_rank": round(terms / n, 2)}
        log("families", ent)
        out.append(ent)
    return out


def run_workload(circ, precision: int, steps: int, warmup: int, fp32_merge: int = 0, label: str = ""):
    """Time `steps` propagation steps of one workload on one context. A step resets the
    generators to Z_j, runs every layer (grouping and passes) and ends with the final
    generators in HBM. Returns the simulator (still open) and the measured figures."""
    from paper_2505_03307_amd.qimax import Simulator

    sim = Simulator(circ.n, precision=precision, fp32_merge=fp32_merge, prune_eps=circ.eps, device=0)

    def step():
        sim.reset()
        sim.run(circ)
        sim.flush()  # a trailing Clifford run too: the final generators are in HBM

    # warm-up with every kernel timed: finds the kernel with the largest device time
    sim.profile(True)
    for i in range(max(warmup, 1)):
        step()
        sim.sync()
        log(label, "warmup", i, "terms", sim.num_terms())
    warm = sim.profile_read()
    sim.profile(False)
    dom_name = max(warm.items(), key=lambda kv: kv[1]["total_ms"])[0]
    # timed region: only the dominant kernel carries HIP events (one pair per launch group)
    s0 = sim.stats()
    sim.profile_only(dom_name)
    sim.profile(True)
    sim.sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    sim.sync()
    t1 = time.perf_counter()
    prof = sim.profile_read()
    sim.profile(False)
    sim.profile_only(None)
    s1 = sim.stats()
    terms = sim.num_terms()
    per = lambda k: (s1[k] - s0[k]) / steps
    updates, alg_step, rounds = per("term_updates"), per("alg_bytes"), per("rounds")
    host = {"busy_ms_per_step": round(per("host_busy_ms"), 3), "sync_wait_ms_per_step": round(per("host_wait_ms"), 3),
            "syncs_per_step": per("syncs")}
    sec = (t1 - t0) / steps
    log(label, "timed", steps, "steps, ms/step", round(sec * 1e3, 3), "updates/step", int(updates), "terms", terms)
    # dominant kernel, timed over the timed region: the step's algorithmic bytes (every live
    # input term read once, every merged output term written once, per pass) per launch
    d = prof[dom_name]
    launches = d["launches"] / steps
    avg_ms = d["total_ms"] / d["launches"]
    alg_per_launch = alg_step / launches
    achieved = alg_per_launch / (avg_ms * 1e-3) / 1e9
    # every kernel, over the same number of extra steps (outside the timed region)
    sim.profile(True)
    for _ in range(steps):
        step()
    allk = sim.profile_read()
    sim.profile(False)
    kernels = {k: {"launches": v["launches"] // steps, "ms_per_step": round(v["total_ms"] / steps, 4),
                   "moved_GBps": round(v["alg_bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1) if v["total_ms"] else None}
               for k, v in sorted(allk.items(), key=lambda kv: -kv[1]["total_ms"])}
    log(label, "kernels", json.dumps(kernels))
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(dom_name, label),
                "avg_launch_ms": round(avg_ms, 5), "alg_bytes_per_launch": int(alg_per_launch),
                "launches_per_step": launches,
                "image_bytes_per_launch": int(d["alg_bytes"] / d["launches"])}
    loop = {"alg_GB_per_step": round(alg_step / 1e9, 4), "alg_GBps": round(alg_step / sec / 1e9, 1),
            "frac": round(alg_step / sec / 1e9 / HBM_PEAK_GBS, 4), "rounds_per_step": rounds,
            "kernel_ms_per_step": round(sum(v["total_ms"] for v in allk.values()) / steps, 4)}
    out = {"value": round(updates / sec, 1), "ms_per_step": round(sec * 1e3, 3), "term_updates_per_step": int(updates),
           "final_terms": terms, "roofline": roofline, "loop": loop, "kernels": kernels, "host": host}
    out["_gen_updates_per_step"] = sim.generator_updates() / (max(warmup, 1) + 2 * steps)
    # the autotuner's size classes and choices (candidate 0: heuristic top-digit passes, 1: one
    # more, 2: one global tile order, 3 / 4: as 0 / 1 with multi-launch global passes, 5: dense)
    out["tuning"] = sim.tuning()
    # the same step recorded once and replayed as one HIP graph (no host work between rounds;
    # the grouping and planning on the host happen once, at recording)
    try:
        g = sim.record_step(circ)
        for _ in range(2):
            g.launch()
        sim.sync()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.launch()
        sim.sync()
        gsec = (time.perf_counter() - t0) / steps
        g.close()
        out["graph_replay"] = {"ms_per_step": round(gsec * 1e3, 3), "term_updates_per_s": round(updates / gsec, 1),
                               "eager_over_replay": round(sec / gsec, 3)}
        log(label, "graph replay ms/step", round(gsec * 1e3, 3))
    except Exception as e:  # reported, not fatal to the bench line
        out["graph_replay"] = {"error": str(e)}
    return sim, out


def cpu_oracle_baseline(circ, gen_updates: np.ndarray, reps: int = 3, gens=None):
    """The CPU oracle (as it stands) on the host cores: the generators `gens` (all by default)
    with the box's thread share, and a sample of generators on one thread; medians of `reps`
    runs."""
    import oracle

    def timed(gens, threads):
        ts = []
        for _ in range(reps):
            c0 = time.perf_counter()
            o = oracle.propagate(circ, gens=gens, threads=threads)
            ts.append(time.perf_counter() - c0)
            o.close()
        return float(np.median(ts)), float(np.mean(ts))

    threads = min(16, os.cpu_count() or 1)
    allg = list(range(circ.n)) if gens is None else list(gens)
    med, mean = timed(allg, threads)
    upd = float(gen_updates[allg].sum())
    res = {"value": round(upd / med, 1), "unit": "term-updates/s", "cores": threads, "kind": "oracle",
           "seconds_median": round(med, 3), "seconds_mean": round(mean, 3), "runs": reps,
           "sample": f"generators {allg[0]}..{allg[-1]} of {circ.n} of the workload, gate by gate in FP64, "
                     f"{threads} threads (generators in parallel); median of {reps} runs"}
    # one thread: the generators with the fewest updates that together hold about 1/16 of them
    order = np.argsort(gen_updates)
    pick, acc = [], 0.0
    for j in order.tolist():
        pick.append(int(j))
        acc += float(gen_updates[j])
        if acc >= upd / 16:
            break
    med1, mean1 = timed(sorted(pick), 1)
    res["single_thread"] = {"value": round(acc / med1, 1), "cores": 1, "seconds_median": round(med1, 3),
                            "seconds_mean": round(mean1, 3), "generators": sorted(pick),
                            "sample_updates": int(acc)}
    try:
        import subprocess
        res["host_cpu"] = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.split(
            "Model name:")[1].splitlines()[0].strip()
    except Exception:
        pass
    log("cpu", res)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--precision", type=int, default=64, choices=(32, 64))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu", type=int, default=1, help="time the CPU oracle baseline (0: skip)")
    ap.add_argument("--workload", choices=("c2", "hea"), default="c2",
                    help="headline: the n=32 Clifford+Rz circuit (c2) or the n=16 two-layer ansatz (hea)")
    ap.add_argument("--c2", type=int, default=1, help="the n=32 Clifford+Rz section when it is not the headline")
    ap.add_argument("--c2-fp32", type=int, default=1, help="the FP32 run of the n=32 Clifford+Rz circuit (0: skip)")
    ap.add_argument("--hea", type=int, default=1, help="the n=16 two-layer ansatz section when it is not the headline")
    ap.add_argument("--hea-fp64", type=int, default=1, help="the FP64 run of the ansatz, the FP32 run's reference (0: skip)")
    ap.add_argument("--families", type=int, default=1, help="the paper's circuit families section (0: skip)")
    ap.add_argument("--batch", type=int, default=256, help="circuits in the batched-vs-plain section (0: skip)")
    ap.add_argument("--serve", type=int, default=200, help="requests in the serving section (0: skip)")
    ap.add_argument("--serve-one-batch", action="store_true", help="also serve the trace with a single batch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one GPU only; --gpus {args.gpus} is not supported "
              "(generator sharding across GPUs is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)

    from paper_2505_03307_amd import workloads as W

    # ---- the n=32 Clifford+Rz circuit, FP64 (and FP32)
    c2 = None
    cpu = None
    if args.workload == "c2" or args.c2:
        circ = W.c2_clifford_rz(seed=args.seed)
        log("workload", circ.name, "instructions", circ.m)
        sim, c2 = run_workload(circ, args.precision, args.steps, args.warmup, label="c2")
        gen_updates = c2.pop("_gen_updates_per_step")
        if args.c2_fp32:
            # FP32 on the same circuit (compensated merge), with the library's stated error per generator
            sim32, c2_32 = run_workload(circ, 32, args.steps, args.warmup, label="c2-fp32")
            c2_32.pop("_gen_updates_per_step")
            dn, rn, kd = sim32.compare(sim, tau=1e-6)
            c2_32["fp32_rel_err_vs_fp64_per_generator_max"] = float(np.max(dn / np.where(rn > 0, rn, 1.0)))
            c2_32["keys_differing_on_K_1e-6"] = int(kd.sum())
            c2["fp32"] = c2_32
            sim32.close()
        sim.close()
        c2["workload"] = (f"random Clifford+Rz circuit, n=32, 200 moments, 40 Rz, seed {args.seed}, eps=0, "
                          f"final terms {c2['final_terms']}")
        c2["note"] = ("each grouped operator counted once; no two images of this circuit ever share a key, so its "
                      "merges sum nothing; most updates are Clifford relabellings done by table lookup")
        if args.cpu and args.workload == "c2":
            cpu = cpu_oracle_baseline(circ, gen_updates)

    # ---- the n=16 two-layer ansatz (the configuration whose images merge), FP32 (and FP64)
    hea = None
    if args.workload == "hea" or args.hea:
        c3 = W.c3_hea(seed=0, n=16, layers=2, eps=1e-9)
        log("workload", c3.name)
        hsteps = args.steps if args.workload == "hea" else max(3, args.steps)
        s32, h32 = run_workload(c3, 32, hsteps, args.warmup, label="hea-fp32")
        h64 = None
        if args.hea_fp64:
            s64, h64 = run_workload(c3, 64, hsteps, args.warmup, label="hea-fp64")
            h64.pop("_gen_updates_per_step")
            dn, rn, kd = s32.compare(s64, tau=1e-6)
            rel = dn / np.where(rn > 0, rn, 1.0)
            h32["fp32_rel_err_vs_fp64_per_generator"] = [float(f"{x:.3e}") for x in rel]
            h32["fp32_rel_err_vs_fp64_max"] = float(rel.max())
            h32["keys_differing_on_K_1e-6"] = int(kd.sum())
            s64.close()
        gen_updates = h32.pop("_gen_updates_per_step")
        s32.close()
        hea = {"workload": "hardware-efficient ansatz n=16, 2 layers (Rx,Ry,Rz per qubit + CX ladder), "
                           "eps=1e-9, seed 0", "fp32": h32, "fp64": h64,
               "note": "two layers reach 1.29e8 terms; a third would exceed 288 GB"}
        if args.cpu and args.workload == "hea":
            # generators 0..3 hold 95% of the terms: the multi-thread sample leaves them out
            cpu = cpu_oracle_baseline(c3, gen_updates, gens=list(range(4, 16)))

    families = bench_families(log) if args.families else None
    batch = bench_batch(log, args.batch) if args.batch else None
    serving = bench_serve(log, args.serve, one_batch=args.serve_one_batch) if args.serve else None
    if args.workload == "c2":
        head, dtype, wl = c2, ("f64" if args.precision == 64 else "f32"), c2["workload"]
        cfg = {"workload": wl, "n_qubits": 32, "instructions": int(circ.m), "final_terms": c2["final_terms"],
               "term_updates_per_step": c2["term_updates_per_step"], "note": c2["note"]}
    else:
        head, dtype = hea["fp32"], "f32"
        cfg = {"workload": hea["workload"] + ", FP32 weights with compensated (TwoSum) merge",
               "n_qubits": 16, "layers": 2, "final_terms": head["final_terms"],
               "term_updates_per_step": head["term_updates_per_step"],
               "fp32_rel_err_vs_fp64_max": head.get("fp32_rel_err_vs_fp64_max")}
    out = {
        "metric": "Pauli-term updates/sec + HBM GB/s fraction; batched vs plain at 5e-6 rel err",
        "value": head["value"],
        "unit": "term-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": cfg,
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "loop": head["loop"],
        "kernels": head["kernels"],
        "host": head["host"],
        "c2_clifford_rz_n32": c2,
        "hea_n16": hea,
        "families": families,
        "batched_vs_plain": batch,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
