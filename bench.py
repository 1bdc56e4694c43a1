"""Benchmark: Pauli-term updates per second of generator propagation on one MI355X.

Workload (one step): the n=32 random Clifford circuit of 200 moments (H, S, CX drawn
uniformly per qubit) with 40 Rz(theta) gates at random slots, seed 0, FP64 weights,
prune eps = 0. A step resets the n generators to Z_j on the device, runs the grouping pass
and every propagation pass, and ends with the final generators resident in HBM (the
paper's timing window, Sec. V). One term update = one output image of one grouped
operator (a Clifford operator counts its input terms).

Prints one JSON line. The roofline object covers the kernel with the largest share of
device time, timed with HIP events on the library's stream over the timed region; the
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


def traffic_for(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it is current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        ent = data.get(kernel)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", type=int, default=64, choices=(32, 64))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-gens", type=str, default="all",
                    help="oracle sample: 'all', 'none', or a comma list of generator ids")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(generator sharding across GPUs is a design note, not implemented)", file=sys.stderr)
        sys.exit(2)

    from paper_2505_03307_amd import workloads as W
    from paper_2505_03307_amd.qimax import Simulator

    circ = W.c2_clifford_rz(seed=args.seed)
    g, a, b, t = circ.gate, circ.q0, circ.q1, circ.theta
    log("workload", circ.name, "instructions", circ.m)
    sim = Simulator(circ.n, precision=args.precision, device=0)

    def step():
        sim.reset()
        sim.apply_circuit((g, a, b, t))

    for i in range(args.warmup):
        step()
        sim.sync()
        log("warmup", i, "terms", sim.num_terms())
    s0 = sim.stats()
    sim.profile(True)
    sim.sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    sim.sync()
    t1 = time.perf_counter()
    prof = sim.profile_read()
    sim.profile(False)
    s1 = sim.stats()
    terms = sim.num_terms()
    updates = (s1["term_updates"] - s0["term_updates"]) / args.steps
    sec = (t1 - t0) / args.steps
    log("timed", args.steps, "steps, ms/step", round(sec * 1e3, 3), "updates/step", int(updates), "terms", terms)

    # dominant kernel by device time
    dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    name, d = dom
    avg_ms = d["total_ms"] / d["launches"]
    alg_per_launch = d["alg_bytes"] / d["launches"]
    achieved = alg_per_launch / (avg_ms * 1e-3) / 1e9
    kernels = {k: {"launches": v["launches"] // args.steps, "ms_per_step": round(v["total_ms"] / args.steps, 4),
                   "alg_GBps": round(v["alg_bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1) if v["total_ms"] else None}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"])}
    log("kernels", json.dumps(kernels))
    roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(name),
                "avg_launch_ms": round(avg_ms, 5), "alg_bytes_per_launch": int(alg_per_launch)}

    # CPU oracle on the host cores (test infrastructure, timed beside the GPU)
    cpu = None
    if args.cpu_gens != "none":
        import oracle
        gen_updates = sim.generator_updates()
        gens = list(range(circ.n)) if args.cpu_gens == "all" else [int(x) for x in args.cpu_gens.split(",")]
        threads = min(16, os.cpu_count() or 1)
        log("cpu oracle on generators", gens, "threads", threads)
        c0 = time.perf_counter()
        o = oracle.propagate(circ, gens=gens, threads=threads)
        c1 = time.perf_counter()
        # generator_updates accumulates over every step run so far: scale to one step
        runs = args.warmup + args.steps
        sample_updates = float(gen_updates[gens].sum()) / runs
        cpu = {"value": round(sample_updates / (c1 - c0), 1), "unit": "term-updates/s", "cores": threads,
               "kind": "oracle", "seconds": round(c1 - c0, 2),
               "sample": f"{len(gens)} of {circ.n} generators of the same circuit, gate by gate in FP64 "
                         f"({int(sum(o.count(i) for i in range(o.num_gens)))} final terms)"}
        log("cpu", cpu)

    sim.close()
    out = {
        "metric": "Pauli-term updates/sec + HBM GB/s fraction; batched vs plain at 5e-6 rel err",
        "value": round(updates / sec, 1),
        "unit": "term-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": f"random Clifford+Rz circuit, n=32, 200 moments, 40 Rz, seed {args.seed}, "
                               f"eps=0, final terms {terms}",
                   "n_qubits": circ.n, "instructions": circ.m, "final_terms": terms,
                   "term_updates_per_step": int(updates)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
