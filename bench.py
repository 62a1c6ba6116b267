#!/usr/bin/env python3
"""Benchmark of the OPH/HOPH hot path on one MI355X.

One step is the whole path over one batch: sketch every set of the collection
(one shared universal hash, k bins, per-bin minimum), refill the resident
index, sketch the query batch, and answer every query with the (1:1) HOPH scan
(coarse pass, per-survivor pass, sorted CSR output).  Workload: 1,000,000
bag-of-visual-words sets over 2^20 codewords (Zipf(1.1) codewords, log-normal
sizes, median 600, clipped to [100, 4000]), h(x) = (a x + b) mod (2^31 - 1),
k = 512 bins in groups of 32, 1,024 queries with 1% of the collection planted as
near-duplicates at J in [0.5, 0.98], T = 4/5, eps = 1e-4.  Inputs are seeded
synthetic data resident in HBM before the timed region.

Prints one JSON line.  ``value`` is query x index pairs decided per second over
whole steps; per-kernel rates, the roofline of the dominant kernel and the
oracle's CPU rate on a bounded sample are attached.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                         # MI355X HBM3E, published
CUS, LANES, CLOCK_HZ = 256, 64, 2.4e9         # MI355X compute units, wavefront lanes, peak engine clock
ALU_PEAK_OPS = CUS * LANES * CLOCK_HZ         # 32-bit VALU lane-operations per second


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-sets", type=int, default=1_000_000)
    ap.add_argument("--n-queries", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=1806)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-sets", type=int, default=200_000)
    ap.add_argument("--cpu-sample-queries", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling HBM counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(w, n_sets, n_q, sample_sets, sample_q):
    """The oracle (plain C, OpenMP, exact rationals) on a bounded sample of the
    same workload, extrapolated linearly to one full step."""
    from fractions import Fraction
    import numpy as np
    from oracle import scale
    ns = min(sample_sets, n_sets)
    nq = min(sample_q, n_q)
    kw = dict(hash_kind=w.hash_kind, universe=w.universe, layout=w.layout, k=w.k, kp=w.kp, ra=w.ra, rb=w.rb,
              ha=w.ha, hb=w.hb, perm=w.perm)
    which = np.arange(ns, dtype=np.uint64)
    t0 = time.perf_counter()
    sig = scale.sketch(w.collection.ids, w.collection.offsets, which=which, **kw)
    t_sk = time.perf_counter() - t0
    qsig = scale.sketch(w.queries.ids, w.queries.offsets, which=np.arange(nq, dtype=np.uint64), **kw)
    t0 = time.perf_counter()
    scale.query(sig, qsig, goph=w.goph, kp=w.kp, T=Fraction(*w.T), eps=Fraction(*w.eps), ra=w.ra, rb=w.rb)
    t_q = time.perf_counter() - t0
    per_set = t_sk / ns
    per_pair = t_q / (ns * nq)
    full = n_sets * per_set + n_q * per_set + n_sets * n_q * per_pair
    return {
        "value": n_sets * n_q / full,
        "unit": "query x index pairs decided/s",
        "cores": scale.max_threads(),
        "kind": "oracle",
        "sample": (f"oracle sketch of the first {ns} sets ({t_sk:.2f} s) and GOPH/HOPH decisions for {nq} queries "
                   f"x {ns} sets ({t_q:.2f} s), extrapolated linearly to {n_sets} sets and {n_q} queries "
                   f"({full:.1f} s per step)"),
        "sets_sketched_per_s": 1.0 / per_set,
        "pairs_decided_per_s": 1.0 / per_pair,
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hoph11_bovw_1M_pmc_traffic.txt")


def kernel_source_hash() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1805_11254_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_traffic():
    """HBM bytes per launch from the committed PMC summary, by kernel name
    prefix, or {} when the kernels changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    lines = open(TRAFFIC_FILE).read().splitlines()
    recorded = next((l.split()[1] for l in lines if l.startswith("kernel_source_sha256")), None)
    if recorded != kernel_source_hash():
        return {}
    out = {}
    for l in lines:
        if l.startswith("traffic "):
            _, name, grid, _, _, b = l.split()
            prefix = name.split("<")[0]
            out[prefix] = max(out.get(prefix, 0.0), float(b))
    return out


def copy_calibration():
    """A plain device-to-device copy of 1 GiB, three times: the reference for
    FETCH_SIZE / WRITE_SIZE counter readings."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 3}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              f"run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1805_11254_amd as H
    import workloads as W

    H.lib()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", 0)))
    dev = torch.device("cuda")

    t0 = time.perf_counter()
    w = W.hoph_bovw(n=args.n_sets, n_q=args.n_queries, seed=args.seed)
    log(f"generated {w.collection.n} sets / {w.collection.ids.size} ids and {w.queries.n} queries "
        f"in {time.perf_counter() - t0:.1f} s")
    ids = torch.from_numpy(w.collection.ids.view(np.int32)).to(dev)
    offs = torch.from_numpy(w.collection.offsets.view(np.int64)).to(dev)
    qids = torch.from_numpy(w.queries.ids.view(np.int32)).to(dev)
    qoffs = torch.from_numpy(w.queries.offsets.view(np.int64)).to(dev)
    p = H.SketchParams(w.layout, w.k, w.kp, w.hash_kind, w.universe, w.ra, w.rb, w.ha, w.hb)
    N, Q, k, kp = w.collection.n, w.queries.n, w.k, w.kp
    nnz = int(w.collection.ids.size)
    sig = torch.empty((N, k), dtype=torch.int32, device=dev)
    qsig = torch.empty((Q, k), dtype=torch.int32, device=dev)
    idx = H.Index(p, sig[:0], capacity=N)
    stream = torch.cuda.current_stream()
    cap = [None]

    def step(ev=None):
        e = ev or [None] * 5
        if e[0] is not None: e[0].record(stream)
        H.sketch_oph(p, ids, offs, out=sig)
        if e[1] is not None: e[1].record(stream)
        idx.reset()
        idx.append(sig)
        if e[2] is not None: e[2].record(stream)
        H.sketch_oph(p, qids, qoffs, out=qsig)
        if e[3] is not None: e[3].record(stream)
        out = H.query_hoph(idx, qsig, T=w.T, eps=w.eps, capacity=cap[0])
        if e[4] is not None: e[4].record(stream)
        return out

    for i in range(args.warmup):
        out = step()
        if cap[0] is None:
            cap[0] = max(1 << 16, 2 * int(out[1].numel()))
    H.sync()
    torch.cuda.synchronize()
    log("warm-up done")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    qms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step(evs[i])
        qms.append(idx.last_query_ms())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1000.0 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")

    def mean_ms(a, b):
        return sum(e[a].elapsed_time(e[b]) for e in evs) / len(evs)

    sketch_ms = mean_ms(0, 1)
    index_ms = mean_ms(1, 2)
    qsketch_ms = mean_ms(2, 3)
    query_ms = mean_ms(3, 4)
    coarse_ms = sum(q[0] for q in qms) / len(qms)
    fine_ms = sum(q[1] for q in qms) / len(qms)
    sort_ms = sum(q[2] for q in qms) / len(qms)

    # algorithmic work per launch
    sketch_bytes = nnz * 4 + (N + 1) * 8 + N * k * 4
    index_bytes = 2 * N * k * 4
    tabs = H.decision_tables(p, w.T, w.eps)
    depth = next((l + 1 for l in range(tabs["L"]) if tabs["rej"][l] >= 0), tabs["L"])
    depth = min(depth, 128 // kp, 4, tabs["L"])
    coarse_cmp = Q * N * kp * depth
    coarse_bytes = N * kp * 4 * depth + Q * k * 4
    traffic = load_traffic()
    kernels = {
        "sketch_oph": {"ms": sketch_ms, "bound": "hbm", "achieved": sketch_bytes / (sketch_ms * 1e-3) / 1e9,
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": traffic.get("sketch_kernel"),
                       "algorithmic_bytes": sketch_bytes, "sets_per_s": N / (sketch_ms * 1e-3)},
        "index_store": {"ms": index_ms, "bound": "hbm", "achieved": index_bytes / (index_ms * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": traffic.get("index_store_vec"),
                        "algorithmic_bytes": index_bytes},
        "scan_coarse": {"ms": coarse_ms, "bound": "alu", "achieved": coarse_cmp / (coarse_ms * 1e-3) / 1e12,
                        "peak": ALU_PEAK_OPS / 1e12, "unit": "Tcompare/s",
                        "traffic": traffic.get("scan_coarse_kernel"), "algorithmic_bytes": coarse_bytes,
                        "hbm_gbs": coarse_bytes / (coarse_ms * 1e-3) / 1e9, "depth": depth},
        "scan_fine": {"ms": fine_ms},
        "sort_and_csr": {"ms": sort_ms},
        "query_sketch": {"ms": qsketch_ms},
    }
    for v in kernels.values():
        if "achieved" in v:
            v["frac"] = v["achieved"] / v["peak"]
    dom_name = max(("sketch_oph", "index_store", "scan_coarse"), key=lambda n: kernels[n]["ms"])
    dom = kernels[dom_name]
    roofline = {"kernel": dom_name, "bound": dom["bound"], "achieved": dom["achieved"], "peak": dom["peak"],
                "unit": dom["unit"], "frac": dom["frac"], "traffic": dom["traffic"],
                "algorithmic_bytes": dom["algorithmic_bytes"]}

    # accuracy against the exact Jaccard similarity (outside the timed region)
    offs_h = out[0].cpu().numpy()
    ids_h = out[1].cpu().numpy().view(np.uint32)
    T = w.T[0] / w.T[1]
    truth = {(q, s) for (q, s, J) in w.planted if J >= T}
    got = set()
    for q in range(Q):
        for s in ids_h[offs_h[q]:offs_h[q + 1]].tolist():
            got.add((q, s))
    tp = 0
    for (q, s) in got:
        a = np.unique(w.queries.set(q))
        b = np.unique(w.collection.set(s))
        inter = np.intersect1d(a, b, assume_unique=True).size
        if inter / (a.size + b.size - inter) >= T:
            tp += 1
    recall = len(truth & got) / max(1, len(truth))
    precision = tp / max(1, len(got))

    rec = {
        "metric": "sets sketched/s + query x index signature compares/s (HBM %), served p99 ms",
        "value": N * Q / (ms_per_step * 1e-3),
        "unit": "query x index pairs decided/s (whole step: sketch + index + query sketch + HOPH scan)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "hoph_1to1_bovw", "n_sets": N, "n_queries": Q, "nnz": nnz, "universe": w.universe,
                   "k": k, "k_group": kp, "groups": k // kp, "ratio": "1:1", "hash": "(a x + b) mod (2^31 - 1)",
                   "T": "4/5", "eps": "1/10000", "empty_policy": "joint", "parallelism": "single GPU"},
        "sets_sketched_per_s": N / (sketch_ms * 1e-3),
        "scan_pairs_per_s": N * Q / (query_ms * 1e-3),
        "scan_hbm_frac": kernels["scan_coarse"]["hbm_gbs"] / HBM_PEAK_GBS,
        "served_p99_ms": None,
        "phase_ms": {"sketch": sketch_ms, "index": index_ms, "query_sketch": qsketch_ms, "query": query_ms,
                     "coarse": coarse_ms, "fine": fine_ms, "sort_csr": sort_ms},
        "kernels": kernels,
        "roofline": roofline,
        "accepted_pairs": len(got),
        "recall_planted": recall,
        "precision_exact_jaccard": precision,
    }
    idx.free()
    if not args.no_cpu_baseline:
        log("timing the oracle on a CPU sample")
        rec["cpu_baseline"] = cpu_baseline(w, N, Q, args.cpu_sample_sets, args.cpu_sample_queries)
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
