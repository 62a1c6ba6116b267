#!/usr/bin/env python3
"""Benchmark of the OPH/HOPH hot path on one MI355X.

One step is the whole path over one batch: sketch every set of the collection
(one shared universal hash, k bins, per-bin minimum) straight into the
resident index (row-major signature rows and the narrowed code planes of the
first groups), sketch the query batch, and answer every query with the (1:1) HOPH
scan (coarse pass on codes, per-survivor pass on the words, sorted CSR output).  Workload: 1,000,000
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
    ap.add_argument("--n-sets", type=int, default=None,
                    help="collection size (default 1,000,000; 2,000,000 batched; 8,000,000 serve)")
    ap.add_argument("--n-queries", type=int, default=1024)
    ap.add_argument("--seed", type=int, default=1806)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-sets", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample-queries", type=int, default=512)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling HBM counters)")
    ap.add_argument("--sweep-q", type=str, default="1,2,4,8,16,32,64,128,256,1024,4096",
                    help="scansweep: query batch sizes")
    ap.add_argument("--sweep-sets", type=str, default="1000000,8000000",
                    help="scansweep: index sizes (k = 512 up to 2,000,000 sets, else 256)")
    ap.add_argument("--mode", choices=["step", "batched", "serve", "comparators", "selfjoin", "sweeps", "scansweep"],
                    default="step",
                    help="step: the whole-path step (default JSON line); batched: uneven query batches through "
                         "graph-replayed plans; serve: Poisson arrivals through the serving loop; comparators: "
                         "one-query-per-launch OPH/HOPH and MinWise on the same GPU; selfjoin: every pair inside "
                         "one collection; sweeps: GOPH group count, error tolerance and threshold sweeps")
    ap.add_argument("--batches", type=int, default=256)
    ap.add_argument("--rates", type=str, default="20000,50000,100000,200000,300000")
    ap.add_argument("--serve-seconds", type=float, default=0.5)
    ap.add_argument("--serve-rate", type=float, default=50_000,
                    help="offered queries/s of the step's serving measurement (0 = skip it)")
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
    """SHA-256 of the device code (the HIP kernels and the header they share):
    the counters in the profiles depend on nothing else."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1805_11254_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "k_*.hip")) + [os.path.join(csrc, "hoph_internal.h")]):
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


def _pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def _plan_results_count(H, plan):
    import ctypes as C
    po, pi, n = C.c_void_p(), C.c_void_p(), C.c_uint64()
    H._check(H.lib().hoph_plan_results(plan._h, C.byref(po), C.byref(pi), C.byref(n), H._stream(None)), n.value)
    return n.value


def _resident_index(H, p, n_sets, seed, capacity=None, chunk=1_000_000):
    """Bag-of-visual-words collection (as in the default step, no planted pairs)
    generated, sketched and appended to one resident index chunk by chunk."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda")
    idx = None
    for c0 in range(0, n_sets, chunk):
        n = min(chunk, n_sets - c0)
        t0 = time.perf_counter()
        coll = W.zipf_sets(n, 1 << 20, 600, 0.75, 100, 4000, seed + 1000 * (c0 // chunk))
        ids = torch.from_numpy(coll.ids.view(np.int32)).to(dev)
        offs = torch.from_numpy(coll.offsets.view(np.int64)).to(dev)
        sig = H.sketch_oph(p, ids, offs)
        if idx is None:
            idx = H.Index(p, sig, capacity=capacity or n_sets)
        else:
            idx.append(sig)
        torch.cuda.synchronize()
        del ids, offs, sig
        log(f"index: {c0 + n}/{n_sets} sets ({time.perf_counter() - t0:.1f} s for this chunk)")
    return idx


def bench_batched(args):
    """Uneven query batches (size round(exp U[0, ln 4096]), query sets of 10-10,000
    ids, log-uniform) against a 2,000,000-set HOPH (1:1) index, k = 512 in groups
    of 32; each batch is one replay of the plan's captured graph of persistent
    kernels, tile shapes tuned on the first batch."""
    import numpy as np
    import torch
    import paper_1805_11254_amd as H
    import workloads as W
    N = args.n_sets or 2_000_000
    batches = W.query_batches(args.batches, args.seed + 50)
    a, b = W.hash_coeffs(W.P31, 1, args.seed + 3)
    dev = torch.device("cuda")
    p = H.SketchParams(W.LAYOUT_HIER, 512, 32, W.HASH_MODP31, 1 << 20, 1, 1, int(a[0]), int(b[0]))
    idx = _resident_index(H, p, N, args.seed)
    dq = [(torch.from_numpy(bt.ids.view(np.int32)).to(dev), torch.from_numpy(bt.offsets.view(np.int64)).to(dev))
          for bt in batches]
    n_q = np.array([bt.n for bt in batches])
    max_ids = max(int(bt.ids.size) for bt in batches)
    out = {"metric": "batched query x index pairs decided/s", "unit": "pairs/s", "mode": "batched",
           "config": {"workload": "hoph_1to1_bovw_batched", "n_sets": N, "k": 512, "k_group": 32,
                      "batches": len(batches), "queries": int(n_q.sum()), "query_ids": int(sum(b.ids.size for b in batches)),
                      "batch_size_median": float(np.median(n_q)), "batch_size_max": int(n_q.max())}}
    for name, use_graph in (("graph", True), ("eager", False)):
        plan = H.Plan(idx, p, T=(4, 5), eps=(1, 10000), max_queries=4096, max_query_ids=max_ids,
                      max_results=1 << 20, use_graph=use_graph, tune=True)
        plan.run(*dq[0]); _plan_results_count(H, plan)          # tuning and capture
        torch.cuda.synchronize()
        lat, found = [], 0
        t0 = time.perf_counter()
        for d in dq:
            tb = time.perf_counter()
            plan.run(*d)
            found += _plan_results_count(H, plan)
            lat.append((time.perf_counter() - tb) * 1e3)
        wall = time.perf_counter() - t0
        info = plan.info()
        out[name] = {"seconds": wall, "queries_per_s": float(n_q.sum()) / wall,
                     "pairs_per_s": float(n_q.sum()) * N / wall, "batch_ms_p50": _pct(lat, 50),
                     "batch_ms_p99": _pct(lat, 99), "accepted_pairs": found, "plan": info}
        log(f"{name}: {wall:.3f} s for {len(dq)} batches")
        plan.free()
    # the host-synchronised path, batch by batch (sketch_oph + query_hoph)
    t0 = time.perf_counter()
    found = 0
    for d in dq:
        qs = H.sketch_oph(p, *d)
        found += int(H.query_hoph(idx, qs, T=(4, 5), eps=(1, 10000))[1].numel())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out["host_path"] = {"seconds": wall, "queries_per_s": float(n_q.sum()) / wall,
                        "pairs_per_s": float(n_q.sum()) * N / wall, "accepted_pairs": found}
    out["value"] = out["graph"]["pairs_per_s"]
    idx.free()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Poisson arrivals of single query sets (log-normal sizes, median 800,
    clipped to [10, 10,000]) against a resident 8,000,000-set HOPH (1:1) index,
    k = 256 in groups of 32, while 5% more sets are inserted online."""
    import threading
    import numpy as np
    import torch
    import paper_1805_11254_amd as H
    import workloads as W
    N = args.n_sets or 8_000_000
    n_ins = N // 20
    extra = W.zipf_sets(n_ins, 1 << 20, 600, 0.75, 100, 4000, args.seed + 90)
    a, b = W.hash_coeffs(W.P31, 1, args.seed + 3)
    p = H.SketchParams(W.LAYOUT_HIER, 256, 32, W.HASH_MODP31, 1 << 20, 1, 1, int(a[0]), int(b[0]))
    idx = _resident_index(H, p, N, args.seed, capacity=N + n_ins)
    srv = H.Server(idx, p, T=(4, 5), eps=(1, 10000), slots=4, max_batch_queries=2048, max_batch_ids=1 << 22,
                   max_batch_results=1 << 20, use_graph=True, tune=True)
    t_w, wq = W.poisson_arrivals(20000, 4000, args.seed + 70)
    srv.replay(wq.ids, wq.offsets, t_w - t_w[0])            # warm-up: tuning, capture
    rates = [float(r) for r in args.rates.split(",")]
    out = {"metric": "served queries/s and latency", "unit": "queries/s", "mode": "serve",
           "config": {"workload": "hoph_1to1_bovw_serving", "n_sets": N, "inserted_online": n_ins, "k": 256,
                      "k_group": 32, "slots": srv.stats()["slots"], "seconds_per_rate": args.serve_seconds},
           "rates": []}
    chunk = max(1, n_ins // (4 * len(rates)))
    pos = [0]

    def inserter(stop):
        while not stop.is_set() and pos[0] < n_ins:
            hi = min(n_ins, pos[0] + chunk)
            o = extra.offsets[pos[0]:hi + 1]
            srv.insert(extra.ids[int(o[0]):int(o[-1])], o - o[0])
            pos[0] = hi
            time.sleep(args.serve_seconds / 5)

    for r in rates:
        n = max(1, int(r * args.serve_seconds))
        # 0.1 s at this rate first, so that the slots this rate keeps busy have
        # run (tuned and captured on) their first batch before the measurement
        t_w, wq = W.poisson_arrivals(r, max(1, int(r * 0.1)), args.seed + 1 + int(r))
        srv.replay(wq.ids, wq.offsets, t_w - t_w[0])
        t, q = W.poisson_arrivals(r, n, args.seed + int(r))
        srv.reset_stats()
        stop = threading.Event()
        th = threading.Thread(target=inserter, args=(stop,))
        th.start()
        t0 = time.perf_counter()
        srv.replay(q.ids, q.offsets, t - t[0])
        wall = time.perf_counter() - t0
        stop.set()
        th.join()
        st = srv.stats()
        out["rates"].append({"offered_qps": r, "requests": n, "served_qps": st["completed"] / max(st["busy_s"], 1e-9),
                             "wall_s": wall, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
                             "max_ms": st["max_ms"], "mean_batch": st["mean_batch_queries"], "batches": st["batches"],
                             "index_sets": len(idx)})
        log(f"rate {r:.0f}: served {out['rates'][-1]['served_qps']:.0f} q/s, p50 {st['p50_ms']:.2f} ms, "
            f"p99 {st['p99_ms']:.2f} ms")
    out["inserted_sets"] = srv.stats()["inserted_sets"]
    out["value"] = max(x["served_qps"] for x in out["rates"])
    srv.close()
    idx.free()
    print(json.dumps(out), flush=True)


def bench_comparators(args):
    """The same GPU and workload as the default step: HOPH one query per launch
    and batched, plain OPH (all k bins, no early stop) one query per launch, and
    MinWise with k = 512 independent hashes; recall and precision of each against
    the exact Jaccard similarity of the returned and planted pairs."""
    import numpy as np
    import torch
    import paper_1805_11254_amd as H
    import workloads as W
    w = W.hoph_bovw(n=args.n_sets or 1_000_000, n_q=args.n_queries, seed=args.seed)
    dev = torch.device("cuda")
    p = H.SketchParams(w.layout, w.k, w.kp, w.hash_kind, w.universe, w.ra, w.rb, w.ha, w.hb)
    ids = torch.from_numpy(w.collection.ids.view(np.int32)).to(dev)
    offs = torch.from_numpy(w.collection.offsets.view(np.int64)).to(dev)
    qids = torch.from_numpy(w.queries.ids.view(np.int32)).to(dev)
    qoffs = torch.from_numpy(w.queries.offsets.view(np.int64)).to(dev)
    sig = H.sketch_oph(p, ids, offs)
    qsig = H.sketch_oph(p, qids, qoffs)
    idx = H.Index(p, sig)
    N, Q = w.collection.n, w.queries.n
    T = w.T[0] / w.T[1]
    truth = {(q, s) for (q, s, J) in w.planted if J >= T}

    def accuracy(offs_h, ids_h, nq=None):
        nq = Q if nq is None else nq
        want = {(q, s) for (q, s) in truth if q < nq}
        got = {(q, int(s)) for q in range(nq) for s in ids_h[offs_h[q]:offs_h[q + 1]]}
        tp = 0
        for (q, s) in got:
            a_ = np.unique(w.queries.set(q))
            b_ = np.unique(w.collection.set(s))
            inter = np.intersect1d(a_, b_, assume_unique=True).size
            tp += inter / (a_.size + b_.size - inter) >= T
        return len(want & got) / max(1, len(want)), tp / max(1, len(got)), len(got)

    out = {"metric": "query x index pairs decided/s, same GPU", "unit": "pairs/s", "mode": "comparators",
           "config": {"workload": "hoph_1to1_bovw", "n_sets": N, "n_queries": Q, "k": w.k, "k_group": w.kp}}
    sample = list(range(0, Q, max(1, Q // 64)))[:64]

    def one_per_launch(fn):
        fn(idx, qsig[:1].contiguous())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in sample:
            fn(idx, qsig[i:i + 1].contiguous())
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / len(sample)

    t_h = one_per_launch(lambda ix, q: H.query_hoph(ix, q, T=w.T, eps=w.eps))
    t_o = one_per_launch(lambda ix, q: H.query_oph_full(ix, q, T=w.T))
    out["hoph_one_query_per_launch"] = {"ms_per_query": t_h * 1e3, "pairs_per_s": N / t_h,
                                        "hbm_gbs_group1": N * w.kp * 4 / t_h / 1e9}
    out["oph_full_one_query_per_launch"] = {"ms_per_query": t_o * 1e3, "pairs_per_s": N / t_o,
                                            "hbm_gbs": N * w.k * 4 / t_o / 1e9}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ho, hi = H.query_hoph(idx, qsig, T=w.T, eps=w.eps)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    out["hoph_batched"] = {"seconds": t_b, "pairs_per_s": N * Q / t_b}
    rec, prec, n = accuracy(ho.cpu().numpy(), hi.cpu().numpy().view(np.uint32))
    out["hoph_batched"].update(recall=rec, precision=prec, accepted=n)
    oo, oi = H.query_oph_full(idx, qsig, T=w.T)
    rec, prec, n = accuracy(oo.cpu().numpy(), oi.cpu().numpy().view(np.uint32))
    out["oph_full_one_query_per_launch"].update(recall=rec, precision=prec, accepted=n)
    idx.free()
    del sig
    # MinWise, k = 512 independent hashes mod 2^31 - 1
    ha, hb = W.hash_coeffs(W.P31, 512, args.seed + 5)
    mp = H.MinwiseParams(512, W.HASH_MODP31, w.universe, torch.from_numpy(ha.view(np.int64)).to(dev),
                         torch.from_numpy(hb.view(np.int64)).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    msig = H.minwise_sketch(mp, ids, offs)
    torch.cuda.synchronize()
    t_ms = time.perf_counter() - t0
    mq = H.minwise_sketch(mp, qids, qoffs)
    t0 = time.perf_counter()
    for i in sample:
        H.minwise_query(mp, msig, mq[i:i + 1].contiguous(), T=w.T)
    torch.cuda.synchronize()
    t_mq = (time.perf_counter() - t0) / len(sample)
    n_mw = min(Q, 128)
    mo, mi = H.minwise_query(mp, msig, mq[:n_mw].contiguous(), T=w.T)
    rec, prec, n = accuracy(mo.cpu().numpy(), mi.cpu().numpy().view(np.uint32), n_mw)
    out["minwise"] = {"accuracy_queries": n_mw, "sketch_seconds": t_ms, "sets_sketched_per_s": N / t_ms, "ms_per_query": t_mq * 1e3,
                      "pairs_per_s": N / t_mq, "recall": rec, "precision": prec, "accepted": n}
    out["value"] = out["hoph_batched"]["pairs_per_s"]
    print(json.dumps(out), flush=True)


def _exact_j(a, b) -> float:
    import numpy as np
    a_ = np.unique(a)
    b_ = np.unique(b)
    inter = np.intersect1d(a_, b_, assume_unique=True).size
    return inter / (a_.size + b_.size - inter)


def _pairs_of(offs, ids):
    """Result pairs (row, id) of a CSR answer (host arrays)."""
    import numpy as np
    rows = np.repeat(np.arange(len(offs) - 1, dtype=np.int64), np.diff(offs))
    return set(zip(rows.tolist(), ids.astype(np.int64).tolist()))


def _workload_params(H, w, k=None, kp=None, layout=None):
    return H.SketchParams(w.layout if layout is None else layout, k or w.k, kp or w.kp, w.hash_kind, w.universe,
                          w.ra, w.rb, w.ha, w.hb)


def bench_selfjoin(args):
    """Near-duplicate pairs inside one collection: the default step's 1,000,000
    bag-of-visual-words sets with its 1,024 query sets placed in front, so that
    each query and its planted near-duplicates are pairs inside the collection;
    HOPH (1:1) k = 512 in groups of 32, T = 4/5, eps = 1e-4.  One call decides
    all N(N-1)/2 pairs i < j with a triangular scan (coarse pass on the codes of
    the first group, per-survivor pass on the words, sorted CSR output).  Recall
    is taken over every pair inside a query's family (the query and its planted
    copies) whose exact Jaccard similarity reaches T; precision from the exact
    similarity of every returned pair."""
    import numpy as np
    import torch
    import paper_1805_11254_amd as H
    import workloads as W
    w = W.hoph_bovw(n=args.n_sets or 1_000_000, n_q=args.n_queries, seed=args.seed)
    Q = w.queries.n
    q, c = w.queries, w.collection
    coll = W.Collection(np.concatenate([q.ids, c.ids]).astype(np.uint32),
                        np.concatenate([q.offsets, c.offsets[1:] + q.offsets[-1]]).astype(np.uint64))
    N = coll.n
    dev = torch.device("cuda")
    p = _workload_params(H, w)
    ids = torch.from_numpy(coll.ids.view(np.int32)).to(dev)
    offs = torch.from_numpy(coll.offsets.view(np.int64)).to(dev)
    idx = H.Index(p, H.sketch_oph(p, ids, offs))
    del ids, offs
    T = w.T[0] / w.T[1]
    # every family pair (query and planted copies, ids shifted by Q) with exact J >= T
    fam = {}
    for (qi, slot, _) in w.planted:
        fam.setdefault(qi, [qi]).append(Q + slot)
    truth = set()
    for members in fam.values():
        members = sorted(members)
        for i in range(len(members)):
            for j in range(i + 1, len(members)):
                if _exact_j(coll.set(members[i]), coll.set(members[j])) >= T:
                    truth.add((members[i], members[j]))
    log(f"self-join: {N} sets, {len(truth)} family pairs at J >= T")
    out = {"metric": "pairs inside the collection decided/s", "unit": "pairs/s", "mode": "selfjoin",
           "config": {"workload": "hoph_1to1_bovw_selfjoin", "n_sets": N, "k": w.k, "k_group": w.kp,
                      "T": list(w.T), "eps": list(w.eps), "pairs": N * (N - 1) // 2}}
    for name, coarse in (("codes", H.COARSE_CODES), ("words", H.COARSE_WORDS)):
        for _ in range(max(1, args.warmup)):
            H.self_join(idx, T=w.T, eps=w.eps, coarse=coarse)
        torch.cuda.synchronize()
        walls, passes = [], []
        for _ in range(max(1, args.steps)):
            t0 = time.perf_counter()
            so, si = H.self_join(idx, T=w.T, eps=w.eps, coarse=coarse)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            passes.append(idx.last_query_ms())
        wall = float(np.median(walls))
        got = _pairs_of(so.cpu().numpy(), si.cpu().numpy().view(np.uint32))
        pr = sorted(got)
        sample = pr[:: max(1, len(pr) // 20000)]
        prec = sum(_exact_j(coll.set(a), coll.set(b)) >= T for (a, b) in sample) / max(1, len(sample))
        coarse_ms, fine_ms, sort_ms = (float(np.median([x[i] for x in passes])) for i in range(3))
        out[name] = {"seconds": wall, "pairs_per_s": N * (N - 1) / 2 / wall, "coarse_ms": coarse_ms,
                     "fine_ms": fine_ms, "sort_ms": sort_ms, "accepted": len(got),
                     "recall": len(truth & got) / max(1, len(truth)), "precision": prec,
                     "precision_sample": len(sample)}
        log(f"self-join {name}: {wall * 1e3:.1f} ms, {len(got)} pairs")
    out["value"] = out["codes"]["pairs_per_s"]
    out["ms_per_step"] = out["codes"]["seconds"] * 1e3
    idx.free()
    print(json.dumps(out), flush=True)


def bench_sweeps(args):
    """Synthetic versions of the paper's parameter studies (experiments
    section): 600,000 bag-of-visual-words sets (the paper's default data
    number) and 1,024 queries with 1% of the collection planted as
    near-duplicates at J in [0.5, 0.98]; defaults T = 0.7, eps = 1e-4.
    (1) GOPH group count n at k = 320 (n = 320/k' for k' in 40 ... 5);
    (2) error tolerance eps in 1e-2 ... 1e-6 for GOPH (n = 10) and HOPH (1:1,
    k = 512 in groups of 32); (3) threshold T in 0.5 ... 0.9 for both; (4) the
    paper's methods side by side: GOPH, HOPH 1:2 / 1:1 / 2:1, plain OPH and
    MinWise.  Each point: the batch's device time (coarse, per-survivor, sort),
    the scan's pairs/s, and recall / precision against exact Jaccard
    similarity."""
    import numpy as np
    import torch
    import paper_1805_11254_amd as H
    import workloads as W
    N = args.n_sets or 600_000
    w = W.hoph_bovw(n=N, n_q=args.n_queries, seed=args.seed + 11, T=(7, 10))
    Q = w.queries.n
    dev = torch.device("cuda")
    ids = torch.from_numpy(w.collection.ids.view(np.int32)).to(dev)
    offs = torch.from_numpy(w.collection.offsets.view(np.int64)).to(dev)
    qids = torch.from_numpy(w.queries.ids.view(np.int32)).to(dev)
    qoffs = torch.from_numpy(w.queries.offsets.view(np.int64)).to(dev)
    jcache = {}

    def exact(qi, s):
        key = (qi, s)
        if key not in jcache:
            jcache[key] = _exact_j(w.queries.set(qi), w.collection.set(s))
        return jcache[key]

    planted = [(qi, s) for (qi, s, _) in w.planted]

    def point(idx, qsig, goph, T, eps, call=None, nq=None):
        fn = H.query_goph if goph else H.query_hoph
        call = call or (lambda: fn(idx, qsig, T=T, eps=eps))
        call()
        torch.cuda.synchronize()
        ms, walls = [], []
        for _ in range(max(1, args.steps)):
            t0 = time.perf_counter()
            o, i = call()
            torch.cuda.synchronize()
            walls.append((time.perf_counter() - t0) * 1e3)
            if idx is not None:
                ms.append(idx.last_query_ms())
        dev_ms = [float(np.median([x[j] for x in ms])) for j in range(3)] if ms else [float(np.median(walls)), 0.0, 0.0]
        got = _pairs_of(o.cpu().numpy(), i.cpu().numpy().view(np.uint32))
        t = T[0] / T[1]
        nq = Q if nq is None else nq
        truth = {pq for pq in planted if exact(*pq) >= t and pq[0] < nq}
        tp = sum(exact(a, b) >= t for (a, b) in got)
        total = sum(dev_ms)
        # wall_ms: the whole host-synchronous call (sub-batches included, should the
        # survivors of one pass overflow their buffer; the device times cover the first pass)
        return {"T": list(T), "eps": list(eps), "wall_ms": float(np.median(walls)), "device_ms": total,
                "coarse_ms": dev_ms[0], "queries": nq,
                "fine_ms": dev_ms[1], "sort_ms": dev_ms[2], "pairs_per_s": nq * N / (total * 1e-3),
                "accepted": len(got), "recall": len(truth & got) / max(1, len(truth)),
                "precision": tp / max(1, len(got))}

    out = {"metric": "query x index pairs decided/s across parameter sweeps", "unit": "pairs/s",
           "mode": "sweeps", "config": {"workload": "bovw_sweeps", "n_sets": N, "n_queries": Q}}
    # (1) GOPH group count at k = 320: one sketch, one index per group size
    pg = _workload_params(H, w, k=320, kp=32, layout=W.LAYOUT_OPH)
    gsig = H.sketch_oph(pg, ids, offs)
    gq = H.sketch_oph(pg, qids, qoffs)
    rows = []
    for kp in (40, 32, 20, 16, 10, 8, 5):
        pk = _workload_params(H, w, k=320, kp=kp, layout=W.LAYOUT_OPH)
        idx = H.Index(pk, gsig)
        r = point(idx, gq, True, (7, 10), (1, 10000))
        r.update(n_groups=320 // kp, k_group=kp)
        rows.append(r)
        log(f"GOPH n={320 // kp}: {r['device_ms']:.3f} ms")
        if kp == 32:
            goph10 = idx
        else:
            idx.free()
    out["goph_groups"] = rows
    # (2), (3): GOPH n = 10 and HOPH 1:1
    ph = _workload_params(H, w)
    hidx = H.Index(ph, H.sketch_oph(ph, ids, offs))
    hq = H.sketch_oph(ph, qids, qoffs)
    for name, idx, qs, goph in (("goph10", goph10, gq, True), ("hoph11", hidx, hq, False)):
        out[f"{name}_eps"] = [point(idx, qs, goph, (7, 10), (1, e)) for e in (100, 1000, 10_000, 100_000, 1_000_000)]
        out[f"{name}_T"] = [point(idx, qs, goph, (t, 10), (1, 10000)) for t in (5, 6, 7, 8, 9)]
        log(f"{name}: eps and T sweeps done")
    # (4) the paper's methods on the same data at the defaults: GOPH n = 10 (above),
    # HOPH 1:2, 1:1, 2:1 and plain OPH over all bins at k = 256 in groups of 32 (ratios
    # other than 1:1 need the smaller k for the exact 64-bit state), MinWise with 256
    # hashes (host wall time per batch of 128 queries, its kernel has no device timer)
    T7, e4 = (7, 10), (1, 10000)
    meth = {"goph_n10_k320": out["goph10_T"][2]}
    for ra, rb in ((1, 2), (1, 1), (2, 1)):
        pr = H.SketchParams(W.LAYOUT_HIER, 256, 32, w.hash_kind, w.universe, ra, rb, w.ha, w.hb)
        ix = H.Index(pr, H.sketch_oph(pr, ids, offs))
        meth[f"hoph{ra}{rb}_k256"] = point(ix, H.sketch_oph(pr, qids, qoffs), False, T7, e4)
        ix.free()
    po = H.SketchParams(W.LAYOUT_OPH, 256, 32, w.hash_kind, w.universe, 1, 1, w.ha, w.hb)
    ix = H.Index(po, H.sketch_oph(po, ids, offs))
    oq = H.sketch_oph(po, qids, qoffs)
    meth["oph_full_k256"] = point(ix, oq, True, T7, e4, call=lambda: H.query_oph_full(ix, oq, T=T7))
    ix.free()
    ha, hb = W.hash_coeffs(W.P31, 256, args.seed + 5)
    mp = H.MinwiseParams(256, W.HASH_MODP31, w.universe, torch.from_numpy(ha.view(np.int64)).to(dev),
                         torch.from_numpy(hb.view(np.int64)).to(dev))
    msig = H.minwise_sketch(mp, ids, offs)
    mq = H.minwise_sketch(mp, qids, qoffs)[:128].contiguous()
    meth["minwise_k256_128q"] = point(None, None, False, T7, e4, nq=128,
                                      call=lambda: H.minwise_query(mp, msig, mq, T=T7))
    del msig, mq
    out["methods"] = meth
    log("methods done")
    goph10.free()
    hidx.free()
    out["value"] = out["hoph11_T"][2]["pairs_per_s"]
    print(json.dumps(out), flush=True)


def _code_pass_shape(H, p, T, eps, goph=False):
    """(depth, plane words W, first-phase planes P1, lane-ops per pair and coded
    group, bytes of one query record) of the coarse pass on codes, as the
    library picks them (see the step's accounting below)."""
    tabs = H.decision_tables(p, T, eps)
    kp, k = p.k_group, p.k
    unit0 = tabs["W"][0] * tabs["dmul"][0]
    m_rej0 = tabs["rej"][0] // unit0 if tabs["rej"][0] >= 0 else -1
    W_planes = 1 if kp <= 32 else 2
    depth, split = None, 0
    if m_rej0 >= 0 and 8 * m_rej0 >= kp:
        depth = 1
        dthr = kp - m_rej0
        split = 2 if 2 * dthr <= kp else (4 if 4 * dthr <= 3 * kp else 0)
    ops = W_planes * (split + 2) + 1 if split else 10 * W_planes + 1
    rec_bytes = (8 * W_planes + 4) * 4
    return depth, W_planes, split, ops, rec_bytes


def bench_scansweep(args):
    """The coarse pass (first group on 8-bit codes) against the query batch
    size Q on two resident HOPH (1:1) indexes: the default step's 1,000,000
    bag-of-visual-words sets at k = 512, and 8,000,000 sets at k = 256 (the
    serving index), groups of 32, T = 4/5, eps = 1e-4.  Per Q: the mean device
    time of one coarse pass with a 1 GiB read before each pass (cold: the
    planes come from HBM; the reads' own time is subtracted), and back to back
    (warm: the planes of the 1,000,000-set index stay in the 256 MB last-level
    cache), its
    algorithmic bytes (each set's first-group code planes, 32 bytes, plus the
    query records) over that time against the HBM peak, its 32-bit lane-ops
    against the VALU peak, and the host wall time of one whole query_hoph call
    (tables, records, coarse and fine passes, output, read-back)."""
    import numpy as np
    import torch
    import paper_1805_11254_amd as H
    import workloads as W
    dev = torch.device("cuda")
    qs_list = [int(x) for x in args.sweep_q.split(",")]
    a, b = W.hash_coeffs(W.P31, 1, args.seed + 3)
    T, eps = (4, 5), (1, 10000)
    qmax = max(qs_list)
    qsets = W.zipf_sets(qmax, 1 << 20, 600, 0.75, 100, 4000, args.seed + 1)
    out = {"metric": "coarse pass HBM rate against query batch size", "unit": "GB/s", "mode": "scansweep",
           "indexes": []}
    # read before every cold pass: four times the 256 MB last-level cache
    flush = torch.zeros(1 << 30, dtype=torch.uint8, device=dev)
    sizes = [int(x) for x in args.sweep_sets.split(",")]
    for N in sizes:
        k = 512 if N <= 2_000_000 else 256
        p = H.SketchParams(W.LAYOUT_HIER, k, 32, W.HASH_MODP31, 1 << 20, 1, 1, int(a[0]), int(b[0]))
        idx = _resident_index(H, p, N, args.seed)
        qids, qoffs = (torch.from_numpy(qsets.ids.view(np.int32)).to(dev),
                       torch.from_numpy(qsets.offsets.view(np.int64)).to(dev))
        qsig = H.sketch_oph(p, qids, qoffs)
        H.sync()
        depth, Wp, split, ops, rec_bytes = _code_pass_shape(H, p, T, eps)
        rows = []
        for Q in qs_list:
            q = qsig[:Q].contiguous()
            reps = max(5, min(200, int(2e9 // (N * 32 + 1) // max(1, Q // 16 + 1))))
            warm_ms = min(H.scan_timing(idx, q, T=T, eps=eps, reps=reps) for _ in range(3))
            kms = min(H.scan_timing(idx, q, T=T, eps=eps, reps=min(reps, 40), flush=flush) for _ in range(3))
            H.query_hoph(idx, q, T=T, eps=eps)        # warm (tables cached, buffers grown)
            walls, phases = [], []
            for _ in range(max(5, args.steps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                H.query_hoph(idx, q, T=T, eps=eps)
                walls.append(time.perf_counter() - t0)
                phases.append(idx.last_query_ms())
            byts = N * 32 * Wp * depth + Q * rec_bytes * depth
            gbs = byts / (kms * 1e-3) / 1e9
            valu = Q * N * depth * ops / (kms * 1e-3)
            rows.append({"Q": Q, "coarse_kernel_ms": kms, "coarse_kernel_ms_warm": warm_ms,
                         "hbm_gbs_warm": byts / (warm_ms * 1e-3) / 1e9, "launches_timed": reps,
                         "algorithmic_bytes": byts,
                         "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS, "valu_ops_per_s": valu,
                         "valu_frac": valu / ALU_PEAK_OPS, "pairs_per_s_kernel": Q * N / (kms * 1e-3),
                         "query_call_ms_p50": 1e3 * float(np.median(walls)),
                         "query_events_ms": [float(np.median([x[i] for x in phases])) for i in range(3)]})
            log(f"N={N} Q={Q}: coarse {kms * 1e3:.1f} us cold, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.2f}); "
                f"warm {warm_ms * 1e3:.1f} us; VALU {valu / ALU_PEAK_OPS:.2f}, "
                f"call {rows[-1]['query_call_ms_p50']:.3f} ms")
        # the ridge: the largest Q whose pass is still at least 0.6 of the peak rate
        hbm_ok = [r["Q"] for r in rows if r["hbm_frac"] >= 0.6]
        out["indexes"].append({"n_sets": N, "k": k, "k_group": 32, "depth": depth, "first_phase_planes": split,
                               "ops_per_pair": ops, "rows": rows,
                               "largest_q_at_0_6_hbm": max(hbm_ok) if hbm_ok else None})
        idx.free()
        del qsig
        torch.cuda.empty_cache()
    out["value"] = max(r["hbm_gbs"] for ix in out["indexes"] for r in ix["rows"])
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.mode != "step":
        if args.gpus != 1:
            print("bench.py measures one GPU (--gpus 1)", file=sys.stderr)
            sys.exit(2)
        import paper_1805_11254_amd as H
        H.lib()
        {"batched": bench_batched, "serve": bench_serve, "comparators": bench_comparators,
         "selfjoin": bench_selfjoin, "sweeps": bench_sweeps, "scansweep": bench_scansweep}[args.mode](args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}); "
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
    w = W.hoph_bovw(n=args.n_sets or 1_000_000, n_q=args.n_queries, seed=args.seed)
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
        # one pass of the path: every set sketched straight into the resident
        # index (rows + code planes), the query batch sketched, the HOPH scan
        e = ev or [None] * 4
        if e[0] is not None: e[0].record(stream)
        idx.reset()
        idx.append_sets(ids, offs)
        if e[1] is not None: e[1].record(stream)
        H.sketch_oph(p, qids, qoffs, out=qsig)
        if e[2] is not None: e[2].record(stream)
        out = H.query_hoph(idx, qsig, T=w.T, eps=w.eps, capacity=cap[0])
        if e[3] is not None: e[3].record(stream)
        return out

    for i in range(args.warmup):
        out = step()
        if cap[0] is None:
            cap[0] = max(1 << 16, 2 * int(out[1].numel()))
    H.sync()
    torch.cuda.synchronize()
    log("warm-up done")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    qms, ams = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step(evs[i])
        qms.append(idx.last_query_ms())
        ams.append(idx.last_append_ms())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1000.0 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")

    def mean_ms(a, b):
        return sum(e[a].elapsed_time(e[b]) for e in evs) / len(evs)

    build_ms = mean_ms(0, 1)
    qsketch_ms = mean_ms(1, 2)
    query_ms = mean_ms(2, 3)
    sketch_ms = sum(a[0] for a in ams) / len(ams)       # the sketch-into-index kernel
    codes_ms = sum(a[1] for a in ams) / len(ams)        # code planes from the rows

    # the two-step build (row-major signatures, then the index store), for comparison
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    two = []
    for _ in range(3):
        e0.record(stream)
        H.sketch_oph(p, ids, offs, out=sig)
        e1.record(stream)
        idx.reset()
        idx.append(sig)
        e2.record(stream)
        torch.cuda.synchronize()
        two.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
    two_sketch_ms = sum(t[0] for t in two) / len(two)
    index_ms = sum(t[1] for t in two) / len(two)

    # the HBM rate a plain device copy reaches here (2 GiB, same stream): the
    # practical ceiling the sketch's rate is also compared with
    cbuf = torch.empty(1 << 29, dtype=torch.int32, device=dev)
    cdst = torch.empty_like(cbuf)
    cdst.copy_(cbuf)
    e0.record(stream)
    for _ in range(5):
        cdst.copy_(cbuf)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * cbuf.numel() * 4 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del cbuf, cdst
    # the sketch with the sets handed over in pinned host memory: host-to-device
    # copy of ids and offsets, then the sketch (the resident copies are overwritten
    # with the same contents)
    ids_pin = torch.from_numpy(w.collection.ids.view(np.int32)).pin_memory()
    offs_pin = torch.from_numpy(w.collection.offsets.view(np.int64)).pin_memory()
    h2d = []
    for _ in range(2):
        e0.record(stream)
        ids.copy_(ids_pin, non_blocking=True)
        offs.copy_(offs_pin, non_blocking=True)
        e1.record(stream)
        H.sketch_oph(p, ids, offs, out=sig)
        e2.record(stream)
        torch.cuda.synchronize()
        h2d.append((e0.elapsed_time(e1), e0.elapsed_time(e2)))
    h2d_copy_ms, h2d_total_ms = min(h[0] for h in h2d), min(h[1] for h in h2d)
    del ids_pin, offs_pin
    coarse_ms = sum(q[0] for q in qms) / len(qms)
    fine_ms = sum(q[1] for q in qms) / len(qms)
    sort_ms = sum(q[2] for q in qms) / len(qms)

    # algorithmic work per launch
    sketch_bytes = nnz * 4 + (N + 1) * 8 + N * k * 4                 # ids, offsets in; signatures out
    # groups that carry 8-bit codes, in code units of pk whole groups (pk = min(32 // k', L)
    # for k' <= 16, else 1): at least 4 units, about 128 bins (HOPH) or 256 (GOPH), at most
    # 24 units (12 for k' > 32), none past the row
    L_groups = k // kp
    pk = min(32 // kp, L_groups) if kp <= 16 else 1
    code_units = min(L_groups // pk, max(4, min(12 if kp > 32 else 24, -(-(256 if w.goph else 128) // (pk * kp)))))
    code_groups = code_units * pk
    code_bytes = N * code_groups * kp * 4 + N * code_units * 32 * (1 if kp <= 32 else 2)
    index_bytes = 2 * N * k * 4 + N * code_units * 32 * (1 if kp <= 32 else 2)   # rows in, index rows + code planes out
    # coarse depth as the library picks it: the first group alone when it rejects at
    # least 1/8 of its match counts (no empty bins), else one group past the first
    # step with a reject cutoff, rounded up to whole code units
    tabs = H.decision_tables(p, w.T, w.eps)
    unit0 = tabs["W"][0] * tabs["dmul"][0]
    m_rej0 = tabs["rej"][0] // unit0 if tabs["rej"][0] >= 0 else -1
    if m_rej0 >= 0 and 8 * m_rej0 >= kp:
        depth = 1
    else:   # one group past the first step with a reject cutoff, in whole code units
        g1 = next((l + 1 for l, r in enumerate(tabs["rej"]) if r >= 0), None)
        depth = code_groups if g1 is None else min(code_groups, -(-(g1 + 1) // pk) * pk)
    # coarse pass on 8-bit bin codes held as 8 bit-planes of 32 bins per word:
    # per (pair, group) 8 W plane operations, W masks, W popcounts, 1 compare.
    # The first-group pass compares the first P1 planes of every pair first and
    # the rest only where a lane might still survive (P1 = 2 when the threshold
    # on differing bins is at most half the bins, 4 when at most three
    # quarters): the work every pair gets is then P1 W plane operations, W
    # masks, W popcounts and 1 compare.
    W_planes = 1 if kp <= 32 else 2
    ops_per_pair_group = 10 * W_planes + 1
    plane_split = 0
    if depth == 1 and w.T is not None:
        dthr = kp + 1 if m_rej0 < 0 else kp - m_rej0
        plane_split = 2 if 2 * dthr <= kp else (4 if 4 * dthr <= 3 * kp else 0)
        if plane_split:
            ops_per_pair_group = W_planes * (plane_split + 2) + 1
    coarse_ops = Q * N * depth * ops_per_pair_group
    coarse_bins = Q * N * kp * depth
    coarse_bytes = N * 32 * W_planes * depth + Q * (32 * W_planes + 16) * depth
    traffic = load_traffic()
    kernels = {
        "sketch_into_index": {"ms": sketch_ms, "bound": "hbm", "achieved": sketch_bytes / (sketch_ms * 1e-3) / 1e9,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": traffic.get("sketch_kernel"),
                              "algorithmic_bytes": sketch_bytes, "sets_per_s": N / (sketch_ms * 1e-3)},
        "code_planes": {"ms": codes_ms, "bound": "hbm", "achieved": code_bytes / (codes_ms * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": traffic.get("row_codes_vec_kernel"),
                        "algorithmic_bytes": code_bytes},
        "two_step_sketch_oph": {"ms": two_sketch_ms, "bound": "hbm",
                                "achieved": sketch_bytes / (two_sketch_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "traffic": traffic.get("sketch_kernel"),
                                "algorithmic_bytes": sketch_bytes},
        "two_step_index_store": {"ms": index_ms, "bound": "hbm", "achieved": index_bytes / (index_ms * 1e-3) / 1e9,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "traffic": (traffic["__amd_rocclr_copyBuffer"] + traffic["row_codes_vec_kernel"]
                                             if "__amd_rocclr_copyBuffer" in traffic and "row_codes_vec_kernel" in traffic
                                             else None),
                                 "algorithmic_bytes": index_bytes},
        "scan_coarse": {"ms": coarse_ms, "bound": "alu", "achieved": coarse_ops / (coarse_ms * 1e-3) / 1e12,
                        "peak": ALU_PEAK_OPS / 1e12, "unit": "Tops/s (32-bit VALU lane-ops)",
                        "ops_per_pair_group": ops_per_pair_group, "first_phase_planes": plane_split,
                        "bin_compares_per_s": coarse_bins / (coarse_ms * 1e-3),
                        "traffic": traffic.get("scan_codes_fast_kernel"), "algorithmic_bytes": coarse_bytes,
                        "hbm_gbs": coarse_bytes / (coarse_ms * 1e-3) / 1e9, "depth": depth},
        "scan_fine": {"ms": fine_ms},
        "sort_and_csr": {"ms": sort_ms},
        "query_sketch": {"ms": qsketch_ms},
    }
    for v in kernels.values():
        if "achieved" in v:
            v["frac"] = v["achieved"] / v["peak"]
    dom_name = max(("sketch_into_index", "code_planes", "scan_coarse"), key=lambda n: kernels[n]["ms"])
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
        "sets_sketched_per_s_with_h2d": N / (h2d_total_ms * 1e-3),
        "h2d_gbs": (nnz * 4 + (N + 1) * 8) / (h2d_copy_ms * 1e-3) / 1e9,
        "copy_ceiling_gbs": copy_gbs,
        "sketch_frac_of_copy": kernels["sketch_into_index"]["achieved"] / copy_gbs,
        "scan_pairs_per_s": N * Q / (query_ms * 1e-3),
        "scan_hbm_frac": kernels["scan_coarse"]["hbm_gbs"] / HBM_PEAK_GBS,
        "served_p99_ms": None,
        "phase_ms": {"build_index": build_ms, "sketch_into_index": sketch_ms, "code_planes": codes_ms,
                     "query_sketch": qsketch_ms, "query": query_ms, "coarse": coarse_ms, "fine": fine_ms,
                     "sort_csr": sort_ms, "two_step_sketch": two_sketch_ms, "two_step_index_store": index_ms},
        "kernels": kernels,
        "roofline": roofline,
        "accepted_pairs": len(got),
        "recall_planted": recall,
        "precision_exact_jaccard": precision,
    }
    if args.serve_rate > 0:
        # serving on the same resident index, outside the timed region: Poisson
        # arrivals of single query sets (log-normal sizes, median 800 ids) at a
        # fixed rate, after a warm-up replay (tuning, graph capture); latency per
        # request from arrival to its result list
        log(f"serving at {args.serve_rate:.0f} q/s for {args.serve_seconds} s")
        srv = H.Server(idx, p, T=w.T, eps=w.eps, slots=4, max_batch_queries=2048, max_batch_ids=1 << 22,
                       max_batch_results=1 << 20, use_graph=True, tune=True)
        # warm-up at the measured rate, so that every slot has run (tuned and
        # captured its graph on) its first batch before the measurement
        t_w, wq = W.poisson_arrivals(args.serve_rate, max(1, int(args.serve_rate * 0.1)), args.seed + 70)
        srv.replay(wq.ids, wq.offsets, t_w - t_w[0])
        n_req = max(1, int(args.serve_rate * args.serve_seconds))
        t_s, sq = W.poisson_arrivals(args.serve_rate, n_req, args.seed + 71)
        srv.reset_stats()
        srv.replay(sq.ids, sq.offsets, t_s - t_s[0])
        st = srv.stats()
        srv.close()
        rec["served_p99_ms"] = st["p99_ms"]
        rec["serving"] = {"offered_qps": args.serve_rate, "requests": n_req,
                          "served_qps": st["completed"] / max(st["busy_s"], 1e-9), "p50_ms": st["p50_ms"],
                          "p99_ms": st["p99_ms"], "mean_batch": st["mean_batch_queries"],
                          "index_sets": len(idx)}
    idx.free()
    if not args.no_cpu_baseline:
        log("timing the oracle on a CPU sample")
        rec["cpu_baseline"] = cpu_baseline(w, N, Q, args.cpu_sample_sets, args.cpu_sample_queries)
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
