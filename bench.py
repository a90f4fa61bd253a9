#!/usr/bin/env python3
"""Benchmark: exact balanced (3,3)-biclique counting on one MI355X.

One step = the whole hot path on the config-2 workload (Chung-Lu signed
bipartite graph, 100000 x 50000, ~2M edges, seed 1) with the COO already in
HBM: validation, degrees, priority ranking and both CSR orientations
(bbc_build_csr with device pointers), then the pair-table, planning and
triplet kernels and the int64 reduction (bbc_count_global). The count is
checked against the oracle's stored value every step.

value = triplets/s, where the number of triplets is a property of the graph:
the same-side (U) triples with at least 3 common neighbours (the survivors of
the |T| < q test of Algorithm 2), counted by the CPU oracle and stored in
tests/golden/cfg2_seed1.json. It does not depend on how the GPU enumerates.

Also reported on the same JSON line:
  roofline      the dominant kernel's achieved rate vs its bound
  roofline_other_phases  the same for the other phases (triplets, CSR build)
  cpu_baseline  the CPU oracle on a bounded sample of the same workload
  batched       8192-graph batch (one build + one persistent, graph-replayed
                count) vs the same graphs built and counted one at a time
  served        Poisson request stream over the batched mix plus 2% config-2
                sized graphs: p50 / p99 latency and graphs/s
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "triplets/s + time to exact count; batched vs per-graph; serve p50/p99 ms"
HBM_PEAK_GBS = 8000.0
MFMA_FP4_PEAK_TFLOPS = 10100.0   # dense fp4 matrix-core peak of MI355X


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def load_golden():
    with open(os.path.join(ROOT, "tests", "golden", "cfg2_seed1.json")) as f:
        return json.load(f)


def source_digest(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2605_03603_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_key, digest):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel_key}_config2_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != digest:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(g, stride, threads):
    from oracle import oracle as O
    O.build()
    t = time.time()
    r = O.count_bbvp(g, side=0, threads=threads, anchor_stride=stride)
    dt = time.time() - t
    return {"value": r["feasible"] / dt, "unit": "triplets/s", "cores": threads, "kind": "oracle",
            "sample": f"U anchors with id % {stride} == 0 of config2 seed 1 "
                      f"({r['feasible']} triplets, {r['candidates']} candidate pairs, {dt:.1f} s)"}


def run_batched(ctx, gs, torch):
    from paper_2605_03603_amd import generators as G
    nu, nv, off, eu, ev, sg = G.concat(gs)
    dev = torch.device("cuda:0")
    d_eu = torch.from_numpy(eu.view(np.int32)).to(dev)
    d_ev = torch.from_numpy(ev.view(np.int32)).to(dev)
    d_sg = torch.from_numpy(sg).to(dev)
    torch.cuda.synchronize()
    # warm up: sizes the workspace, tunes the launch shape, captures the graph
    hs = ctx.build_csr_batch(nu, nv, off, d_eu, d_ev, d_sg)
    ref = ctx.count_batch(hs)
    for h in hs:
        h.free()
    reps = 3
    torch.cuda.synchronize()
    t = time.time()
    for _ in range(reps):
        hs = ctx.build_csr_batch(nu, nv, off, d_eu, d_ev, d_sg)
        got = ctx.count_batch(hs)
        for h in hs:
            h.free()
    torch.cuda.synchronize()
    t_batch = (time.time() - t) / reps
    assert np.array_equal(got, ref)
    # the same graphs, one build and one count each
    offs = off.astype(np.int64)
    t = time.time()
    per = np.zeros(len(gs), np.int64)
    for i, g in enumerate(gs):
        a, b = int(offs[i]), int(offs[i + 1])
        h = ctx.build_csr(int(nu[i]), int(nv[i]), d_eu[a:b], d_ev[a:b], d_sg[a:b])
        per[i] = ctx.count_global(h)
        h.free()
    torch.cuda.synchronize()
    t_per = time.time() - t
    return ref, {
        "graphs": len(gs), "edges": int(off[-1]),
        "batched_ms": round(1e3 * t_batch, 3), "per_graph_ms": round(1e3 * t_per, 3),
        "batched_graphs_per_s": round(len(gs) / t_batch, 1),
        "per_graph_graphs_per_s": round(len(gs) / t_per, 1),
        "speedup": round(t_per / t_batch, 2),
        "counts_equal": bool(np.array_equal(per, ref)),
        "total_count": int(ref.sum()),
    }


def run_served(ctx, pool, pool_counts, large, large_counts, n_requests, qps, seed):
    rng = np.random.default_rng([5, seed])
    arrivals = np.cumsum(rng.exponential(1.0 / qps, size=n_requests))
    picks = []
    for _ in range(n_requests):
        if large and rng.random() < 0.02:
            picks.append(("L", int(rng.integers(0, len(large)))))
        else:
            picks.append(("S", int(rng.integers(0, len(pool)))))
    from collections import deque
    pending = deque()     # (ticket, arrival time, kind, index) in submission order
    lat = []
    wrong = 0
    t0 = time.time()
    nxt = 0
    while nxt < n_requests or pending:
        now = time.time() - t0
        while nxt < n_requests and arrivals[nxt] <= now:
            kind, i = picks[nxt]
            g = pool[i] if kind == "S" else large[i]
            tk = ctx.submit_coo(g.n_u, g.n_v, g.eu, g.ev, g.sign)
            pending.append((tk, t0 + arrivals[nxt], kind, i))
            nxt += 1
        # results come back batch by batch, roughly in submission order: poll
        # a bounded window at the front
        progressed = False
        for _ in range(min(64, len(pending))):
            tk, ta, kind, i = pending.popleft()
            v = ctx.poll(tk)
            if v is None:
                pending.append((tk, ta, kind, i))
                continue
            lat.append(time.time() - ta)
            want = pool_counts[i] if kind == "S" else large_counts[i]
            wrong += int(v != want)
            progressed = True
        if not progressed:
            time.sleep(0.0001)
    wall = time.time() - t0
    lat = np.array(lat) * 1e3
    return {"requests": n_requests, "offered_qps": round(qps, 1),
            "graphs_per_s": round(n_requests / wall, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3),
            "large_fraction": round(sum(1 for k, _ in picks if k == "L") / n_requests, 4),
            "wrong_counts": wrong}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-stride", type=int, default=2)
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--batch-graphs", type=int, default=8192)
    ap.add_argument("--serve-requests", type=int, default=3000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-edges", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-general-q", action="store_true",
                    help="skip the timing of the (3, q) and (q, 3) counts, q = 4..7")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (5 times), the reference for "
                         "the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_03603_amd import bbc, generators as G

    if args.copy_calibration:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 5}))
        return

    gold = load_golden()
    log("generating config2 seed 1")
    g = G.config2(1)
    assert g.m == gold["m"], "generator output differs from the stored workload"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ctx = bbc.Context(0, stream=stream)
    ctx.set_timing(True)
    d_eu = torch.from_numpy(g.eu.view(np.int32)).to(dev)
    d_ev = torch.from_numpy(g.ev.view(np.int32)).to(dev)
    d_sg = torch.from_numpy(g.sign).to(dev)
    torch.cuda.synchronize()

    def step():
        h = ctx.build_csr(g.n_u, g.n_v, d_eu, d_ev, d_sg)
        st_build = ctx.last_stats()["ms_build"]
        c = ctx.count_global(h)
        side = h.info().anchor_side
        h.free()
        st = ctx.last_stats()
        st["ms_build"] = st_build
        return c, side, st

    log("warmup", args.warmup)
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    log("timed steps", args.steps)
    kern = {"ms_build": 0.0, "ms_pair": 0.0, "ms_plan": 0.0, "ms_triplet": 0.0}
    counts = set()
    t0 = time.time()
    for _ in range(args.steps):
        c, side, st = step()
        counts.add(c)
        for k in kern:
            kern[k] += st[k]
    torch.cuda.synchronize()
    t1 = time.time()
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    count_ok = counts == {gold["total"]}
    triplets = gold["feasible_triplets_u"]
    value = triplets / (ms_per_step / 1e3)
    kern_avg = {k: round(v / args.steps, 4) for k, v in kern.items()}

    # end-to-end from host COO (includes the PCIe upload)
    t = time.time()
    reps = 3
    for _ in range(reps):
        h = ctx.build_csr(g.n_u, g.n_v, g.eu, g.ev, g.sign)
        ctx.count_global(h)
        h.free()
    e2e_ms = 1e3 * (time.time() - t) / reps

    # roofline of each phase; the dominant one is reported as "roofline"
    digest = source_digest(["count.hip", "bbc_dev.h", "bbc_count.h"])

    def roof_triplet():
        # |M_x n M_y| over all examined pairs as 0/1 products: 32 bits per
        # mask word, a multiply and an add each. Masks of 3 words and more run
        # on the fp4 matrix cores, 1 and 2 words on the int8 ones; the fp4
        # peak (the higher) is the bound.
        ops = 64.0 * st["pair_words"]
        achieved = ops / (kern_avg["ms_triplet"] / 1e3) / 1e12
        return {"kernel": "triplet phase: k_triplet<0,0> + k_triplet<0,1>", "bound": "mfma",
                "achieved": round(achieved, 3), "peak": MFMA_FP4_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / MFMA_FP4_PEAK_TFLOPS, 4),
                "algorithmic_ops_per_launch": ops,
                "traffic": traffic_from_profile("triplet", digest)}

    def roof_pair():
        # one read of every oriented wedge's entry, the suffix table, and the
        # mask words written
        byts = 4.0 * st["wedges"] + 8.0 * g.m + 4.0 * st["mask_words"]
        achieved = byts / (kern_avg["ms_pair"] / 1e3) / 1e9
        return {"kernel": "pair phase: k_pair_wave + k_pair_lds + k_pair_big + 2 x k_pair_global",
                "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "algorithmic_bytes_per_launch": byts,
                "traffic": traffic_from_profile("pair", digest)}

    def roof_build():
        byts = 17.5 * g.m
        achieved = byts / (kern_avg["ms_build"] / 1e3) / 1e9
        return {"kernel": "csr build", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "algorithmic_bytes_per_launch": byts, "traffic": None}

    phases = {"ms_triplet": roof_triplet, "ms_pair": roof_pair, "ms_build": roof_build}
    dominant = max(phases, key=lambda k: kern_avg[k])
    roof = phases[dominant]()
    roof_other = [phases[k]() for k in sorted(phases, key=lambda k: -kern_avg[k]) if k != dominant]

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "triplets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "config2: Chung-Lu signed bipartite, |U|=100000, |V|=50000, "
                               "gamma 2.1/2.1, 80% positive, 200 balanced + 200 random-sign 12x12 "
                               "planted blocks, seed 1",
                   "n_u": g.n_u, "n_v": g.n_v, "n_edges": g.m, "anchor_side": "UV"[side],
                   "triplets": triplets, "parallelism": "1 GPU"},
        "count": sorted(counts)[0] if len(counts) == 1 else sorted(counts),
        "count_ok": count_ok,
        "time_to_exact_count_ms": {"resident_coo": round(ms_per_step, 3),
                                   "host_coo_e2e": round(e2e_ms, 3)},
        "kernel_ms": kern_avg,
        "last_count_stats": {k: st[k] for k in ("active_anchors", "virtual_candidates", "mask_words",
                                                 "pair_units", "candidate_pairs", "pair_words",
                                                 "wedges", "attempts", "deferred_a", "deferred_b",
                                                 "deferred_c", "deferred_d")},
        "roofline": roof,
        "roofline_other_phases": roof_other,
    }

    if not args.no_general_q:
        # balanced (3, q) on a U-anchored build and (q, 3) on a V-anchored one,
        # same workload; exactness against the oracle is in the GPU tests
        log("general q")
        gq = {"(3,q)": {}, "(q,3)": {}}
        for flags, key in ((1 << 4, "(3,q)"), (1 << 5, "(q,3)")):
            h = ctx.build_csr(g.n_u, g.n_v, d_eu, d_ev, d_sg, flags)
            for q in range(4, 8):
                pq = (3, q) if key == "(3,q)" else (q, 3)
                ts = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    t = time.time()
                    c = ctx.count_global(h, *pq)
                    ts.append(1e3 * (time.time() - t))
                gq[key][str(q)] = {"count": c, "ms": round(sorted(ts)[1], 3)}
            h.free()
        # 4 vertices on the anchor side (triples of candidates), one count each
        for pq in ((4, 3), (4, 4)):
            h = ctx.build_csr(g.n_u, g.n_v, d_eu, d_ev, d_sg, 1 << 4)
            ctx.count_global(h, *pq)                 # sizes the workspace
            torch.cuda.synchronize()
            t = time.time()
            c = ctx.count_global(h, *pq)
            gq["%d,%d" % pq] = {"count": c, "ms": round(1e3 * (time.time() - t), 1)}
            h.free()
        out["general_q"] = gq

    if not args.no_edges:
        # edge queries (balanced bicliques through an edge: the change of the
        # count on inserting, deleting or re-signing it), 20000 existing edges
        # with their own sign and 2000 new pairs in one call (batched);
        # exactness against the oracle is in the GPU tests
        log("edge queries")
        rng = np.random.default_rng(7)
        h = ctx.build_csr(g.n_u, g.n_v, d_eu, d_ev, d_sg, 1 << 4)
        ne, nn = 20000, 2000
        idx = rng.choice(g.m, size=ne, replace=False)
        qu = np.concatenate([g.eu[idx], rng.integers(0, g.n_u, nn)]).astype(np.uint32)
        qv = np.concatenate([g.ev[idx], rng.integers(0, g.n_v, nn)]).astype(np.uint32)
        qs = np.concatenate([g.sign[idx], np.ones(nn, np.int8)]).astype(np.int8)
        ctx.count_through_edges(h, qu[:64], qv[:64], qs[:64])
        torch.cuda.synchronize()
        t = time.time()
        through = ctx.count_through_edges(h, qu, qv, qs)
        ms = 1e3 * (time.time() - t)
        h.free()
        out["edge_queries"] = {"queries": int(qu.size), "ms_total": round(ms, 2),
                               "us_per_query": round(1e3 * ms / qu.size, 3),
                               "existing_edges_sum": int(through[:ne].sum()),
                               "new_pairs_sum": int(through[ne:].sum())}

    if not args.no_cpu:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        log("cpu baseline: oracle on every", args.cpu_stride, "th anchor,", threads, "threads")
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_stride, threads)

    if not args.no_batched or not args.no_serve:
        log("generating", args.batch_graphs, "batched graphs")
        gs = G.config4(1, n_graphs=args.batch_graphs)
        ref, batched = run_batched(ctx, gs, torch)
        if not args.no_batched:
            out["batched"] = batched
        if not args.no_serve:
            # capacity: 98% batched-mix graphs at the batched rate, 2% config-2
            # sized graphs at their end-to-end time; offer 70% of it
            per_req_s = 0.98 / batched["batched_graphs_per_s"] + 0.02 * e2e_ms / 1e3
            qps = 0.7 / per_req_s
            log("serving", args.serve_requests, "requests at", round(qps, 1), "qps")
            out["served"] = run_served(ctx, gs, ref, [g], [gold["total"]], args.serve_requests,
                                       qps, 1)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
