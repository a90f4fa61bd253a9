"""Write the stored expected values for the large parity cases.

Calls only the CPU oracle (oracle/) on the seeded generators; nothing here
touches the HIP library. Run from the repository root:
    python tests/golden/make_golden.py [cfg2] [cfg3] [cfg2q]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2605_03603_amd import generators as G  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
THREADS = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def degree(n, ids):
    return np.bincount(ids.astype(np.int64), minlength=n)


def pick(rng, deg, lo, hi, k):
    idx = np.flatnonzero((deg >= lo) & (deg <= hi))
    return sorted(int(x) for x in rng.choice(idx, size=min(k, idx.size), replace=False))


def cfg2():
    g = G.config2(1)
    t = time.time()
    ru = O.count_bbvp(g, side=0, threads=THREADS, per_vertex=True)
    rv = O.count_bbvp(g, side=1, threads=THREADS, per_vertex=True)
    assert ru["total"] == rv["total"]
    pu, pv = ru["per_vertex"], rv["per_vertex"]
    assert int(pu.sum()) == 3 * ru["total"] == int(pv.sum())
    rng = np.random.default_rng(12)
    su = sorted(int(x) for x in rng.choice(g.n_u, 64, replace=False))
    out = {
        "workload": "config2 seed 1: Chung-Lu 100000 x 50000, 2M edges, gamma 2.1/2.1, 80% positive, "
                    "200 balanced + 200 random 12x12 planted blocks",
        "source": "oracle/ Algorithm 2 (p=q=3) anchored on U and on V (tests/golden/make_golden.py)",
        "n_u": g.n_u, "n_v": g.n_v, "m": g.m,
        "total": ru["total"],
        "feasible_triplets_u": ru["feasible"], "candidate_pairs_u": ru["candidates"],
        "feasible_triplets_v": rv["feasible"], "candidate_pairs_v": rv["candidates"],
        "per_u_sha256": digest(pu), "per_v_sha256": digest(pv),
        "per_u_sample": {str(x): int(pu[x]) for x in su},
        "oracle_seconds": round(time.time() - t, 1), "oracle_threads": THREADS,
    }
    with open(os.path.join(HERE, "cfg2_seed1.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("cfg2", out["total"], out["oracle_seconds"])


def cfg3():
    g = G.config3(1)
    du, dv = degree(g.n_u, g.eu), degree(g.n_v, g.ev)
    rng = np.random.default_rng(13)
    xs_u = pick(rng, du, 3, 30, 40) + pick(rng, du, 31, 300, 16)
    xs_v = pick(rng, dv, 3, 30, 16) + pick(rng, dv, 31, 200, 8)
    t = time.time()
    cu = O.vertex_counts(g, 0, xs_u)
    cv = O.vertex_counts(g, 1, xs_v)
    out = {
        "workload": "config3 seed 1: Chung-Lu 2M x 500k, 40M edges, gamma 1.9/2.3, hidden-label signs "
                    "with 10% flips",
        "source": "oracle/ per-vertex counts (tests/golden/make_golden.py)",
        "n_u": g.n_u, "n_v": g.n_v, "m": g.m,
        "per_u_sample": {str(x): c for x, c in zip(xs_u, cu)},
        "per_v_sample": {str(x): c for x, c in zip(xs_v, cv)},
        "oracle_seconds": round(time.time() - t, 1),
    }
    with open(os.path.join(HERE, "cfg3_seed1_sample.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("cfg3 sample", out["oracle_seconds"])


def cfg2q():
    """Balanced (3, q) and (q, 3) counts of config 2 for q = 4, 5: Algorithm 2
    with that q, anchored on U and on V respectively."""
    g = G.config2(1)
    t = time.time()
    counts = {}
    for q in (4, 5):
        counts[f"3,{q}"] = O.count_bbvp_q(g, q, 0, threads=THREADS)["total"]
        counts[f"{q},3"] = O.count_bbvp_q(g, q, 1, threads=THREADS)["total"]
    out = {
        "workload": "config2 seed 1 (as cfg2_seed1.json)",
        "source": "oracle/ Algorithm 2 with p = 3 on the anchor side and q on the other "
                  "(orc_count_bbvp_q; (q, 3) anchored on V) (tests/golden/make_golden.py)",
        "m": g.m, "counts": counts,
        "oracle_seconds": round(time.time() - t, 1), "oracle_threads": THREADS,
    }
    with open(os.path.join(HERE, "cfg2_seed1_general_q.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("cfg2q", counts, out["oracle_seconds"])


if __name__ == "__main__":
    which = sys.argv[1:] or ["cfg2", "cfg3", "cfg2q"]
    O.build()
    for w in which:
        globals()[w]()
