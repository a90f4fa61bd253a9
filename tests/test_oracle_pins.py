"""Pins of the CPU oracle to values fixed by the paper and by mathematics.

Nothing here runs on the GPU. Each test names the passage or fact it checks.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from paper_2605_03603_amd import generators as G

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def C3(n):
    return math.comb(n, 3)


# ------------------------------------------------------------- figure pins
def test_fig2_butterfly_balance(oracle):
    for case in load("fig2_butterflies.json")["cases"]:
        assert oracle.butterfly_balanced(*case["signs"]) == case["balanced"], case["label"]


def test_fig3b_wedge_types(oracle):
    for case in load("fig3b_wedge_types.json")["cases"]:
        assert oracle.wedge_type(*case["signs"]) == case["type"], case["label"]
        # negating every sign does not change the type (it compares signs)
        assert oracle.wedge_type(*[-s for s in case["signs"]]) == case["type"]


def test_fig1b_signed_k44(oracle):
    fx = load("fig1b.json")
    g = G.from_rows(fx["rows"])
    total, pu, pv = oracle.count_bruteforce(g, per_vertex=True)
    assert total == fx["balanced_33"]
    assert list(pu) == fx["per_u"] and list(pv) == fx["per_v"]
    for side, key in ((0, "per_u"), (1, "per_v")):
        r = oracle.count_bbvp(g, side=side, per_vertex=True)
        assert r["total"] == fx["balanced_33"]
        assert list(r["per_vertex"]) == fx[key]
    unsigned = G.from_rows(["++++"] * 4)
    assert oracle.count_bruteforce(unsigned) == fx["unsigned_33"]
    assert oracle.count_bbvp(unsigned)["total"] == fx["unsigned_33"]


def _fig4_graph(fx, signs=None):
    us = sorted(fx["adjacency"])
    vs = sorted({v for lst in fx["adjacency"].values() for v in lst})
    eu, ev = [], []
    for u in us:
        for v in fx["adjacency"][u]:
            eu.append(us.index(u)); ev.append(vs.index(v))
    s = np.ones(len(eu), np.int8) if signs is None else np.asarray(signs, np.int8)
    return G._finish(len(us), len(vs), np.array(eu), np.array(ev), s), us, vs


def test_fig4_worked_example(oracle):
    fx = load("fig4.json")
    g, us, vs = _fig4_graph(fx)
    a = us.index(fx["anchor"])
    # the figure takes u1 as the anchor with every other U vertex as partner
    d = oracle.anchor_detail(g, side=0, u=a, oriented=False)
    assert sorted(us[c] for c in d["candidates"]) == fx["candidate_set"]
    assert len(d["pairs"]) == fx["triplets"]
    for (w1, w2, size_t, *x) in d["pairs"]:
        key = ",".join(sorted([us[w1], us[w2]]))
        assert size_t == fx["wedge_pair_counts"][key]
        trip = ",".join(sorted([fx["anchor"], us[w1], us[w2]]))
        assert size_t == len(fx["common_neighbours"][trip])
        assert sum(x) == size_t
    # wedges from the anchor as Algorithm 1 would enumerate them
    adj = fx["adjacency"]
    wedges = sum(math.comb(sum(1 for u in us if v in adj[u] and u != fx["anchor"]), 2)
                 for v in adj[fx["anchor"]])
    assert wedges == fx["wedges_from_anchor"]
    # zero balanced (3,3)-bicliques for every one of the 2^12 sign assignments
    m = g.m
    for bits in range(1 << m):
        s = [1 if (bits >> i) & 1 else -1 for i in range(m)]
        gs, _, _ = _fig4_graph(fx, s)
        assert oracle.count_bruteforce(gs) == fx["balanced_33"]
        if bits % 97 == 0:
            assert oracle.count_bbvp(gs)["total"] == 0
            assert oracle.count_bbvp(gs, side=1)["total"] == 0


# ------------------------------------------------------------ closed forms
def complete(n, m, sign_fn):
    rows = ["".join("+" if sign_fn(i, j) > 0 else "-" for j in range(m)) for i in range(n)]
    return G.from_rows(rows)


@pytest.mark.parametrize("n,m", [(3, 3), (4, 5), (6, 4), (7, 7), (3, 9)])
def test_complete_all_positive(oracle, n, m):
    """All-positive K_{n,m}: every (3,3)-biclique is balanced: C(n,3) C(m,3)."""
    g = complete(n, m, lambda i, j: 1)
    want = C3(n) * C3(m)
    assert oracle.count_bruteforce(g) == want
    r0 = oracle.count_bbvp(g, 0, per_vertex=True)
    r1 = oracle.count_bbvp(g, 1, per_vertex=True)
    assert r0["total"] == r1["total"] == want
    # each U vertex lies in C(n-1,2) C(m,3) of them
    assert list(r0["per_vertex"]) == [math.comb(n - 1, 2) * C3(m)] * n
    assert list(r1["per_vertex"]) == [math.comb(m - 1, 2) * C3(n)] * m


@pytest.mark.parametrize("seed", range(5))
def test_rank_one_signs(oracle, seed):
    """Signs a(u) b(v) are a vertex switching of all-positive: same count."""
    rng = np.random.default_rng(seed)
    n, m = int(rng.integers(3, 9)), int(rng.integers(3, 9))
    a = rng.choice([-1, 1], n); b = rng.choice([-1, 1], m)
    g = complete(n, m, lambda i, j: a[i] * b[j])
    assert oracle.count_bbvp(g, 0)["total"] == C3(n) * C3(m)
    assert oracle.count_bruteforce(g) == C3(n) * C3(m)


@pytest.mark.parametrize("n1,n2,m1,m2", [(3, 4, 4, 3), (2, 5, 3, 3), (4, 4, 5, 2), (1, 6, 6, 1), (5, 3, 3, 5)])
def test_two_block_closed_form(oracle, n1, n2, m1, m2):
    """K_{n,m} with U = U1+U2, V = V1+V2 and sign -1 exactly on U2 x V2.
    Triples inside U1 or inside U2 have identical rows: any 3 columns.
    Mixed triples have rows equal on V1 and opposite on V2: columns all in V1
    or all in V2."""
    n, m = n1 + n2, m1 + m2
    g = complete(n, m, lambda i, j: -1 if (i >= n1 and j >= m1) else 1)
    pure = C3(n1) + C3(n2)
    want = pure * C3(m) + (C3(n) - pure) * (C3(m1) + C3(m2))
    if n1 == 3 and n2 == 4 and m1 == 4 and m2 == 3:
        assert want == 325
    assert oracle.count_bruteforce(g) == want
    assert oracle.count_bbvp(g, 0)["total"] == want
    assert oracle.count_bbvp(g, 1)["total"] == want


def test_disjoint_planted_blocks_additive(oracle):
    """Disjoint complete blocks with rank-1 signs on an empty graph:
    sum of C(k,3) C(k',3) (6x6: 400, 12x12: 48400, 5x5: 100)."""
    rng = np.random.default_rng(7)
    sizes = [(6, 6), (12, 12), (5, 5), (3, 4)]
    n_u = sum(a for a, _ in sizes) + 5
    n_v = sum(b for _, b in sizes) + 3
    u, v, s, _ = G.plant_blocks(rng, n_u, n_v, np.zeros(0, np.int64), np.zeros(0, np.int64),
                                np.zeros(0, np.int8), [(a, b, "balanced") for a, b in sizes])
    g = G._finish(n_u, n_v, u, v, s)
    want = sum(C3(a) * C3(b) for a, b in sizes)
    assert [C3(6) * C3(6), C3(12) * C3(12), C3(5) * C3(5)] == [400, 48400, 100]
    assert oracle.count_bbvp(g, 0)["total"] == want
    assert oracle.count_bbvp(g, 1)["total"] == want


def test_choose3_exact(oracle):
    for n in list(range(0, 40)) + [2642245, 2642246, 10**6]:
        assert oracle.choose3(n) == C3(n)


# ----------------------------------------- brute force on random tiny graphs
def test_bruteforce_equals_bbvp_tiny(oracle):
    """O1 (definition) = O2 (Algorithm 2 on U) = O3 (on V), totals and every
    per-vertex count, on random tiny graphs of all densities and sign mixes."""
    rng = np.random.default_rng(2026)
    nonzero = 0
    for it in range(3000):
        g = G.tiny_random(rng, 8, 8)
        b, pu, pv = oracle.count_bruteforce(g, per_vertex=True)
        r0 = oracle.count_bbvp(g, 0, per_vertex=True)
        r1 = oracle.count_bbvp(g, 1, per_vertex=True)
        assert r0["total"] == b and r1["total"] == b, it
        assert (r0["per_vertex"] == pu).all() and (r1["per_vertex"] == pv).all(), it
        assert int(pu.sum()) == 3 * b and int(pv.sum()) == 3 * b
        nonzero += b > 0
    assert nonzero > 300


def test_bruteforce_equals_bbvp_denser(oracle):
    rng = np.random.default_rng(99)
    for it in range(60):
        g = G.tiny_random(rng, 11, 11, density=float(rng.choice([0.7, 0.85, 1.0])))
        b = oracle.count_bruteforce(g)
        assert oracle.count_bbvp(g, 0)["total"] == b
        assert oracle.count_bbvp(g, 1)["total"] == b


def test_watch_list_counts_the_opposite_side(oracle):
    """Opposite-side watch lists of the anchored run: on random tiny graphs each
    watched V vertex gets the definition's per-vertex count (brute force),
    from U anchors; the anchors' neighbours alone, and the shards summed, give
    the same values; on K_{n,m} every V vertex lies in C(m - 1, 2) C(n, 3)
    bicliques."""
    rng = np.random.default_rng(77)
    for it in range(400):
        g = G.tiny_random(rng, 8, 8)
        b, pu, pv = oracle.count_bruteforce(g, per_vertex=True)
        ids = list(range(g.n_v))
        r = oracle.count_bbvp_watch(g, 0, ids)
        assert r["total"] == b and r["watch"] == [int(x) for x in pv], it
    g = G.config1(3)
    ids = [int(x) for x in np.argsort(-np.bincount(g.ev, minlength=g.n_v), kind="stable")[:12]]
    whole = oracle.count_bbvp_watch(g, 0, ids, threads=4)
    assert whole["watch"] == oracle.vertex_counts(g, 1, ids)
    on = np.zeros(g.n_u, bool)
    on[np.unique(g.eu[np.isin(g.ev, ids)])] = True
    near = oracle.count_bbvp_watch(g, 0, ids, threads=4, anchor_on=on)
    assert near["watch"] == whole["watch"] and near["total"] < whole["total"]
    parts = [oracle.count_bbvp_watch(g, 0, ids, n_shards=5, shard=r, threads=2) for r in range(5)]
    assert [sum(p["watch"][i] for p in parts) for i in range(len(ids))] == whole["watch"]
    n, m = 9, 7
    u, v = np.divmod(np.arange(n * m, dtype=np.int64), m)
    kg = G._finish(n, m, u, v, np.ones(n * m, np.int8))
    assert oracle.count_bbvp_watch(kg, 0, list(range(m)))["watch"] == [math.comb(m - 1, 2) * C3(n)] * m
    with pytest.raises(ValueError):
        oracle.count_bbvp_watch(kg, 0, [0, 0])


def test_vertex_counts_match_per_vertex(oracle):
    g = G.config1(3)
    for side in (0, 1):
        r = oracle.count_bbvp(g, side, per_vertex=True)
        n = g.n_u if side == 0 else g.n_v
        xs = list(range(0, n, 7))
        assert oracle.vertex_counts(g, side, xs) == [int(r["per_vertex"][x]) for x in xs]
        assert int(r["per_vertex"].sum()) == 3 * r["total"]


# --------------------------------------------------------------- invariants
def _switch(g, rng):
    fu = rng.choice([-1, 1], g.n_u).astype(np.int8)
    fv = rng.choice([-1, 1], g.n_v).astype(np.int8)
    return G._finish(g.n_u, g.n_v, g.eu, g.ev, (g.sign * fu[g.eu] * fv[g.ev]).astype(np.int8))


def _relabel(g, rng):
    pu = rng.permutation(g.n_u); pv = rng.permutation(g.n_v)
    order = rng.permutation(g.m)
    return G._finish(g.n_u, g.n_v, pu[g.eu][order], pv[g.ev][order], g.sign[order]), pu, pv


@pytest.mark.parametrize("maker", ["config1", "config2_small"])
def test_invariants(oracle, maker):
    g = G.config1(1) if maker == "config1" else G.config2(1, scale=0.02)
    rng = np.random.default_rng(5)
    base = oracle.count_bbvp(g, 0, threads=4, per_vertex=True)
    B = base["total"]
    assert B > 0
    # U <-> V transpose
    assert oracle.count_bbvp(g, 1, threads=4)["total"] == B
    assert oracle.count_bbvp(g.transpose(), 0, threads=4)["total"] == B
    # vertex switching (any set of vertices) and global negation
    sw = _switch(g, rng)
    r = oracle.count_bbvp(sw, 0, threads=4, per_vertex=True)
    assert r["total"] == B and (r["per_vertex"] == base["per_vertex"]).all()
    neg = G._finish(g.n_u, g.n_v, g.eu, g.ev, (-g.sign).astype(np.int8))
    assert oracle.count_bbvp(neg, 0, threads=4)["total"] == B
    # relabelling vertices and reordering the edge list
    rl, pu, pv = _relabel(g, rng)
    r = oracle.count_bbvp(rl, 0, threads=4, per_vertex=True)
    assert r["total"] == B
    assert (r["per_vertex"][pu] == base["per_vertex"]).all()
    # inserting an edge never lowers the count
    present = set(zip(g.eu.tolist(), g.ev.tolist()))
    for _ in range(3):
        while True:
            a, b = int(rng.integers(g.n_u)), int(rng.integers(g.n_v))
            if (a, b) not in present:
                break
        g2 = G._finish(g.n_u, g.n_v, np.append(g.eu, a), np.append(g.ev, b),
                       np.append(g.sign, np.int8(rng.choice([-1, 1]))))
        assert oracle.count_bbvp(g2, 0, threads=4)["total"] >= B
    # the planted balanced blocks alone give a lower bound
    if maker == "config1":
        assert B >= 3 * C3(6) * C3(6)


def test_config3_switching_reduction(oracle):
    """Signs l(u) l(v) flip are a switching of the flip signs alone."""
    g = G.config3(1, scale=0.0005)
    lu, lv = g.meta["label_u"], g.meta["label_v"]
    unsw = G._finish(g.n_u, g.n_v, g.eu, g.ev, (g.sign * lu[g.eu] * lv[g.ev]).astype(np.int8))
    assert oracle.count_bbvp(g, 0, threads=4)["total"] == oracle.count_bbvp(unsw, 0, threads=4)["total"]


def test_anchor_shards_partition_the_count(oracle):
    """Algorithm 2 sums per-anchor contributions, so running it over the
    anchors of each residue class (id modulo k) and adding the parts gives the
    whole count, feasible and candidate tallies and per-vertex arrays: the
    basis of the sharded runs that store the large-graph golden values."""
    for g in (G.config1(2), G.config2(1, scale=0.02)):
        for side in (0, 1):
            whole = oracle.count_bbvp(g, side, threads=4, per_vertex=True)
            for k in (1, 3, 7):
                parts = [oracle.count_bbvp_shard(g, side, k, r, threads=4, per_vertex=True)
                         for r in range(k)]
                for key in ("total", "feasible", "candidates"):
                    assert sum(p[key] for p in parts) == whole[key]
                assert (sum(p["per_vertex"] for p in parts) == whole["per_vertex"]).all()
            # each shard keeps only its own anchors: a shard with no anchors is empty
            n = g.n_u if side == 0 else g.n_v
            empty = oracle.count_bbvp_shard(g, side, n + 5, n + 4, threads=2, per_vertex=True)
            assert empty["total"] == 0 and empty["candidates"] == 0
    with pytest.raises(ValueError):
        oracle.count_bbvp_shard(G.config1(1), 0, 4, 4)


def test_bad_edges_rejected(oracle):
    g = G.from_rows(["++", "+-"])
    dup = G._finish(2, 2, np.array([0, 0]), np.array([1, 1]), np.array([1, 1], np.int8))
    with pytest.raises(ValueError):
        oracle.count_bbvp(dup)
    oob = G._finish(2, 2, np.array([0, 2]), np.array([1, 1]), np.array([1, 1], np.int8))
    with pytest.raises(ValueError):
        oracle.count_bbvp(oob)
    assert oracle.count_bbvp(g)["total"] == 0
    empty = G._finish(0, 0, np.zeros(0), np.zeros(0), np.zeros(0, np.int8))
    assert oracle.count_bbvp(empty)["total"] == 0


# ------------------------------------------ general q (p = 3 on one side)
# Section 3 defines balanced (p, q)-bicliques for any p, q; Algorithm 2 takes
# (p - 1)-subsets of the candidate set and sums C(x, q). The oracle's _q
# variant keeps p = 3 on the anchor side; anchored on V it counts (q, 3).

@pytest.mark.parametrize("n,m", [(5, 8), (7, 7), (8, 6)])
def test_general_q_complete_all_positive(oracle, n, m):
    """All-positive K_{n,m}: every (p,q) vertex choice is a balanced
    biclique, C(n,p) C(m,q)."""
    g = complete(n, m, lambda i, j: 1)
    for p, q in [(3, 4), (3, 5), (4, 3), (3, 7), (5, 3), (4, 4), (2, 6)]:
        assert oracle.count_bruteforce_pq(g, p, q) == math.comb(n, p) * math.comb(m, q), (p, q)
    for q in range(3, 8):
        assert oracle.count_bbvp_q(g, q, 0)["total"] == C3(n) * math.comb(m, q), q
        assert oracle.count_bbvp_q(g, q, 1)["total"] == math.comb(n, q) * C3(m), q


@pytest.mark.parametrize("n1,n2,m1,m2", [(3, 4, 4, 3), (2, 5, 5, 4), (4, 4, 6, 2), (1, 6, 7, 1)])
def test_general_q_two_block_closed_form(oracle, n1, n2, m1, m2):
    """The two-block sign pattern (sign -1 exactly on U2 x V2) for (3, q): a
    triple inside U1 or U2 has equal rows, any q columns; a mixed triple needs
    its q columns all in V1 or all in V2. For (p, 3) the same holds with the
    sides exchanged (the pattern is its own transpose up to relabelling)."""
    n, m = n1 + n2, m1 + m2
    g = complete(n, m, lambda i, j: -1 if (i >= n1 and j >= m1) else 1)
    pure = C3(n1) + C3(n2)
    pure_t = C3(m1) + C3(m2)
    for q in range(3, 8):
        want = pure * math.comb(m, q) + (C3(n) - pure) * (math.comb(m1, q) + math.comb(m2, q))
        assert oracle.count_bbvp_q(g, q, 0)["total"] == want, q
        assert oracle.count_bruteforce_pq(g, 3, q) == want, q
        want_t = pure_t * math.comb(n, q) + (C3(m) - pure_t) * (math.comb(n1, q) + math.comb(n2, q))
        assert oracle.count_bbvp_q(g, q, 1)["total"] == want_t, q
        assert oracle.count_bruteforce_pq(g, q, 3) == want_t, q


def test_general_q_bruteforce_equals_bbvp_tiny(oracle):
    """O1 for (3, q) and (q, 3) = Algorithm 2 with that q on U and on V, on
    random tiny graphs (dense enough that q >= 4 common neighbours occur)."""
    rng = np.random.default_rng(515)
    nonzero = {q: 0 for q in (4, 5)}
    for it in range(400):
        g = G.tiny_random(rng, 9, 9, density=float(rng.choice([0.6, 0.8, 1.0])))
        for q in (4, 5):
            b = oracle.count_bruteforce_pq(g, 3, q)
            assert oracle.count_bbvp_q(g, q, 0)["total"] == b, (it, q)
            assert oracle.count_bbvp_q(g, q, 1)["total"] == oracle.count_bruteforce_pq(g, q, 3), (it, q)
            nonzero[q] += b > 0
    assert min(nonzero.values()) > 40


def test_general_q_three_is_the_default(oracle):
    g = G.config1(2)
    for side in (0, 1):
        assert oracle.count_bbvp_q(g, 3, side)["total"] == oracle.count_bbvp(g, side)["total"]
    rng = np.random.default_rng(3)
    for it in range(50):
        t = G.tiny_random(rng, 8, 8, density=0.9)
        assert oracle.count_bruteforce_pq(t, 3, 3) == oracle.count_bruteforce(t), it


# ------------------------------------------------------- edges (dynamic graphs)
def test_through_edge_closed_forms(oracle):
    """All-positive K_{n,m}: every edge lies in C(n-1, 2) C(m-1, 2) balanced
    (3,3)-bicliques; with its sign flipped, in none (each butterfly through it
    then has one negative edge); a missing edge inserted with + closes the
    complete graph again."""
    for n, m in [(3, 3), (4, 5), (6, 4)]:
        g = G.from_rows(["+" * m] * n)
        want = math.comb(n - 1, 2) * math.comb(m - 1, 2)
        assert oracle.count_through_edge(g, 1, 2, 1, brute=True) == want
        assert oracle.count_through_edge(g, 1, 2, -1, brute=True) == 0
        rows = ["+" * m] * n
        rows[0] = "." + "+" * (m - 1)
        assert oracle.count_through_edge(G.from_rows(rows), 0, 0, 1, brute=True) == want


def test_through_edge_sums_to_nine_times_count(oracle):
    """Every balanced (3,3)-biclique has 9 edges, so the queries of all edges
    with their own signs sum to 9 B (brute force on tiny random graphs)."""
    rng = np.random.default_rng(41)
    for _ in range(25):
        n_u, n_v = int(rng.integers(3, 8)), int(rng.integers(3, 8))
        dense = rng.random((n_u, n_v)) < rng.uniform(0.5, 1.0)
        u, v = np.nonzero(dense)
        s = np.where(rng.random(u.size) < rng.uniform(0.3, 1.0), 1, -1).astype(np.int8)
        g = G._finish(n_u, n_v, u, v, s)
        tot = sum(oracle.count_through_edge(g, int(a), int(b), int(c), brute=True) for a, b, c in zip(u, v, s))
        assert tot == 9 * oracle.count_bruteforce(g)


# ------------------------------------------------- p = 4 on the anchor side
def test_p4_closed_forms(oracle):
    """All-positive K_{n,m}: C(n,4) C(m,q); the two-block sign pattern (sign -1
    exactly on U2 x V2): [C(n1,4) + C(n2,4)] C(m,q) + [C(n,4) - C(n1,4) -
    C(n2,4)] [C(m1,q) + C(m2,q)]; and the transposes on the other side."""
    C = math.comb
    for n, m, q in [(5, 6, 3), (6, 7, 4), (7, 5, 5), (4, 8, 7)]:
        g = G.from_rows(["+" * m] * n)
        assert oracle.count_bbvp_p4(g, q, 0)["total"] == C(n, 4) * C(m, q)
        gt = G.from_rows(["+" * n] * m)
        assert oracle.count_bbvp_p4(gt, q, 1)["total"] == C(n, 4) * C(m, q)
    for (n1, n2, m1, m2, q) in [(3, 4, 4, 3, 3), (4, 5, 5, 3, 4), (2, 6, 3, 6, 5)]:
        n, m = n1 + n2, m1 + m2
        rows = ["".join("-" if (i >= n1 and j >= m1) else "+" for j in range(m)) for i in range(n)]
        pure = C(n1, 4) + C(n2, 4)
        want = pure * C(m, q) + (C(n, 4) - pure) * (C(m1, q) + C(m2, q))
        assert oracle.count_bbvp_p4(G.from_rows(rows), q, 0)["total"] == want


def test_p4_equals_definition_tiny(oracle):
    """Algorithm 2 with p = 4 equals the definition (brute force over all
    (4, q) and (q, 4) pairs of vertex sets) on dense tiny random graphs."""
    rng = np.random.default_rng(77)
    nonzero = 0
    for _ in range(120):
        n_u, n_v = int(rng.integers(4, 9)), int(rng.integers(4, 9))
        dense = rng.random((n_u, n_v)) < rng.uniform(0.5, 1.0)
        u, v = np.nonzero(dense)
        s = np.where(rng.random(u.size) < rng.uniform(0.3, 1.0), 1, -1).astype(np.int8)
        g = G._finish(n_u, n_v, u, v, s)
        for q in (3, 4, 5):
            want = oracle.count_bruteforce_pq(g, 4, q)
            assert oracle.count_bbvp_p4(g, q, 0)["total"] == want
            assert oracle.count_bbvp_p4(g, q, 1)["total"] == oracle.count_bruteforce_pq(g, q, 4)
            nonzero += want > 0
    assert nonzero > 40


# ------------------------------------------------- p = 5 on the anchor side
def test_p5_closed_forms_and_definition(oracle):
    """Algorithm 2 with p = 5 (4-subsets of the candidate set, 16 classes):
    C(n,5) C(m,q) on all-positive K_{n,m}, the two-block closed form, the
    definition on dense tiny graphs (both sides), and the dense form with
    p = 4 equals the merge form."""
    C = math.comb
    for n, m, q in [(6, 6, 3), (7, 8, 4), (8, 5, 5)]:
        g = G.from_rows(["+" * m] * n)
        assert oracle.count_bbvp_pk(g, 5, q, 0)["total"] == C(n, 5) * C(m, q)
    for (n1, n2, m1, m2, q) in [(4, 5, 4, 3, 3), (5, 3, 5, 4, 4)]:
        n, m = n1 + n2, m1 + m2
        rows = ["".join("-" if (i >= n1 and j >= m1) else "+" for j in range(m)) for i in range(n)]
        pure = C(n1, 5) + C(n2, 5)
        want = pure * C(m, q) + (C(n, 5) - pure) * (C(m1, q) + C(m2, q))
        assert oracle.count_bbvp_pk(G.from_rows(rows), 5, q, 0)["total"] == want
    rng = np.random.default_rng(55)
    nonzero = 0
    for _ in range(80):
        n_u, n_v = int(rng.integers(5, 9)), int(rng.integers(5, 9))
        dense = rng.random((n_u, n_v)) < rng.uniform(0.6, 1.0)
        u, v = np.nonzero(dense)
        s = np.where(rng.random(u.size) < rng.uniform(0.3, 1.0), 1, -1).astype(np.int8)
        g = G._finish(n_u, n_v, u, v, s)
        for q in (3, 4):
            want = oracle.count_bruteforce_pq(g, 5, q)
            assert oracle.count_bbvp_pk(g, 5, q, 0)["total"] == want
            assert oracle.count_bbvp_pk(g, 5, q, 1)["total"] == oracle.count_bruteforce_pq(g, q, 5)
            assert oracle.count_bbvp_pk(g, 4, q, 0, dense=True)["total"] == oracle.count_bbvp_p4(g, q, 0)["total"]
            nonzero += want > 0
    assert nonzero > 20
