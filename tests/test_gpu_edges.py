"""GPU parity of the edge queries (bbc_count_through_edges) against the
oracle: balanced (3,3)-bicliques through an edge, i.e. the change of the
count when the edge is inserted, deleted or re-signed. Exact (tolerance 0).
"""
import math

import numpy as np
import pytest

from paper_2605_03603_amd import generators as G
from tests.gpu_common import build, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_2605_03603_amd import bbc
    c = bbc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def B():
    from paper_2605_03603_amd import bbc
    return bbc


def _queries(g, rng, n):
    """Existing edges with their sign and flipped, missing pairs with both
    signs, and pairs at an isolated vertex when there is one."""
    have = set(zip(g.eu.tolist(), g.ev.tolist()))
    qs = []
    idx = rng.choice(g.eu.size, size=min(n, g.eu.size), replace=False)
    for i in idx:
        s = int(g.sign[i])
        qs.append((int(g.eu[i]), int(g.ev[i]), s))
        qs.append((int(g.eu[i]), int(g.ev[i]), -s))
    for _ in range(50 * n):             # a dense graph may have few missing pairs
        if len(qs) >= 4 * n:
            break
        u, v = int(rng.integers(0, g.n_u)), int(rng.integers(0, g.n_v))
        if (u, v) not in have:
            qs.append((u, v, 1))
            qs.append((u, v, -1))
    deg_u = np.bincount(g.eu.astype(np.int64), minlength=g.n_u)
    iso = np.flatnonzero(deg_u == 0)
    if iso.size:
        qs.append((int(iso[0]), 0, 1))
    return qs


def test_edges_complete_closed_form(ctx):
    """All-positive K_{n,m}: C(n-1, 2) C(m-1, 2) through each edge, 0 with its
    sign flipped; the same with the graph anchored on either side."""
    for n, m in [(3, 3), (6, 9), (40, 7)]:
        say("edges complete", n, m)
        g = G.from_rows(["+" * m] * n)
        want = math.comb(n - 1, 2) * math.comb(m - 1, 2)
        for flags in (1 << 4, 1 << 5):
            h = build(ctx, g, flags)
            got = ctx.count_through_edges(h, [0, n - 1, 1], [0, m - 1, 2], [1, 1, -1])
            assert got.tolist() == [want, want, 0]


def test_edges_vs_oracle_config1(ctx, oracle):
    for seed in (1, 2):
        g = G.config1(seed)
        rng = np.random.default_rng([11, seed])
        qs = _queries(g, rng, 12)
        say("edges config1", seed, len(qs))
        want = [oracle.count_through_edge(g, u, v, s, threads=8) for u, v, s in qs]
        for flags in (1 << 4, 1 << 5):
            h = build(ctx, g, flags)
            got = ctx.count_through_edges(h, *zip(*qs))
            assert got.tolist() == want, (seed, flags)


def test_edges_tiny_vs_bruteforce(ctx, oracle):
    rng = np.random.default_rng(12)
    for t in range(60):
        n_u, n_v = int(rng.integers(3, 9)), int(rng.integers(3, 9))
        dense = rng.random((n_u, n_v)) < rng.uniform(0.4, 1.0)
        u, v = np.nonzero(dense)
        if u.size == 0:
            continue
        s = np.where(rng.random(u.size) < rng.uniform(0.2, 1.0), 1, -1).astype(np.int8)
        g = G._finish(n_u, n_v, u, v, s)
        qs = _queries(g, rng, 3)
        want = [oracle.count_through_edge(g, a, b, c, brute=True) for a, b, c in qs]
        got = ctx.count_through_edges(build(ctx, g), *zip(*qs))
        assert got.tolist() == want, t


def test_edges_sum_to_nine_times_count(ctx, oracle):
    """Every edge with its own sign: the queries sum to 9 B (config 1, all
    edges)."""
    g = G.config1(3)
    say("edges 9B", g.m)
    total = oracle.count_bbvp(g, 0, threads=8)["total"]
    h = build(ctx, g)
    got = ctx.count_through_edges(h, g.eu, g.ev, g.sign)
    assert int(got.sum()) == 9 * total
    assert ctx.count_global(h) == total


def test_edges_errors(ctx, B):
    g = G.from_rows(["+++", "+++", "+++"])
    h = build(ctx, g)
    with pytest.raises(B.BBCError) as e:
        ctx.count_through_edges(h, [3], [0], [1])
    assert e.value.name == "BBC_E_RANGE"
    with pytest.raises(B.BBCError) as e:
        ctx.count_through_edges(h, [0], [0], [0])
    assert e.value.name == "BBC_E_SIGN"
    assert ctx.count_through_edges(h, [], [], []).tolist() == []


def test_edges_config2_all_edges(ctx):
    """Config 2 at full size: the queries of all 2,057,578 edges with their own
    signs sum to 9 B, B from tests/golden/cfg2_seed1.json (the oracle's count)."""
    from tests.gpu_common import golden
    want = golden("cfg2_seed1.json")["total"]
    g = G.config2(1)
    h = build(ctx, g, 1 << 4)
    say("edges config2 all", g.m)
    got = ctx.count_through_edges(h, g.eu, g.ev, g.sign)
    assert int(got.sum()) == 9 * want
    assert (got >= 0).all()
