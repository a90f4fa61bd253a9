"""GPU parity of the rank-window pair tier.

Heavy anchors (at least 16384 wedges) whose partners all rank within 2^17
above them are counted with a table indexed by partner rank instead of a hash
table. Each case is checked against a closed form or the CPU oracle, and
against the same graph counted with the rank-window tier switched off (the
hash tiers alone), with tolerance 0.
"""
import math

import numpy as np
import pytest

from paper_2605_03603_amd import generators as G
from tests.gpu_common import build, need_gpu, say

pytestmark = pytest.mark.gpu

ANCHOR_U, ANCHOR_V = 1 << 4, 1 << 5


@pytest.fixture(scope="module")
def B():
    need_gpu()
    from paper_2605_03603_amd import bbc
    return bbc


@pytest.fixture(scope="module")
def ctx(B):
    c = B.Context(0)
    yield c
    c.close()


def C3(n):
    return math.comb(n, 3)


def complete_signed(n, m, n1, m1):
    """K_{n,m} with sign -1 exactly on rows >= n1 x columns >= m1."""
    u, v = np.divmod(np.arange(n * m, dtype=np.int64), m)
    s = np.where((u >= n1) & (v >= m1), -1, 1).astype(np.int8)
    return G._finish(n, m, u, v, s)


def two_block_total(n, n1, m, m1):
    """Balanced (3,3)-bicliques of complete_signed(n, m, n1, m1): a triple
    inside one row block sees all columns in one class, a mixed triple sees
    the two column blocks as two classes."""
    pure = C3(n1) + C3(n - n1)
    return pure * C3(m) + (C3(n) - pure) * (C3(m1) + C3(m - m1))


def dense(seed, n_u=700, n_v=400, p=0.5, p_pos=0.8):
    rng = np.random.default_rng(seed)
    u, v = np.nonzero(rng.random((n_u, n_v)) < p)
    s = np.where(rng.random(u.size) < p_pos, 1, -1).astype(np.int8)
    return G._finish(n_u, n_v, u, v, s)


def count_both_routes(ctx, B, h):
    """Count with the rank-window tier and without it; return both counts and
    the number of anchors the first count handed to the tier."""
    got = ctx.count_global(h)
    n_window = ctx.last_stats()["deferred_r"]
    ctx.set_test_hook(B.BBC_HOOK_NO_WINDOW_TIER, 1)
    try:
        hashed = ctx.count_global(h)
        assert ctx.last_stats()["deferred_r"] == 0
    finally:
        ctx.set_test_hook(B.BBC_HOOK_NO_WINDOW_TIER, 0)
    return got, hashed, n_window


@pytest.mark.parametrize("n,n1,m,m1", [
    (3000, 3000, 300, 300),   # all positive: one class, up to 2999 candidates
    (3000, 1500, 300, 150),   # two blocks: up to 4499 candidates, masks staged in slabs
    (2200, 900, 70, 35),      # 3-word masks
])
def test_window_tier_closed_forms(ctx, B, n, n1, m, m1):
    say("window tier closed form", n, n1, m, m1)
    h = build(ctx, complete_signed(n, m, n1, m1), ANCHOR_U)
    got, hashed, n_window = count_both_routes(ctx, B, h)
    want = two_block_total(n, n1, m, m1)
    assert got == want and hashed == want
    assert n_window > 0
    h.free()


def test_window_tier_per_vertex_closed_form(ctx):
    """Per-vertex counts of both sides through rank-window anchors (their
    candidates are numbered by class and rank): a U vertex of row block b lies
    in C(n_b - 1, 2) pure triples and C(n - 1, 2) - C(n_b - 1, 2) mixed ones;
    a V vertex of column block c in C(m - 1, 2) R-sets of each pure triple and
    C(m_c - 1, 2) of each mixed one."""
    C = math.comb
    n, n1, m, m1 = 3000, 1500, 300, 150
    say("window tier per vertex")
    h = build(ctx, complete_signed(n, m, n1, m1), ANCHOR_U)
    pure_l = C3(n1) + C3(n - n1)
    mixed_l = C3(n) - pure_l
    total = two_block_total(n, n1, m, m1)
    pu, tu = ctx.count_per_vertex(h, 0)
    assert tu == total
    assert ctx.last_stats()["deferred_r"] > 0
    nb = np.where(np.arange(n) < n1, n1, n - n1)
    want_u = [C(int(b) - 1, 2) * C3(m) + (C(n - 1, 2) - C(int(b) - 1, 2)) * (C3(m1) + C3(m - m1))
              for b in nb]
    assert [int(x) for x in pu] == want_u
    pv, tv = ctx.count_per_vertex(h, 1)
    assert tv == total
    want_v = [pure_l * C(m - 1, 2) + mixed_l * C((m1 if v < m1 else m - m1) - 1, 2) for v in range(m)]
    assert [int(x) for x in pv] == want_v
    h.free()


def test_window_tier_vs_oracle(ctx, B, oracle):
    """A dense random signed graph (700 x 400, edge probability 0.5, 80%
    positive): about three quarters of the U anchors reach 16384 wedges. Totals on both
    anchor sides and per-vertex counts of both sides against the oracle."""
    g = dense(1)
    say("window tier vs oracle: oracle")
    ru = oracle.count_bbvp(g, 0, threads=8, per_vertex=True)
    rv = oracle.count_bbvp(g, 1, threads=8, per_vertex=True)
    assert ru["total"] == rv["total"]
    say("window tier vs oracle: gpu")
    hu = build(ctx, g, ANCHOR_U)
    got, hashed, n_window = count_both_routes(ctx, B, hu)
    assert got == hashed == ru["total"]
    assert n_window > 0
    pu, tu = ctx.count_per_vertex(hu, 0)
    assert tu == ru["total"] and (pu == ru["per_vertex"]).all()
    pv, tv = ctx.count_per_vertex(hu, 1)
    assert tv == ru["total"] and (pv == rv["per_vertex"]).all()
    hu.free()
    hv = build(ctx, g, ANCHOR_V)
    assert ctx.count_global(hv) == ru["total"]
    hv.free()


def test_window_tier_batch(ctx, oracle):
    """Graphs of one batch each index their own rank window (partners rank
    inside the anchor's graph): a batch of heavy and light graphs against the
    per-graph values, twice (the second a replay of the captured launch)."""
    gs = [dense(2), complete_signed(2200, 70, 900, 35), G.config1(3), dense(3, n_u=500)]
    want = [oracle.count_bbvp(gs[0], 0, threads=8)["total"], two_block_total(2200, 900, 70, 35),
            oracle.count_bbvp(gs[2], 0, threads=8)["total"],
            oracle.count_bbvp(gs[3], 0, threads=8)["total"]]
    say("window tier batch")
    nu, nv, off, eu, ev, sg = G.concat(gs)
    hs = ctx.build_csr_batch(nu, nv, off, eu, ev, sg, ANCHOR_U)
    assert list(ctx.count_batch(hs)) == want
    assert list(ctx.count_batch(hs)) == want
    assert ctx.last_stats()["deferred_r"] > 0
    for h in hs:
        h.free()
