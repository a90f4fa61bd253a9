"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Counts are integers, so every comparison is exact (tolerance 0).
"""
import hashlib
import math

import numpy as np
import pytest

from paper_2605_03603_amd import generators as G
from tests.gpu_common import build, golden, need_gpu, say

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


def C3(n):
    return math.comb(n, 3)


# ------------------------------------------------------------ paper pins
def test_fig1b_and_fig4(ctx, oracle):
    say("fig1b")
    g = G.from_rows(["++++", "++++", "-+++", "--++"])
    h = build(ctx, g)
    assert ctx.count_global(h) == 1
    pu, tot = ctx.count_per_vertex(h, 0)
    assert tot == 1 and list(pu) == [1, 1, 1, 0]
    pv, _ = ctx.count_per_vertex(h, 1)
    assert list(pv) == [0, 1, 1, 1]
    say("fig4")
    g4 = G.from_rows(["++++", "+++.", "++.+", "+.++"])
    assert ctx.count_global(build(ctx, g4)) == 0


@pytest.mark.parametrize("n,m", [(3, 3), (5, 7), (40, 3), (70, 70), (130, 20)])
def test_complete_bipartite(ctx, n, m):
    say("complete", n, m)
    rows = ["+" * m] * n
    g = G.from_rows(rows)
    assert ctx.count_global(build(ctx, g)) == C3(n) * C3(m)
    for side in (0, 1):
        pv, tot = ctx.count_per_vertex(build(ctx, g), side)
        k, other = (n, m) if side == 0 else (m, n)
        assert tot == C3(n) * C3(m)
        assert (pv == math.comb(k - 1, 2) * C3(other)).all()


def test_two_block_closed_form(ctx):
    say("two-block")
    for (n1, n2, m1, m2) in [(3, 4, 4, 3), (10, 20, 15, 5), (33, 31, 40, 2)]:
        n, m = n1 + n2, m1 + m2
        rows = ["".join("-" if (i >= n1 and j >= m1) else "+" for j in range(m)) for i in range(n)]
        g = G.from_rows(rows)
        pure = C3(n1) + C3(n2)
        want = pure * C3(m) + (C3(n) - pure) * (C3(m1) + C3(m2))
        for flags in (0, 1 << 4, 1 << 5):
            assert ctx.count_global(build(ctx, g, flags)) == want


def _complete_signed(n, m, n1, m1):
    """K_{n,m} with sign -1 exactly on rows >= n1 x columns >= m1, as COO."""
    u, v = np.divmod(np.arange(n * m, dtype=np.int64), m)
    s = np.where((u >= n1) & (v >= m1), -1, 1).astype(np.int8)
    return G._finish(n, m, u, v, s)


@pytest.mark.parametrize("w", [1, 2, 3, 4, 5, 8, 9, 16, 17, 32, 33, 64])
def test_full_masks_every_width(ctx, w):
    """Anchored on U, every mask of K_{67, 32 w} has all 32 w bits set, so
    each candidate pair has the largest intersection its width allows (the
    top of each width class of the triplet kernels); 67 rows leave a ragged
    second row block. The two-block sign pattern splits each anchor's
    candidates into two classes of different sizes."""
    n, m = 67, 32 * w
    say("full masks", w)
    g = _complete_signed(n, m, n, m)
    assert ctx.count_global(build(ctx, g, 1 << 4)) == C3(n) * C3(m)
    n1, m1 = 40, m - m // 3
    n2, m2 = n - n1, m - m1
    g = _complete_signed(n, m, n1, m1)
    pure = C3(n1) + C3(n2)
    want = pure * C3(m) + (C3(n) - pure) * (C3(m1) + C3(m2))
    assert ctx.count_global(build(ctx, g, 1 << 4)) == want


def _width_mix(w, seed):
    """Random masks of exactly w words: 40 U vertices of degree 32 w - 3 over
    V[0, 48 w), and 150 of degree 32 w - 1 that take a random share of their
    neighbours there (0 to all of them) and the rest from V[48 w, 96 w), so
    that candidate pairs meet in anywhere from 0 to most of their bits."""
    rng = np.random.default_rng(seed)
    d_a, d_c, half = 32 * w - 3, 32 * w - 1, 48 * w
    eu, ev = [], []
    for u in range(40):
        eu.append(np.full(d_a, u)); ev.append(rng.choice(half, d_a, replace=False))
    for u in range(40, 190):
        k = int(rng.integers(0, d_c + 1))
        eu.append(np.full(d_c, u))
        ev.append(np.concatenate([rng.choice(half, k, replace=False),
                                  half + rng.choice(half, d_c - k, replace=False)]))
    u = np.concatenate(eu); v = np.concatenate(ev)
    s = np.where(rng.random(u.size) < 0.8, 1, -1).astype(np.int8)
    return G._finish(190, 2 * half, u, v, s)


@pytest.mark.parametrize("w", list(range(1, 21)))
def test_every_width_random_vs_oracle(ctx, oracle, w):
    """Every mask width of the triplet kernels up to 20 words (the int8 and
    fp4 forms, word-by-word and whole loads, the 16-bit epilogue and its
    wider fallback, the wide path): totals and per-vertex counts of both
    sides against the oracle. Anchors have 189 candidates in two classes, so
    row blocks and column tiles are ragged."""
    g = _width_mix(w, 100 + w)
    say("every width", w)
    ru = oracle.count_bbvp(g, 0, threads=8, per_vertex=True)
    rv = oracle.count_bbvp(g, 1, threads=8, per_vertex=True)
    assert ru["total"] == rv["total"] > 0
    h = build(ctx, g, 1 << 4)
    assert ctx.count_global(h) == ru["total"]
    pu, t = ctx.count_per_vertex(h, 0)
    assert t == ru["total"] and (pu == ru["per_vertex"]).all()
    pv, t = ctx.count_per_vertex(h, 1)
    assert t == ru["total"] and (pv == rv["per_vertex"]).all()
    h.free()


def test_launch_shapes_same_count(ctx, oracle, B):
    """The unit column base and the workgroups per compute unit change how
    the work is cut and spread, never the count: config 1 seed 2 and random
    masks of 6 and 13 words, totals and anchor-side per-vertex counts, under
    the extreme shapes, against the oracle. Invalid shapes are refused."""
    gs = [G.config1(2), _width_mix(6, 206), _width_mix(13, 213)]
    want = [oracle.count_bbvp(g, 0, threads=8, per_vertex=True) for g in gs]
    hs = [build(ctx, g, 1 << 4) for g in gs]
    try:
        for cb, gt, ga in [(256, 1, 1), (16384, 16, 8), (512, 3, 2), (4096, 9, 4)]:
            say("launch shape", cb, gt, ga)
            ctx.set_test_hook(B.BBC_HOOK_LAUNCH_SHAPE, B.launch_shape(cb, gt, ga))
            for h, r in zip(hs, want):
                assert ctx.count_global(h) == r["total"]
                pu, t = ctx.count_per_vertex(h, 0)
                assert t == r["total"] and (pu == r["per_vertex"]).all()
        for bad in [B.launch_shape(3000, 4), B.launch_shape(128, 4), B.launch_shape(32768, 4),
                    B.launch_shape(2048, 0), B.launch_shape(2048, 17), B.launch_shape(2048, 4, 9),
                    B.launch_shape(2048, 4) | (1 << 50)]:
            with pytest.raises(B.BBCError):
                ctx.set_test_hook(B.BBC_HOOK_LAUNCH_SHAPE, bad)
    finally:
        ctx.set_test_hook(B.BBC_HOOK_LAUNCH_SHAPE, 0)
    for h, r in zip(hs, want):
        assert ctx.count_global(h) == r["total"]
        h.free()


# --------------------------------------------------------- random tiny
def test_tiny_random_batch_vs_bruteforce(ctx, oracle):
    say("tiny batch")
    rng = np.random.default_rng(4242)
    gs = [G.tiny_random(rng, 9, 9) for _ in range(1500)]
    want = [oracle.count_bruteforce(g) for g in gs]
    nu, nv, off, eu, ev, sg = G.concat(gs)
    hs = ctx.build_csr_batch(nu, nv, off, eu, ev, sg)
    got = ctx.count_batch(hs)
    assert list(got) == want
    # the same graphs one at a time, forced to each side
    for i in range(0, 1500, 37):
        for flags in (1 << 4, 1 << 5):
            assert ctx.count_global(build(ctx, gs[i], flags)) == want[i], i


def test_tiny_per_vertex(ctx, oracle):
    say("tiny per-vertex")
    rng = np.random.default_rng(77)
    for it in range(120):
        g = G.tiny_random(rng, 8, 8, density=0.8)
        b, pu, pv = oracle.count_bruteforce(g, per_vertex=True)
        h = build(ctx, g, 1 << (4 + it % 2))
        gu, t = ctx.count_per_vertex(h, 0)
        gv, _ = ctx.count_per_vertex(h, 1)
        assert t == b and (gu == pu).all() and (gv == pv).all(), it


# -------------------------------------------------------- config sizes
@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_config1(ctx, oracle, seed):
    say("config1 seed", seed)
    g = G.config1(seed)
    r0 = oracle.count_bbvp(g, 0, per_vertex=True)
    r1 = oracle.count_bbvp(g, 1, per_vertex=True)
    for flags in (0, 1 << 4, 1 << 5, 1 << 6):
        h = build(ctx, g, flags)
        assert ctx.count_global(h) == r0["total"]
    h = build(ctx, g)
    pu, t = ctx.count_per_vertex(h, 0)
    pv, _ = ctx.count_per_vertex(h, 1)
    assert t == r0["total"]
    assert (pu == r0["per_vertex"]).all() and (pv == r1["per_vertex"]).all()


@pytest.mark.parametrize("scale", [0.02, 0.1])
def test_config2_scaled(ctx, oracle, scale):
    say("config2 scale", scale)
    g = G.config2(3, scale=scale)
    r = oracle.count_bbvp(g, 0, threads=8, per_vertex=True)
    for flags in (0, 1 << 4, 1 << 5):
        assert ctx.count_global(build(ctx, g, flags)) == r["total"]
    pu, t = ctx.count_per_vertex(build(ctx, g), 0)
    assert t == r["total"] and (pu == r["per_vertex"]).all()


def test_sign_encodings(ctx, B):
    say("sign encodings")
    g = G.config2(5, scale=0.02)
    want = ctx.count_global(build(ctx, g))
    packed = B.pack_signs_2bit(g.sign)
    h = ctx.build_csr(g.n_u, g.n_v, g.eu, g.ev, packed, B.BBC_SIGNS_2BIT_PACKED)
    assert ctx.count_global(h) == want
    s01 = (g.sign > 0).astype(np.int8)
    h = ctx.build_csr(g.n_u, g.n_v, g.eu, g.ev, s01, B.BBC_SIGNS_01)
    assert ctx.count_global(h) == want


def test_device_pointer_input(ctx):
    say("device pointers")
    import torch
    g = G.config1(2)
    want = ctx.count_global(build(ctx, g))
    d = torch.device("cuda:0")
    eu = torch.from_numpy(g.eu.astype(np.int32)).to(d)
    ev = torch.from_numpy(g.ev.astype(np.int32)).to(d)
    sg = torch.from_numpy(g.sign).to(d)
    torch.cuda.synchronize()
    h = ctx.build_csr(g.n_u, g.n_v, eu, ev, sg)
    assert ctx.count_global(h) == want


def _wide_sparse(seed):
    """Wide masks that meet in few bits: 40 U vertices of degree 700 over a
    random part of V[0, 3000) (22-word masks) and 200 of degree 800 that share
    about 40 neighbours with that part and take the rest from V[3000, 6000)."""
    rng = np.random.default_rng(seed)
    eu, ev = [], []
    for u in range(40):
        vs = rng.choice(3000, 700, replace=False)
        eu.append(np.full(700, u)); ev.append(vs)
    for u in range(40, 240):
        vs = np.concatenate([rng.choice(3000, 40, replace=False),
                             3000 + rng.choice(3000, 760, replace=False)])
        eu.append(np.full(800, u)); ev.append(vs)
    u = np.concatenate(eu); v = np.concatenate(ev)
    s = np.where(rng.random(u.size) < 0.8, 1, -1).astype(np.int8)
    return G._finish(240, 6000, u, v, s)


def test_wide_masks_small_and_large_intersections(ctx, oracle):
    """Masks over 16 words whose pairs meet in at most 256 bits take the
    packed 16-bit epilogue tile by tile, the others the 64-bit one: a graph of
    wide sparse masks against the oracle (total and per vertex), and all-ones
    masks of 19 and 38 words (every pair meets in 608 or 1216 bits) against
    the closed form, alone and in one batch."""
    g = _wide_sparse(3)
    say("wide sparse masks: oracle")
    r = oracle.count_bbvp(g, 0, threads=8, per_vertex=True)
    h = build(ctx, g, 1 << 4)
    assert ctx.count_global(h) == r["total"]
    pu, t = ctx.count_per_vertex(h, 0)
    assert t == r["total"] and (pu == r["per_vertex"]).all()
    h.free()
    full = [_complete_signed(70, 608, 70, 608), _complete_signed(40, 1216, 25, 1000)]
    want_full = [C3(70) * C3(608),
                 (C3(25) + C3(15)) * C3(1216) + (C3(40) - C3(25) - C3(15)) * (C3(1000) + C3(216))]
    for gf, w in zip(full, want_full):
        hf = build(ctx, gf, 1 << 4)
        assert ctx.count_global(hf) == w
        hf.free()
    gs = [g] + full
    nu, nv, off, eu, ev, sg = G.concat(gs)
    hs = ctx.build_csr_batch(nu, nv, off, eu, ev, sg, 1 << 4)
    assert list(ctx.count_batch(hs)) == [r["total"]] + want_full
    for hh in hs:
        hh.free()


def test_per_vertex_device_output(ctx, oracle):
    """Per-vertex counts written straight into a device tensor (both sides,
    so both the anchor side's rank-to-id remap and the other side's copy run
    on the GPU) equal the host-array results and the oracle's."""
    import torch
    d = torch.device("cuda:0")
    for g in (G.config1(2), G.config2(1, scale=0.02)):
        h = build(ctx, g, 1 << 4)
        for side in (0, 1):
            n = g.n_u if side == 0 else g.n_v
            say("per-vertex to device", g.m, side)
            want = oracle.count_bbvp(g, side, threads=8, per_vertex=True)
            host, t_host = ctx.count_per_vertex(h, side)
            out = torch.full((n,), -7, dtype=torch.int64, device=d)
            got, t_dev = ctx.count_per_vertex(h, side, out=out)
            torch.cuda.synchronize()
            assert t_dev == t_host == want["total"]
            assert (got.cpu().numpy() == host).all() and (host == want["per_vertex"]).all()
        h.free()


# ------------------------------------------------ edge and error cases
def test_degenerate_inputs(ctx):
    say("degenerate")
    e = np.zeros(0, np.uint32)
    s = np.zeros(0, np.int8)
    assert ctx.count_global(ctx.build_csr(0, 0, e, e, s)) == 0
    assert ctx.count_global(ctx.build_csr(5, 7, e, e, s)) == 0
    assert ctx.count_global(build(ctx, G.from_rows(["+++", "+++"]))) == 0
    one = ctx.build_csr(3, 3, np.array([1], np.uint32), np.array([2], np.uint32), np.array([-1], np.int8))
    assert ctx.count_global(one) == 0
    pv, t = ctx.count_per_vertex(ctx.build_csr(4, 0, e, e, s), 0)
    assert t == 0 and list(pv) == [0, 0, 0, 0]


def test_invalid_inputs(ctx, B):
    say("invalid inputs")
    u = np.array([0, 1, 1], np.uint32)
    v = np.array([0, 0, 0], np.uint32)
    s = np.array([1, 1, -1], np.int8)
    with pytest.raises(B.BBCError) as ei:
        ctx.build_csr(2, 2, u, v, s)
    assert ei.value.name == "BBC_E_DUP_EDGE"
    with pytest.raises(B.BBCError) as ei:
        ctx.build_csr(2, 2, np.array([0, 2], np.uint32), np.array([0, 1], np.uint32), np.array([1, 1], np.int8))
    assert ei.value.name == "BBC_E_RANGE"
    with pytest.raises(B.BBCError) as ei:
        ctx.build_csr(2, 2, np.array([0, 1], np.uint32), np.array([0, 1], np.uint32), np.array([1, 0], np.int8))
    assert ei.value.name == "BBC_E_SIGN"
    h = build(ctx, G.config1(1))
    with pytest.raises(B.BBCError) as ei:
        ctx.count_global(h, 6, 6)
    assert ei.value.name == "BBC_E_UNSUPPORTED"
    # the context is still usable after errors
    assert ctx.count_global(h) > 0


def test_heavy_anchors_all_tiers(ctx, oracle):
    """Anchors whose tables overflow the 4096-slot tier, masks wider than 16
    words, and degrees above 1024 (global-memory tier)."""
    say("heavy anchors")
    rng = np.random.default_rng(8)
    # a dense core: 40 U vertices adjacent to ~1100 V vertices each
    n_u, n_v = 60, 1300
    dense = rng.random((n_u, n_v)) < np.where(np.arange(n_u)[:, None] < 40, 0.9, 0.05)
    u, v = np.nonzero(dense)
    s = np.where(rng.random(u.size) < 0.8, 1, -1).astype(np.int8)
    g = G._finish(n_u, n_v, u, v, s)
    r = oracle.count_bbvp(g, 0, threads=8)
    assert ctx.count_global(build(ctx, g, 1 << 4)) == r["total"]
    # V-anchored: many distinct 2-hop partners per anchor (hash overflow tiers)
    assert ctx.count_global(build(ctx, g, 1 << 5)) == r["total"]
    pu, t = ctx.count_per_vertex(build(ctx, g), 0)
    assert t == r["total"]
    assert (pu == oracle.count_bbvp(g, 0, threads=8, per_vertex=True)["per_vertex"]).all()


def test_two_hop_overflow(ctx, oracle):
    """Low-degree anchors adjacent to hubs: > 3072 distinct higher-priority
    partners per anchor."""
    say("two-hop overflow")
    rng = np.random.default_rng(9)
    n_u, n_v = 20000, 400
    eu, ev = [], []
    hubs = np.arange(6)
    for h in hubs:                       # 6 hub V vertices adjacent to most U
        us = rng.choice(n_u, 6000, replace=False)
        eu.append(us); ev.append(np.full(us.size, h))
    others = rng.integers(6, n_v, size=40000)
    eu.append(rng.integers(0, n_u, size=others.size)); ev.append(others)
    u = np.concatenate(eu); v = np.concatenate(ev)
    key = np.unique(u.astype(np.int64) * n_v + v)
    u, v = key // n_v, key % n_v
    s = np.where(rng.random(u.size) < 0.7, 1, -1).astype(np.int8)
    g = G._finish(n_u, n_v, u, v, s)
    r = oracle.count_bbvp(g, 0, threads=8)
    assert ctx.count_global(build(ctx, g, 1 << 4)) == r["total"]
    assert ctx.count_global(build(ctx, g, 1 << 5)) == r["total"]
    st = ctx.last_stats()
    say("stats", st)


# ------------------------------------------------------------ batching
def test_config4_batch(ctx, oracle):
    say("config4 batch of 200")
    gs = G.config4(7, n_graphs=200)
    want = [oracle.count_bbvp(g, 0, threads=8)["total"] for g in gs]
    nu, nv, off, eu, ev, sg = G.concat(gs)
    hs = ctx.build_csr_batch(nu, nv, off, eu, ev, sg)
    got = ctx.count_batch(hs)
    assert list(got) == want
    again = ctx.count_batch(hs)          # replay of the captured launch
    assert list(again) == want
    for i in range(0, 200, 23):
        assert ctx.count_global(hs[i]) == want[i]
    # a sub-range and a permuted list of the same graphs
    sub = ctx.count_batch(hs[10:50])
    assert list(sub) == want[10:50]
    perm = list(range(199, -1, -3))
    assert list(ctx.count_batch([hs[i] for i in perm])) == [want[i] for i in perm]
    assert sum(want) > 0


def test_config4_full_batch(ctx):
    """All 8192 graphs of config 4 seed 1 in one batch (3.3e8 edges), built
    and counted once and replayed, against the oracle's stored per-graph
    counts (their sum and the sha256 of the int64 array)."""
    gold = golden("cfg4_seed1.json")
    say("config4 full batch: generate")
    gs = G.config4(1, n_graphs=gold["n_graphs"])
    want = np.array(gold["counts"], np.int64)
    nu, nv, off, eu, ev, sg = G.concat(gs)
    say("config4 full batch: build and count")
    hs = ctx.build_csr_batch(nu, nv, off, eu, ev, sg)
    got = np.asarray(ctx.count_batch(hs), np.int64)
    assert (got == want).all()
    assert int(got.sum()) == gold["sum"] and _digest(got) == gold["sha256"]
    assert (np.asarray(ctx.count_batch(hs), np.int64) == want).all()
    for h in hs:
        h.free()


def test_batch_rebuild_cycles(ctx, oracle):
    """Regression: batches built, counted, freed and rebuilt (new device
    buffers each time) must not replay a launch captured for an earlier
    batch; single-graph counts in between change the workspace too."""
    say("batch rebuild cycles")
    gs = G.config4(21, n_graphs=300)
    want = [oracle.count_bbvp(g, 0, threads=8)["total"] for g in gs]
    nu, nv, off, eu, ev, sg = G.concat(gs)
    for cycle in range(3):
        hs = ctx.build_csr_batch(nu, nv, off, eu, ev, sg)
        assert list(ctx.count_batch(hs)) == want, cycle
        assert list(ctx.count_batch(hs)) == want, cycle
        for h in hs:
            h.free()
        one = build(ctx, gs[cycle])
        assert ctx.count_global(one) == want[cycle]
        one.free()
    half = G.concat(gs[:150])
    hs = ctx.build_csr_batch(*half)
    assert list(ctx.count_batch(hs)) == want[:150]


# -------------------------------------------------------------- serving
def test_serving_mix_matches_alone(ctx, oracle, B):
    say("serving")
    rng = np.random.default_rng(31)
    gs = G.config4(11, n_graphs=60) + [G.config2(2, scale=0.05)]
    want = [oracle.count_bbvp(g, 0, threads=8)["total"] for g in gs]
    order = rng.permutation(len(gs))
    tickets = {}
    for i in order:
        g = gs[i]
        tickets[i] = ctx.submit_coo(g.n_u, g.n_v, g.eu, g.ev, g.sign)
    got = {i: ctx.wait(t) for i, t in tickets.items()}
    assert [got[i] for i in range(len(gs))] == want
    # poll semantics
    t = ctx.submit_coo(gs[0].n_u, gs[0].n_v, gs[0].eu, gs[0].ev, gs[0].sign)
    while True:
        v = ctx.poll(t)
        if v is not None:
            break
    assert v == want[0]
    with pytest.raises(B.BBCError) as ei:
        ctx.poll(t)
    assert ei.value.name == "BBC_E_UNKNOWN_TICKET"
    # a bad request fails alone
    bad = ctx.submit_coo(2, 2, np.array([0, 0], np.uint32), np.array([1, 1], np.uint32),
                         np.array([1, 1], np.int8))
    good = ctx.submit_coo(gs[1].n_u, gs[1].n_v, gs[1].eu, gs[1].ev, gs[1].sign)
    with pytest.raises(B.BBCError) as ei:
        ctx.wait(bad)
    assert ei.value.name == "BBC_E_DUP_EDGE"
    assert ctx.wait(good) == want[1]
    # prebuilt graphs through submit
    hs = [build(ctx, gs[i]) for i in range(5)]
    ts = [ctx.submit(h) for h in hs]
    assert [ctx.wait(t) for t in ts] == want[:5]


# --------------------------------------------------- full-size configs
def test_config2_full(ctx):
    gold = golden("cfg2_seed1.json")
    say("config2 full")
    g = G.config2(1)
    assert g.m == gold["m"]
    h = build(ctx, g)
    assert ctx.count_global(h) == gold["total"]
    pu, t = ctx.count_per_vertex(h, 0)
    assert t == gold["total"]
    assert hashlib.sha256(pu.astype("<i8").tobytes()).hexdigest() == gold["per_u_sha256"]
    pv, _ = ctx.count_per_vertex(h, 1)
    assert hashlib.sha256(pv.astype("<i8").tobytes()).hexdigest() == gold["per_v_sha256"]
    for flags in (1 << 4, 1 << 5):
        assert ctx.count_global(build(ctx, g, flags)) == gold["total"]


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i8").tobytes()).hexdigest()


def _optional_golden(name):
    import os
    from tests.gpu_common import GOLD
    p = os.path.join(GOLD, name)
    if not os.path.exists(p):
        return None
    import json
    with open(p) as f:
        return json.load(f)


def test_config3_full(ctx):
    """Config 3 at full size (2M x 500k, 40M edges).

    Against the oracle, which ran Algorithm 2 over every anchor, in shards:
    - the U-anchored total;
    - the sha256 of all 2M per-U-vertex counts;
    - the values of the 16 highest-degree U vertices and of 64 sampled ones;
    - the per-vertex values of the highest-degree V vertices.
    Also against earlier sampled per-vertex values of both sides. U- and
    V-anchored totals must agree, and per-vertex sums must be 3 x the total."""
    gold = golden("cfg3_seed1_sample.json")
    full = _optional_golden("cfg3_seed1_full.json")
    vhubs = _optional_golden("cfg3_seed1_v_hubs.json")
    say("config3 full: generate")
    g = G.config3(1)
    assert g.m == gold["m"]
    say("config3 full: U anchored")
    hu = build(ctx, g, 1 << 4)
    pu, tu = ctx.count_per_vertex(hu, 0)
    for k, v in gold["per_u_sample"].items():
        assert int(pu[int(k)]) == v, k
    assert int(pu.sum()) == 3 * tu
    assert ctx.count_global(hu) == tu
    if full is not None:
        say("config3 full: against the whole-graph oracle values")
        assert full["m"] == g.m
        assert tu == full["total"]
        for k, v in full["per_u_hubs"].items():
            assert int(pu[int(k)]) == v, k
        for k, v in full["per_u_sample"].items():
            assert int(pu[int(k)]) == v, k
        assert _digest(pu) == full["per_u_sha256"]
    hu.free()
    say("config3 full: V anchored")
    hv = build(ctx, g, 1 << 5)
    pv, tv = ctx.count_per_vertex(hv, 1)
    assert tv == tu
    for k, v in gold["per_v_sample"].items():
        assert int(pv[int(k)]) == v, k
    if vhubs is not None:
        for k, v in vhubs["per_v_hubs"].items():
            assert int(pv[int(k)]) == v, k
    assert int(pv.sum()) == 3 * tu


def test_config3_switching_invariance(ctx):
    """A switching (signs times l(u) l(v) for any labels) and the negation of
    every sign keep each (3,3)-biclique's balance, so they keep the count:
    config 3 at full size with its hidden labels taken out of the signs, and
    with all signs negated, counts the same as config 3 itself."""
    say("config3 switching: generate")
    g = G.config3(1)
    lu, lv = g.meta["label_u"], g.meta["label_v"]
    h0 = build(ctx, g, 1 << 4)
    base = ctx.count_global(h0)
    h0.free()
    full = _optional_golden("cfg3_seed1_full.json")
    if full is not None:
        assert base == full["total"]
    unsw = (g.sign * lu[g.eu] * lv[g.ev]).astype(np.int8)
    for name, sg in (("unswitched", unsw), ("negated", (-g.sign).astype(np.int8))):
        say("config3 switching:", name)
        h = ctx.build_csr(g.n_u, g.n_v, g.eu, g.ev, sg, 1 << 4)
        assert ctx.count_global(h) == base, name
        h.free()


# ------------------------------------------------- side from degree sums
def _side_rule(g):
    """The documented default of the anchor side: sum_o C(d_o, 2) wedges,
    weighted by 1 + (edge-weighted mean degree of the anchor side) / 32."""
    du = np.bincount(np.asarray(g.eu, np.int64), minlength=g.n_u).astype(np.int64)
    dv = np.bincount(np.asarray(g.ev, np.int64), minlength=g.n_v).astype(np.int64)
    m = int(du.sum())
    if m == 0:
        return 0
    c2u, c2v = int((du * (du - 1) // 2).sum()), int((dv * (dv - 1) // 2).sum())
    d2u, d2v = int((du * du).sum()), int((dv * dv).sum())
    cost_u = float(c2v) * (1.0 + (d2u / m) / 32.0)
    cost_v = float(c2u) * (1.0 + (d2v / m) / 32.0)
    return 1 if cost_v < cost_u else 0


def test_side_stats_batch(ctx):
    """The per-graph degree sums behind the side choice, for a batch mixing
    many small graphs (several per workgroup and per wave) with graphs that
    span many workgroups, in both orientations."""
    say("side statistics")
    rng = np.random.default_rng(99)
    gs = G.config4(5, n_graphs=300)
    gs.insert(120, G.config2(3, scale=0.2))
    gs.insert(7, G.config2(4, scale=0.1).transpose())
    gs += [G.tiny_random(rng, 9, 9) for _ in range(200)]
    want = [_side_rule(g) for g in gs]
    assert 0 < sum(want) < len(want)          # both sides occur
    nu, nv, off, eu, ev, sg = G.concat(gs)
    hs = ctx.build_csr_batch(nu, nv, off, eu, ev, sg)
    got = [h.info().anchor_side for h in hs]
    assert got == want



# ------------------------------------------- general q (p = 3 on one side)
def _complete_rows(n, m, neg):
    return ["".join("-" if neg(i, j) else "+" for j in range(m)) for i in range(n)]


def test_general_q_closed_forms(ctx):
    """All-positive K_{n,m}: C(n,p) C(m,q); the two-block pattern (sign -1
    on U2 x V2): pure C(m,q) + mixed (C(m1,q) + C(m2,q)) for (3, q), and the
    same with the sides exchanged for (q, 3)."""
    say("general q closed forms")
    comb = math.comb
    for n, m in [(6, 9), (9, 7)]:
        g = G.from_rows(_complete_rows(n, m, lambda i, j: False))
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        for q in range(3, 8):
            assert ctx.count_global(hu, 3, q) == C3(n) * comb(m, q), (n, m, q)
            assert ctx.count_global(hv, q, 3) == comb(n, q) * C3(m), (n, m, q)
    for n1, n2, m1, m2 in [(3, 4, 6, 3), (5, 4, 4, 5), (2, 7, 8, 1)]:
        n, m = n1 + n2, m1 + m2
        g = G.from_rows(_complete_rows(n, m, lambda i, j: i >= n1 and j >= m1))
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        pure, pure_t = C3(n1) + C3(n2), C3(m1) + C3(m2)
        for q in range(3, 8):
            want = pure * comb(m, q) + (C3(n) - pure) * (comb(m1, q) + comb(m2, q))
            want_t = pure_t * comb(n, q) + (C3(m) - pure_t) * (comb(n1, q) + comb(n2, q))
            assert ctx.count_global(hu, 3, q) == want, (n1, n2, m1, m2, q)
            assert ctx.count_global(hv, q, 3) == want_t, (n1, n2, m1, m2, q)


def test_general_q_vs_oracle(ctx, oracle):
    """(3, q) on U and (q, 3) on V against Algorithm 2 with that q, on the
    small configurations (planted balanced blocks make q >= 4 counts large),
    and against the definition on dense tiny graphs."""
    say("general q vs oracle")
    for g in [G.config1(1), G.config1(4), G.config2(5, scale=0.04)]:
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        for q in (4, 5, 6, 7):
            want_u = oracle.count_bbvp_q(g, q, 0, threads=8)["total"]
            want_v = oracle.count_bbvp_q(g, q, 1, threads=8)["total"]
            assert ctx.count_global(hu, 3, q) == want_u, (g.n_u, q)
            assert ctx.count_global(hv, q, 3) == want_v, (g.n_u, q)
        # q = 3 through the same call equals the (3,3) count on either side
        assert ctx.count_global(hu, 3, 3) == ctx.count_global(hv, 3, 3)
    rng = np.random.default_rng(808)
    nonzero = 0
    for it in range(120):
        g = G.tiny_random(rng, 9, 9, density=float(rng.choice([0.7, 0.9, 1.0])))
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        for q in (4, 5):
            b = oracle.count_bruteforce_pq(g, 3, q)
            assert ctx.count_global(hu, 3, q) == b, (it, q)
            assert ctx.count_global(hv, q, 3) == oracle.count_bruteforce_pq(g, q, 3), (it, q)
            nonzero += b > 0
        hu.free(); hv.free()
    assert nonzero > 20


def test_general_q_rejected(ctx, B):
    say("general q rejected")
    g = G.config1(2)
    hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
    for h, p, q in [(hv, 3, 6), (hu, 6, 3), (hu, 3, 8), (hu, 6, 6), (hv, 4, 8), (hu, 2, 3), (hv, 3, 2)]:
        with pytest.raises(B.BBCError) as ei:
            ctx.count_global(h, p, q)
        assert ei.value.name == "BBC_E_UNSUPPORTED", (p, q)
    assert ctx.count_global(hu, 3, 5) >= 0


def test_general_q_config2_full(ctx):
    """Config 2 at full size: (3, 4), (3, 5) anchored on U and (4, 3), (5, 3)
    anchored on V against the oracle's values (cfg2_seed1_general_q.json,
    written by tests/golden/make_golden.py from oracle/ only)."""
    say("general q config2 full")
    gold = golden("cfg2_seed1_general_q.json")
    g = G.config2(1)
    assert g.m == gold["m"]
    hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
    for key, want in gold["counts"].items():
        p, q = (int(x) for x in key.split(","))
        got = ctx.count_global(hu if p == 3 else hv, p, q)
        assert got == want, key


# ------------------------------------------------- 4 vertices on the anchor side
@pytest.mark.parametrize("n,n1,m,m1", [(12, 5, 544, 200), (10, 4, 633, 400), (9, 3, 1056, 700)])
def test_general_pq_wide_masks(ctx, n, n1, m, m1):
    """Masks of 17, 20 (ragged) and 33 words, anchored on U, for every count
    mode: K_{n,m} with sign -1 on U2 x V2 holds pure(p) C(m, q) + (C(n, p) -
    pure(p)) (C(m1, q) + C(m2, q)) balanced (p, q)-bicliques, pure(p) = C(n1, p)
    + C(n2, p). The pure pairs meet in m > 512 common bits and the mixed ones
    in m1 or m2."""
    C = math.comb
    n2, m2 = n - n1, m - m1
    h = build(ctx, _complete_signed(n, m, n1, m1), 1 << 4)
    qs = {3: (3, 4, 5, 7), 4: (3, 4, 5), 5: (3, 4)} if m < 1000 else {3: (3, 4, 5), 4: (3, 4), 5: (3,)}
    for p, ql in qs.items():
        for q in ql:
            say("wide masks", n, m, p, q)
            pure = C(n1, p) + C(n2, p)
            want = pure * C(m, q) + (C(n, p) - pure) * (C(m1, q) + C(m2, q))
            assert want < 1 << 64
            assert ctx.count_global(h, p, q) == want, (n, m, p, q)


@pytest.mark.parametrize("n,n1,m,m1", [(12, 5, 544, 200), (10, 4, 633, 400), (9, 3, 1056, 700)])
def test_per_vertex_wide_masks(ctx, n, n1, m, m1):
    """Per-vertex counts on both sides with masks of 17, 20 and 33 words
    (anchored on U), K_{n,m} with sign -1 on U2 x V2. A U vertex of block b
    lies in C(n_b - 1, 2) pure triples (all of V one class) and C(n - 1, 2) -
    C(n_b - 1, 2) mixed ones (classes V1, V2); a V vertex of block c lies in
    C(m - 1, 2) of the R-sets of each pure triple and C(m_c - 1, 2) of each
    mixed one."""
    C = math.comb
    n2, m2 = n - n1, m - m1
    h = build(ctx, _complete_signed(n, m, n1, m1), 1 << 4)
    pure_l = C3(n1) + C3(n2)
    mixed_l = C3(n) - pure_l
    total = pure_l * C3(m) + mixed_l * (C3(m1) + C3(m2))
    say("per-vertex wide", n, m)
    pu, tu = ctx.count_per_vertex(h, 0)
    pv, tv = ctx.count_per_vertex(h, 1)
    assert tu == total and tv == total
    for u in range(n):
        nb = n1 if u < n1 else n2
        want = C(nb - 1, 2) * C3(m) + (C(n - 1, 2) - C(nb - 1, 2)) * (C3(m1) + C3(m2))
        assert pu[u] == want, u
    for v in range(m):
        mc = m1 if v < m1 else m2
        assert pv[v] == pure_l * C(m - 1, 2) + mixed_l * C(mc - 1, 2), v


def test_p4_closed_forms(ctx):
    """All-positive K_{n,m}: C(n,4) C(m,q) for (4, q) anchored on U and for
    (q, 4) anchored on V; the two-block sign pattern for (4, q)."""
    C = math.comb
    for n, m in [(5, 6), (9, 40), (70, 5)]:
        g = G.from_rows(["+" * m] * n)
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        for q in range(3, 8):
            say("p4 complete", n, m, q)
            assert ctx.count_global(hu, 4, q) == C(n, 4) * C(m, q)
            assert ctx.count_global(hv, q, 4) == C(n, q) * C(m, 4)
    for (n1, n2, m1, m2, q) in [(3, 4, 4, 3, 3), (10, 20, 15, 5, 4), (33, 31, 40, 2, 5)]:
        n, m = n1 + n2, m1 + m2
        rows = ["".join("-" if (i >= n1 and j >= m1) else "+" for j in range(m)) for i in range(n)]
        pure = C(n1, 4) + C(n2, 4)
        want = pure * C(m, q) + (C(n, 4) - pure) * (C(m1, q) + C(m2, q))
        assert ctx.count_global(build(ctx, G.from_rows(rows), 1 << 4), 4, q) == want


def test_p4_vs_oracle(ctx, oracle):
    """Config 1 (seeds 1, 2, planted blocks included) against Algorithm 2 with
    p = 4 on both sides; (4, 3) and (3, 4) also through the p = 3 path on the
    other side."""
    for seed in (1, 2):
        g = G.config1(seed)
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        for q in (3, 4, 5):
            say("p4 config1", seed, q)
            want_u = oracle.count_bbvp_p4(g, q, 0, threads=8)["total"]
            want_v = oracle.count_bbvp_p4(g, q, 1, threads=8)["total"]
            assert ctx.count_global(hu, 4, q) == want_u
            assert ctx.count_global(hv, q, 4) == want_v
        assert ctx.count_global(hu, 4, 3) == ctx.count_global(hv, 4, 3)
        assert ctx.count_global(hv, 3, 4) == ctx.count_global(hu, 3, 4)


def test_p4_tiny_vs_bruteforce(ctx, oracle):
    rng = np.random.default_rng(23)
    for t in range(80):
        n_u, n_v = int(rng.integers(4, 10)), int(rng.integers(4, 10))
        dense = rng.random((n_u, n_v)) < rng.uniform(0.5, 1.0)
        u, v = np.nonzero(dense)
        s = np.where(rng.random(u.size) < rng.uniform(0.3, 1.0), 1, -1).astype(np.int8)
        g = G._finish(n_u, n_v, u, v, s)
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        for q in (3, 4, 5):
            assert ctx.count_global(hu, 4, q) == oracle.count_bruteforce_pq(g, 4, q), (t, q)
            assert ctx.count_global(hv, q, 4) == oracle.count_bruteforce_pq(g, q, 4), (t, q)


def test_p4_config2_full(ctx):
    """Config 2 at full size through the path with 4 vertices on the anchor
    side: (4, 3) anchored on U and (3, 4) anchored on V equal the oracle's
    counts of the same bicliques through 3 vertices on the other side
    (tests/golden/cfg2_seed1_general_q.json)."""
    gold = golden("cfg2_seed1_general_q.json")["counts"]
    g = G.config2(1)
    say("p4 config2 (4,3) U")
    assert ctx.count_global(build(ctx, g, 1 << 4), 4, 3) == gold["4,3"]
    say("p4 config2 (3,4) V")
    assert ctx.count_global(build(ctx, g, 1 << 5), 3, 4) == gold["3,4"]


# ------------------------------------------------- 5 vertices on the anchor side
def test_p5_closed_forms(ctx):
    C = math.comb
    for n, m in [(6, 7), (12, 33), (40, 5)]:
        g = G.from_rows(["+" * m] * n)
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        for q in range(3, 8):
            say("p5 complete", n, m, q)
            assert ctx.count_global(hu, 5, q) == C(n, 5) * C(m, q)
            assert ctx.count_global(hv, q, 5) == C(n, q) * C(m, 5)
    for (n1, n2, m1, m2, q) in [(4, 5, 4, 3, 3), (10, 12, 15, 5, 4)]:
        n, m = n1 + n2, m1 + m2
        rows = ["".join("-" if (i >= n1 and j >= m1) else "+" for j in range(m)) for i in range(n)]
        pure = C(n1, 5) + C(n2, 5)
        want = pure * C(m, q) + (C(n, 5) - pure) * (C(m1, q) + C(m2, q))
        assert ctx.count_global(build(ctx, G.from_rows(rows), 1 << 4), 5, q) == want


def test_p5_vs_oracle(ctx, oracle):
    """Config 1 (seed 1) against Algorithm 2 with p = 5 on both sides, and 40
    dense tiny graphs against the definition."""
    g = G.config1(1)
    hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
    for q in (3, 4):
        say("p5 config1", q)
        assert ctx.count_global(hu, 5, q) == oracle.count_bbvp_pk(g, 5, q, 0, threads=8)["total"]
        assert ctx.count_global(hv, q, 5) == oracle.count_bbvp_pk(g, 5, q, 1, threads=8)["total"]
    rng = np.random.default_rng(31)
    for t in range(40):
        n_u, n_v = int(rng.integers(5, 10)), int(rng.integers(5, 10))
        dense = rng.random((n_u, n_v)) < rng.uniform(0.6, 1.0)
        u, v = np.nonzero(dense)
        s = np.where(rng.random(u.size) < rng.uniform(0.3, 1.0), 1, -1).astype(np.int8)
        gt = G._finish(n_u, n_v, u, v, s)
        hu, hv = build(ctx, gt, 1 << 4), build(ctx, gt, 1 << 5)
        for q in (3, 4):
            assert ctx.count_global(hu, 5, q) == oracle.count_bruteforce_pq(gt, 5, q), (t, q)
            assert ctx.count_global(hv, q, 5) == oracle.count_bruteforce_pq(gt, q, 5), (t, q)


def test_top_vertices(ctx, oracle):
    """The k vertices in the most balanced (3,3)-bicliques, from the oracle's
    per-vertex counts (descending, ties to the smaller id), on both sides and
    for either anchor side of the build."""
    g = G.config1(1)
    per = {0: oracle.count_bbvp(g, 0, per_vertex=True)["per_vertex"],
           1: oracle.count_bbvp(g, 1, per_vertex=True)["per_vertex"]}
    for flags in (1 << 4, 1 << 5):
        h = build(ctx, g, flags)
        for side in (0, 1):
            pv = per[side]
            order = sorted(range(len(pv)), key=lambda i: (-int(pv[i]), i))
            for k in (1, 10, len(pv) + 5):
                ids, cnt = ctx.top_vertices(h, side, k)
                want = order[:k]
                assert ids.tolist() == want, (flags, side, k)
                assert cnt.tolist() == [int(pv[i]) for i in want]
    assert ctx.top_vertices(build(ctx, g), 0, 0)[0].size == 0
