"""GPU parity of the wedge-centric path (Algorithm 1, bbc_count_bbwc) against
closed forms, the oracle and the definition. Exact (tolerance 0)."""
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


def test_bbwc_closed_forms(ctx):
    C = math.comb
    for n, m in [(3, 3), (6, 9), (40, 7)]:
        g = G.from_rows(["+" * m] * n)
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        for q in (3, 4, 7):
            say("bbwc complete", n, m, q)
            assert ctx.count_bbwc(hu, 3, q) == C(n, 3) * C(m, q)
            assert ctx.count_bbwc(hv, q, 3) == C(n, q) * C(m, 3)
    for (n1, n2, m1, m2) in [(3, 4, 4, 3), (10, 20, 15, 5)]:
        n, m = n1 + n2, m1 + m2
        rows = ["".join("-" if (i >= n1 and j >= m1) else "+" for j in range(m)) for i in range(n)]
        pure = C(n1, 3) + C(n2, 3)
        want = pure * C(m, 3) + (C(n, 3) - pure) * (C(m1, 3) + C(m2, 3))
        assert ctx.count_bbwc(build(ctx, G.from_rows(rows)), 3, 3) == want


def test_bbwc_vs_oracle_and_bbvp(ctx, oracle):
    """Config 1 (seeds 1..3) and config 2 at 1 % scale: Algorithm 1 on the GPU
    equals Algorithm 2 in the oracle and on the GPU, for q = 3..5 both ways."""
    graphs = [G.config1(s) for s in (1, 2, 3)] + [G.config2(3, scale=0.01)]
    for gi, g in enumerate(graphs):
        hu, hv = build(ctx, g, 1 << 4), build(ctx, g, 1 << 5)
        for q in (3, 4, 5):
            say("bbwc vs oracle", gi, q)
            want = oracle.count_bbvp_q(g, q, 0, threads=8)["total"]
            assert ctx.count_bbwc(hu, 3, q) == want == ctx.count_global(hu, 3, q)
            want_v = oracle.count_bbvp_q(g, q, 1, threads=8)["total"]
            assert ctx.count_bbwc(hv, q, 3) == want_v == ctx.count_global(hv, q, 3)


def test_bbwc_tiny_vs_bruteforce(ctx, oracle):
    rng = np.random.default_rng(19)
    for t in range(60):
        g = G.tiny_random(rng, 8, 8, density=float(rng.uniform(0.4, 1.0)))
        assert ctx.count_bbwc(build(ctx, g), 3, 3) == oracle.count_bruteforce(g), t


def test_bbwc_limits(ctx, B):
    """(p, q) other than 3 on the anchor side, and an anchor beyond the
    per-anchor table (K_{100,100}: 100 C(99, 2) wedge pairs at the top anchor)."""
    g = G.config1(1)
    with pytest.raises(B.BBCError) as e:
        ctx.count_bbwc(build(ctx, g, 1 << 4), 4, 3)
    assert e.value.name == "BBC_E_UNSUPPORTED"
    big = G.from_rows(["+" * 100] * 100)
    with pytest.raises(B.BBCError) as e:
        ctx.count_bbwc(build(ctx, big, 1 << 4), 3, 3)
    assert e.value.name == "BBC_E_UNSUPPORTED"
    assert ctx.count_global(build(ctx, big)) == math.comb(100, 3) ** 2
