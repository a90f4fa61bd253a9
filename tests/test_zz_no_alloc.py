"""The no-allocation entry point (bbc_count_global_noalloc) against
bbc_count_global on the same graphs: two calls in a row, the second on a
smaller graph, then a graph too large for the static scratch (a clear
BBC_E_NOMEM, and the scratch still works afterwards). Exact (tolerance 0)."""
import ctypes

import pytest

from paper_2605_03603_amd import generators as G
from tests.gpu_common import build, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    need_gpu()
    from paper_2605_03603_amd import bbc
    return bbc


def noalloc(B, ctx, h, p=3, q=3):
    out = ctypes.c_int64()
    st = B.lib.bbc_count_global_noalloc(ctx.handle, h.handle, p, q, ctypes.byref(out))
    return st, out.value


def test_noalloc_matches_count_global(B):
    with B.Context(0) as ctx:
        big, small = G.config2(1, scale=0.05), G.config1(2)
        for g in (big, small):                     # the second call on a smaller graph
            h = build(ctx, g, 1 << 4)
            want = ctx.count_global(h)
            say("noalloc", g.m, want)
            st, got = noalloc(B, ctx, h)
            assert st == 0 and got == want
            h.free()
        # general (p, q) through the same scratch
        h = build(ctx, G.config1(3), 1 << 4)
        for p, q in ((3, 4), (4, 3)):
            st, got = noalloc(B, ctx, h, p, q)
            assert st == 0 and got == ctx.count_global(h, p, q)
        h.free()


def test_noalloc_rejects_beyond_scratch(B):
    with B.Context(0) as ctx:
        g = G.config2(1)                            # needs more than 256 MiB of workspace
        h = build(ctx, g, 1 << 4)
        st, _ = noalloc(B, ctx, h)
        assert B.STATUS_NAMES[st] == "BBC_E_NOMEM"
        assert "static scratch" in B.lib.bbc_last_error(ctx.handle).decode()
        h.free()
        small = build(ctx, G.config1(4))
        st, got = noalloc(B, ctx, small)
        assert st == 0 and got == ctx.count_global(small)
        small.free()
