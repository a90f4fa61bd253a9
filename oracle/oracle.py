"""Python access to the plain CPU oracle (bbc_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this module; the product package never does.

Every function takes a :class:`SignedBipartite`-like object (attributes n_u,
n_v, eu, ev, sign) and returns exact Python integers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bbc_oracle.c")
_LIB = os.path.join(_HERE, "libbbc_oracle.so")
_LIB_NATIVE = os.path.join(_HERE, "libbbc_oracle_native.so")
_lib = None

_u32p = ctypes.POINTER(ctypes.c_uint32)
_i8p = ctypes.POINTER(ctypes.c_int8)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False, out: Optional[str] = None, mutant: int = 0,
          native: bool = False) -> str:
    """Compile the oracle with gcc: plain -O2 for the tests (the library then
    runs on any x86-64 host), or -O3 -march=native (native=True, into
    libbbc_oracle_native.so unless `out` is given) for timing it on the host
    that runs it. Same source, same arithmetic. `mutant` > 0 builds a variant
    with a planted mistake (mutation test)."""
    target = out or (_LIB_NATIVE if native else _LIB)
    if force or out or not os.path.exists(target) or os.path.getmtime(target) < os.path.getmtime(_SRC):
        tmp = target + f".tmp{os.getpid()}"
        opt = ["-O3", "-march=native"] if native else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-std=gnu11", "-shared", "-fPIC", "-pthread",
                               f"-DORC_MUTANT={int(mutant)}", "-o", tmp, _SRC])
        os.replace(tmp, target)
    return target


def use_library(path: Optional[str]):
    """Point the wrappers at another build of the oracle (None: the default)."""
    global _lib
    _lib = None if path is None else _bind(ctypes.CDLL(path))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(L):
    L.orc_butterfly_balanced.argtypes = [ctypes.c_int] * 4
    L.orc_butterfly_balanced.restype = ctypes.c_int
    L.orc_wedge_type.argtypes = [ctypes.c_int] * 3
    L.orc_wedge_type.restype = ctypes.c_int
    L.orc_choose3.argtypes = [ctypes.c_uint64]
    L.orc_choose3.restype = ctypes.c_uint64
    L.orc_count_bruteforce.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _u32p, _u32p,
                                       _i8p, _u64p, _i64p, _i64p]
    L.orc_count_bruteforce.restype = ctypes.c_int
    L.orc_count_bbvp.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _u32p, _u32p,
                                 _i8p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _u64p, _u64p,
                                 _i64p]
    L.orc_count_bbvp.restype = ctypes.c_int
    L.orc_count_bbvp_shard.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _u32p,
                                       _u32p, _i8p, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_int64, _u64p, _u64p, _i64p]
    L.orc_count_bbvp_shard.restype = ctypes.c_int
    L.orc_count_bbvp_watch.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _u32p,
                                       _u32p, _i8p, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int64, _u32p,
                                       ctypes.POINTER(ctypes.c_uint8), _u64p, _u64p, _u64p]
    L.orc_count_bbvp_watch.restype = ctypes.c_int
    L.orc_count_bbvp_q.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _u32p, _u32p,
                                   _i8p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                   _u64p, _u64p, _i64p]
    L.orc_count_bbvp_q.restype = ctypes.c_int
    L.orc_count_bbvp_pk.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _u32p, _u32p,
                                    _i8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    _u64p, _u64p]
    L.orc_count_bbvp_pk.restype = ctypes.c_int
    L.orc_count_bruteforce_pq.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, _u32p,
                                          _u32p, _i8p, ctypes.c_int, ctypes.c_int, _u64p]
    L.orc_count_bruteforce_pq.restype = ctypes.c_int
    L.orc_vertex_counts.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _u32p, _u32p,
                                    _i8p, ctypes.c_int, ctypes.c_int64, _u32p, _u64p]
    L.orc_vertex_counts.restype = ctypes.c_int
    L.orc_anchor_detail.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, _u32p, _u32p,
                                    _i8p, ctypes.c_int, ctypes.c_uint32, ctypes.c_int,
                                    ctypes.c_int64, _u32p, _i64p, ctypes.c_int64, _i64p, _i64p,
                                    _u64p]
    L.orc_anchor_detail.restype = ctypes.c_int
    return L


def _arrs(g):
    eu = np.ascontiguousarray(g.eu, dtype=np.uint32)
    ev = np.ascontiguousarray(g.ev, dtype=np.uint32)
    sg = np.ascontiguousarray(g.sign, dtype=np.int8)
    return eu, ev, sg


def _p(a, t):
    return a.ctypes.data_as(t)


def butterfly_balanced(s1: int, s2: int, s3: int, s4: int) -> bool:
    return bool(lib().orc_butterfly_balanced(s1, s2, s3, s4))


WEDGE_TYPES = ("ss", "sd", "ds", "dd")


def wedge_type(s_u1v: int, s_w1v: int, s_w2v: int) -> str:
    return WEDGE_TYPES[lib().orc_wedge_type(s_u1v, s_w1v, s_w2v)]


def choose3(n: int) -> int:
    return int(lib().orc_choose3(n))


def count_bruteforce(g, per_vertex: bool = False):
    """Definition-level count (O1); tiny graphs only (n_u, n_v <= 24)."""
    eu, ev, sg = _arrs(g)
    out = np.zeros(1, np.uint64)
    pu = np.zeros(max(g.n_u, 1), np.int64)
    pv = np.zeros(max(g.n_v, 1), np.int64)
    rc = lib().orc_count_bruteforce(g.n_u, g.n_v, eu.size, _p(eu, _u32p), _p(ev, _u32p),
                                    _p(sg, _i8p), _p(out, _u64p), _p(pu, _i64p), _p(pv, _i64p))
    if rc != 0:
        raise ValueError(f"orc_count_bruteforce failed ({rc})")
    if per_vertex:
        return int(out[0]), pu[:g.n_u].copy(), pv[:g.n_v].copy()
    return int(out[0])


def count_bbvp(g, side: int = 0, threads: int = 1, anchor_stride: int = 1,
               per_vertex: bool = False):
    """Algorithm 2 for p = q = 3 (O2; O3 is side=1).

    Returns dict(total, feasible, candidates, side[, per_vertex])."""
    eu, ev, sg = _arrs(g)
    out = np.zeros(2, np.uint64)
    st = np.zeros(3, np.uint64)
    n_side = g.n_v if (side == 1 or (side < 0 and g.n_v < g.n_u)) else g.n_u
    pv = np.zeros(max(n_side, 1), np.int64) if per_vertex else None
    rc = lib().orc_count_bbvp(g.n_u, g.n_v, eu.size, _p(eu, _u32p), _p(ev, _u32p), _p(sg, _i8p),
                              side, threads, anchor_stride, _p(out, _u64p), _p(st, _u64p),
                              _p(pv, _i64p) if pv is not None else None)
    if rc == -1:
        raise ValueError("orc_count_bbvp: repeated or out-of-range edge")
    total = int(out[0]) | (int(out[1]) << 64)
    res = {"total": total, "feasible": int(st[0]), "candidates": int(st[1]), "side": int(st[2])}
    if per_vertex:
        if rc == -2:
            raise OverflowError("per-vertex count exceeds int64")
        res["per_vertex"] = pv[:n_side].copy()
    return res


def count_bbvp_shard(g, side: int, n_shards: int, shard: int, threads: int = 1,
                     per_vertex: bool = False) -> dict:
    """Algorithm 2 for p = q = 3 over the anchors whose id is `shard` modulo
    `n_shards` (side 0: U, 1: V). The shards partition the anchors, so their
    totals, feasible and candidate counts and per-vertex arrays sum to those
    of count_bbvp over the whole side.

    Returns dict(total, feasible, candidates, side[, per_vertex])."""
    eu, ev, sg = _arrs(g)
    out = np.zeros(2, np.uint64)
    st = np.zeros(3, np.uint64)
    n_side = g.n_v if side == 1 else g.n_u
    pv = np.zeros(max(n_side, 1), np.int64) if per_vertex else None
    rc = lib().orc_count_bbvp_shard(g.n_u, g.n_v, eu.size, _p(eu, _u32p), _p(ev, _u32p),
                                    _p(sg, _i8p), side, threads, n_shards, shard,
                                    _p(out, _u64p), _p(st, _u64p),
                                    _p(pv, _i64p) if pv is not None else None)
    if rc == -2:
        raise OverflowError("per-vertex count exceeds int64")
    if rc != 0:
        raise ValueError(f"orc_count_bbvp_shard failed ({rc})")
    total = int(out[0]) | (int(out[1]) << 64)
    res = {"total": total, "feasible": int(st[0]), "candidates": int(st[1]), "side": int(st[2])}
    if per_vertex:
        res["per_vertex"] = pv[:n_side].copy()
    return res


def count_bbvp_watch(g, side: int, watch, n_shards: int = 1, shard: int = 0, threads: int = 1,
                     anchor_on=None) -> dict:
    """count_bbvp_shard with a watch list of distinct vertices of the opposite
    side: for each, the number of balanced (3,3)-bicliques that contain it and
    are anchored in this shard (Lemma 1: a watched vertex in the wedge-type
    class of x members lies in C(x - 1, 2) of its class's bicliques).
    anchor_on: optional boolean array over the anchor side; anchors marked
    False are skipped (every biclique through a watched vertex is anchored at
    one of its neighbours).

    Returns dict(total, feasible, candidates, side, watch=[int per vertex])."""
    w = np.ascontiguousarray(np.asarray(watch, dtype=np.uint32))
    if w.size == 0:
        r = count_bbvp_shard(g, side, n_shards, shard, threads)
        r["watch"] = []
        return r
    eu, ev, sg = _arrs(g)
    out = np.zeros(2, np.uint64)
    st = np.zeros(3, np.uint64)
    wo = np.zeros(2 * max(w.size, 1), np.uint64)
    on = None
    if anchor_on is not None:
        on = np.ascontiguousarray(np.asarray(anchor_on, dtype=np.uint8))
        n_side = g.n_v if side == 1 else g.n_u
        if on.size != n_side:
            raise ValueError("anchor_on needs one entry per anchor-side vertex")
    rc = lib().orc_count_bbvp_watch(g.n_u, g.n_v, eu.size, _p(eu, _u32p), _p(ev, _u32p),
                                    _p(sg, _i8p), side, threads, n_shards, shard, w.size,
                                    _p(w, _u32p),
                                    on.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
                                    if on is not None else None,
                                    _p(out, _u64p), _p(st, _u64p), _p(wo, _u64p))
    if rc != 0:
        raise ValueError(f"orc_count_bbvp_watch failed ({rc})")
    total = int(out[0]) | (int(out[1]) << 64)
    return {"total": total, "feasible": int(st[0]), "candidates": int(st[1]), "side": int(st[2]),
            "watch": [int(wo[2 * i]) | (int(wo[2 * i + 1]) << 64) for i in range(w.size)]}


def count_bbvp_q(g, q: int, side: int = 0, threads: int = 1, anchor_stride: int = 1) -> dict:
    """Algorithm 2 with p = 3 on the anchor side and q (3..7) on the other:
    side 0 counts balanced (3, q)-bicliques, side 1 balanced (q, 3)-bicliques.

    Returns dict(total, feasible, candidates, side)."""
    eu, ev, sg = _arrs(g)
    out = np.zeros(2, np.uint64)
    st = np.zeros(3, np.uint64)
    rc = lib().orc_count_bbvp_q(g.n_u, g.n_v, eu.size, _p(eu, _u32p), _p(ev, _u32p),
                                _p(sg, _i8p), side, threads, anchor_stride, q, _p(out, _u64p),
                                _p(st, _u64p), None)
    if rc != 0:
        raise ValueError(f"orc_count_bbvp_q failed ({rc})")
    total = int(out[0]) | (int(out[1]) << 64)
    return {"total": total, "feasible": int(st[0]), "candidates": int(st[1]), "side": int(st[2])}


def count_bbvp_pk(g, p: int, q: int, side: int = 0, threads: int = 1, dense: bool = False) -> dict:
    """Algorithm 2 with p = 4 or 5 on the anchor side ((p - 1)-subsets of the
    candidate set, 2^(p-1) wedge-type classes) and q (3..7) on the other:
    side 0 counts balanced (p, q)-bicliques, side 1 balanced (q, p)-bicliques.
    dense=True takes the dense-vector form for p = 4 as well.

    Returns dict(total, feasible, candidates)."""
    eu, ev, sg = _arrs(g)
    out = np.zeros(2, np.uint64)
    st = np.zeros(2, np.uint64)
    pp = -4 if (dense and p == 4) else p
    rc = lib().orc_count_bbvp_pk(g.n_u, g.n_v, eu.size, _p(eu, _u32p), _p(ev, _u32p),
                                 _p(sg, _i8p), side, threads, pp, q, _p(out, _u64p), _p(st, _u64p))
    if rc != 0:
        raise ValueError(f"orc_count_bbvp_pk failed ({rc})")
    total = int(out[0]) | (int(out[1]) << 64)
    return {"total": total, "feasible": int(st[0]), "candidates": int(st[1])}


def count_bruteforce_pq(g, p: int, q: int) -> int:
    """Definition-level count of balanced (p, q)-bicliques (|L| = p in U,
    |R| = q in V); tiny graphs only (n_u, n_v <= 24)."""
    eu, ev, sg = _arrs(g)
    out = np.zeros(1, np.uint64)
    rc = lib().orc_count_bruteforce_pq(g.n_u, g.n_v, eu.size, _p(eu, _u32p), _p(ev, _u32p),
                                       _p(sg, _i8p), p, q, _p(out, _u64p))
    if rc != 0:
        raise ValueError(f"orc_count_bruteforce_pq failed ({rc})")
    return int(out[0])


def vertex_counts(g, side: int, xs: Sequence[int]) -> list:
    """Number of balanced (3,3)-bicliques containing each listed vertex."""
    eu, ev, sg = _arrs(g)
    x = np.ascontiguousarray(np.asarray(xs, dtype=np.uint32))
    out = np.zeros(2 * max(x.size, 1), np.uint64)
    rc = lib().orc_vertex_counts(g.n_u, g.n_v, eu.size, _p(eu, _u32p), _p(ev, _u32p),
                                 _p(sg, _i8p), side, x.size, _p(x, _u32p), _p(out, _u64p))
    if rc != 0:
        raise ValueError(f"orc_vertex_counts failed ({rc})")
    return [int(out[2 * i]) | (int(out[2 * i + 1]) << 64) for i in range(x.size)]


def anchor_detail(g, side: int, u: int, oriented: bool = True, cap: int = 4096):
    """Intermediate values of Algorithm 2 at anchor u: dict with the candidate
    set C and per-pair records (w1, w2, |T|, x_ss, x_sd, x_ds, x_dd)."""
    eu, ev, sg = _arrs(g)
    cand = np.zeros(cap, np.uint32)
    pairs = np.zeros(7 * cap, np.int64)
    nc = np.zeros(1, np.int64)
    npairs = np.zeros(1, np.int64)
    tot = np.zeros(2, np.uint64)
    rc = lib().orc_anchor_detail(g.n_u, g.n_v, eu.size, _p(eu, _u32p), _p(ev, _u32p), _p(sg, _i8p),
                                 side, u, int(oriented), cap, _p(cand, _u32p), _p(nc, _i64p),
                                 cap, _p(pairs, _i64p), _p(npairs, _i64p), _p(tot, _u64p))
    if rc != 0:
        raise ValueError("orc_anchor_detail failed")
    n = int(npairs[0])
    return {"candidates": [int(c) for c in cand[:int(nc[0])]],
            "pairs": [tuple(int(x) for x in pairs[7 * i:7 * i + 7]) for i in range(n)],
            "total": int(tot[0]) | (int(tot[1]) << 64)}


class _Edges:
    """A graph with an edge list of its own (the attributes the counts read)."""

    def __init__(self, n_u, n_v, eu, ev, sign):
        self.n_u, self.n_v = n_u, n_v
        self.eu = np.ascontiguousarray(eu, np.uint32)
        self.ev = np.ascontiguousarray(ev, np.uint32)
        self.sign = np.ascontiguousarray(sign, np.int8)


def count_through_edge(g, u: int, v: int, s: int, brute: bool = False, threads: int = 1) -> int:
    """Balanced (3,3)-bicliques that contain the edge (u, v) of sign s in g
    with that edge set to s (added or re-signed): by definition the count of
    that graph minus the count of g without the edge, both from the counts
    above (the definition itself with brute=True, else Algorithm 2). This is
    the change of the count when the edge is inserted with sign s, the
    quantity behind dynamic updates, which Section 6 names as the next
    direction. No arithmetic of its own: it rests on the two (pinned) counts
    it subtracts."""
    eu = np.asarray(g.eu, np.int64)
    ev = np.asarray(g.ev, np.int64)
    sg = np.asarray(g.sign, np.int8)
    keep = ~((eu == u) & (ev == v))
    without = _Edges(g.n_u, g.n_v, eu[keep], ev[keep], sg[keep])
    with_e = _Edges(g.n_u, g.n_v, np.append(eu[keep], u), np.append(ev[keep], v),
                    np.append(sg[keep], np.int8(s)))
    if brute:
        return count_bruteforce(with_e) - count_bruteforce(without)
    return count_bbvp(with_e, 0, threads=threads)["total"] - count_bbvp(without, 0, threads=threads)["total"]


def count_bbvp_p4(g, q: int, side: int = 0, threads: int = 1) -> dict:
    """count_bbvp_pk with p = 4 (merges of the L lists)."""
    return count_bbvp_pk(g, 4, q, side, threads)
