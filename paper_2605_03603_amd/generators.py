"""Seeded synthetic signed bipartite graphs.

This module only draws random graphs. It holds none of the counting
arithmetic, so both the CPU oracle tests and the GPU path may use it to
obtain the same inputs from the same seed.

A graph is returned as a :class:`SignedBipartite`: vertex counts ``n_u``,
``n_v`` and a COO edge list ``eu`` (uint32, < n_u), ``ev`` (uint32, < n_v),
``sign`` (int8, +1 or -1). Edges are distinct pairs (the paper's edge set is a
subset of U x V, Section 3) in no particular order.

Workload shapes (the paper's own datasets are not available; these stand in
for them):

* ER:       every (u, v) pair independently with probability p.
* Chung-Lu: expected degrees w_i proportional to i^(-1/(gamma-1)), scaled so
            that they sum to |E| and water-filled under the cap sqrt(|E|);
            edges are drawn endpoint-by-endpoint proportional to the weights
            and deduplicated until exactly |E| distinct pairs remain.
* signs:    i.i.d. +1 with a given probability (Section 5 gives 0.7 positive
            for the paper's synthetically signed datasets), or from hidden
            vertex labels l(u) l(v) with independent noise flips.
* planted:  k x k' complete blocks on disjoint random vertex sets; balanced
            blocks carry signs a(u) b(v) (vertex-switching of an all-positive
            block), random blocks carry i.i.d. uniform signs. A planted block
            replaces any background edge between its own vertices.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class SignedBipartite:
    n_u: int
    n_v: int
    eu: np.ndarray   # uint32 [m]
    ev: np.ndarray   # uint32 [m]
    sign: np.ndarray  # int8 [m], +1 / -1
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.eu.shape[0])

    def transpose(self) -> "SignedBipartite":
        return SignedBipartite(self.n_v, self.n_u, self.ev.copy(), self.eu.copy(),
                               self.sign.copy(), dict(self.meta))


def _finish(n_u, n_v, u, v, s, meta=None) -> SignedBipartite:
    return SignedBipartite(int(n_u), int(n_v), np.ascontiguousarray(u, dtype=np.uint32),
                           np.ascontiguousarray(v, dtype=np.uint32),
                           np.ascontiguousarray(s, dtype=np.int8), dict(meta or {}))


def iid_signs(rng: np.random.Generator, m: int, p_pos: float) -> np.ndarray:
    return np.where(rng.random(m) < p_pos, 1, -1).astype(np.int8)


# --------------------------------------------------------------------------- ER
def er_edges(rng: np.random.Generator, n_u: int, n_v: int, p: float) -> Tuple[np.ndarray, np.ndarray]:
    """Each of the n_u*n_v pairs independently with probability p."""
    total = n_u * n_v
    if total == 0 or p <= 0.0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if total <= (1 << 22):
        keys = np.flatnonzero(rng.random(total) < p)
    else:
        m = int(rng.binomial(total, p))
        keys = np.zeros(0, np.int64)
        while keys.size < m:
            extra = rng.integers(0, total, size=int((m - keys.size) * 1.05) + 16, dtype=np.int64)
            keys = np.unique(np.concatenate([keys, extra]))
        if keys.size > m:
            keys = rng.choice(keys, size=m, replace=False)
    keys = np.asarray(keys, dtype=np.int64)
    return keys // n_v, keys % n_v


# --------------------------------------------------------------------- Chung-Lu
def chung_lu_weights(n: int, gamma: float, total: float, cap: float) -> np.ndarray:
    """Expected degrees ~ i^(-1/(gamma-1)), summing to `total`, each <= cap."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    w *= total / w.sum()
    for _ in range(200):
        w = np.minimum(w, cap)
        s = w.sum()
        if abs(s - total) <= 1e-9 * total:
            break
        free = w < cap
        if not free.any():
            break
        w[free] *= (total - cap * (~free).sum()) / w[free].sum()
    return np.minimum(w, cap)


def chung_lu_edges(rng: np.random.Generator, n_u: int, n_v: int, m: int,
                   gamma_u: float, gamma_v: float) -> Tuple[np.ndarray, np.ndarray]:
    """Exactly m distinct pairs drawn endpoint-wise proportional to capped
    power-law weights; vertex ids are randomly permuted so that id and degree
    are unrelated."""
    cap = math.sqrt(m)
    pu = chung_lu_weights(n_u, gamma_u, m, cap)
    pv = chung_lu_weights(n_v, gamma_v, m, cap)
    cu = np.cumsum(pu); cu /= cu[-1]
    cv = np.cumsum(pv); cv /= cv[-1]
    perm_u = rng.permutation(n_u).astype(np.int64)
    perm_v = rng.permutation(n_v).astype(np.int64)
    keys = np.zeros(0, np.int64)
    while keys.size < m:
        need = m - keys.size
        k = need + need // 8 + 64
        a = np.searchsorted(cu, rng.random(k), side="right")
        b = np.searchsorted(cv, rng.random(k), side="right")
        np.minimum(a, n_u - 1, out=a)
        np.minimum(b, n_v - 1, out=b)
        new = perm_u[a] * n_v + perm_v[b]
        keys = np.unique(np.concatenate([keys, new]))
    if keys.size > m:
        keys = rng.choice(keys, size=m, replace=False)
    return keys // n_v, keys % n_v


# ---------------------------------------------------------------------- planted
def plant_blocks(rng: np.random.Generator, n_u: int, n_v: int,
                 u: np.ndarray, v: np.ndarray, s: np.ndarray,
                 blocks: List[Tuple[int, int, str]]):
    """Plant complete blocks on disjoint random vertex sets.

    blocks: list of (k_u, k_v, kind) with kind 'balanced' (signs a(u)b(v)) or
    'random' (i.i.d. uniform +-1). Returns new (u, v, s) and the block list
    [(U-vertices, V-vertices, kind)]."""
    if not blocks:
        return u, v, s, []
    tot_u = sum(b[0] for b in blocks)
    tot_v = sum(b[1] for b in blocks)
    assert tot_u <= n_u and tot_v <= n_v, "planted blocks do not fit"
    pu = rng.permutation(n_u)[:tot_u]
    pv = rng.permutation(n_v)[:tot_v]
    block_of_u = np.full(n_u, -1, np.int64)
    block_of_v = np.full(n_v, -1, np.int64)
    out = []
    bu, bv, bs = [], [], []
    iu = iv = 0
    for bi, (ku, kv, kind) in enumerate(blocks):
        us = pu[iu:iu + ku]; vs = pv[iv:iv + kv]
        iu += ku; iv += kv
        block_of_u[us] = bi
        block_of_v[vs] = bi
        gu, gv = np.meshgrid(us, vs, indexing="ij")
        if kind == "balanced":
            a = np.where(rng.random(ku) < 0.5, 1, -1)
            b = np.where(rng.random(kv) < 0.5, 1, -1)
            sg = np.outer(a, b)
        elif kind == "random":
            sg = np.where(rng.random((ku, kv)) < 0.5, 1, -1)
        else:
            raise ValueError(kind)
        bu.append(gu.ravel()); bv.append(gv.ravel()); bs.append(sg.ravel())
        out.append((us.copy(), vs.copy(), kind))
    u = np.asarray(u, np.int64); v = np.asarray(v, np.int64)
    keep = ~((block_of_u[u] >= 0) & (block_of_u[u] == block_of_v[v]))
    u = np.concatenate([u[keep]] + bu)
    v = np.concatenate([v[keep]] + bv)
    s = np.concatenate([np.asarray(s, np.int8)[keep]] + [x.astype(np.int8) for x in bs])
    return u, v, s, out


# ---------------------------------------------------------------------- configs
def config1(seed: int = 1) -> SignedBipartite:
    """ER 200 x 300, p = 0.05, 70% positive, plus 3 planted balanced 6x6 blocks."""
    rng = np.random.default_rng([1, seed])
    n_u, n_v = 200, 300
    u, v = er_edges(rng, n_u, n_v, 0.05)
    s = iid_signs(rng, u.size, 0.7)
    u, v, s, blocks = plant_blocks(rng, n_u, n_v, u, v, s, [(6, 6, "balanced")] * 3)
    return _finish(n_u, n_v, u, v, s, {"config": 1, "seed": seed, "blocks": blocks})


def config2(seed: int = 1, scale: float = 1.0) -> SignedBipartite:
    """Chung-Lu 100k x 50k, ~2M edges, gamma 2.1/2.1, 80% positive, 200
    balanced and 200 random-sign 12x12 planted blocks. `scale` < 1 shrinks
    every size proportionally (for quick tests)."""
    rng = np.random.default_rng([2, seed])
    n_u, n_v, m = int(100_000 * scale), int(50_000 * scale), int(2_000_000 * scale)
    nb = max(1, int(200 * scale))
    u, v = chung_lu_edges(rng, n_u, n_v, m, 2.1, 2.1)
    s = iid_signs(rng, u.size, 0.8)
    u, v, s, blocks = plant_blocks(rng, n_u, n_v, u, v, s,
                                   [(12, 12, "balanced")] * nb + [(12, 12, "random")] * nb)
    return _finish(n_u, n_v, u, v, s, {"config": 2, "seed": seed, "scale": scale,
                                       "blocks": blocks})


def config3(seed: int = 1, scale: float = 1.0) -> SignedBipartite:
    """Chung-Lu 2M x 500k, ~40M edges, gamma 1.9 on U and 2.3 on V. Signs are
    l(u) l(v) for hidden labels with P(l = -1) = 0.0323 on both sides, each
    flipped independently with probability 0.10 (85% positive overall). The
    labels are returned in meta['label_u'], meta['label_v']."""
    rng = np.random.default_rng([3, seed])
    n_u, n_v, m = int(2_000_000 * scale), int(500_000 * scale), int(40_000_000 * scale)
    u, v = chung_lu_edges(rng, n_u, n_v, m, 1.9, 2.3)
    pi = 0.0323
    lu = np.where(rng.random(n_u) < pi, -1, 1).astype(np.int8)
    lv = np.where(rng.random(n_v) < pi, -1, 1).astype(np.int8)
    flip = np.where(rng.random(u.size) < 0.10, -1, 1).astype(np.int8)
    s = (lu[u] * lv[v] * flip).astype(np.int8)
    return _finish(n_u, n_v, u, v, s, {"config": 3, "seed": seed, "scale": scale,
                                       "label_u": lu, "label_v": lv})


def config4_graph(rng: np.random.Generator) -> SignedBipartite:
    """One graph of the batched mix: N = |U|+|V| log-uniform on [50, 20000],
    |U| = round(f N) with f ~ U(0.3, 0.7), mean degree ~ U(8, 40), ER with
    p = min(0.5, |E| / (|U||V|)), 75% positive, 0..5 planted balanced 5x5."""
    n = int(round(math.exp(rng.uniform(math.log(50), math.log(20000)))))
    f = rng.uniform(0.3, 0.7)
    n_u = min(max(int(round(f * n)), 1), n - 1)
    n_v = n - n_u
    dbar = rng.uniform(8, 40)
    p = min(0.5, dbar * n / 2.0 / (n_u * n_v))
    u, v = er_edges(rng, n_u, n_v, p)
    s = iid_signs(rng, u.size, 0.75)
    k = int(rng.integers(0, 6))
    k = min(k, n_u // 5, n_v // 5)
    u, v, s, blocks = plant_blocks(rng, n_u, n_v, u, v, s, [(5, 5, "balanced")] * k)
    return _finish(n_u, n_v, u, v, s, {"config": 4, "blocks": blocks})


def config4(seed: int = 1, n_graphs: int = 8192) -> List[SignedBipartite]:
    rng = np.random.default_rng([4, seed])
    return [config4_graph(rng) for _ in range(n_graphs)]


def serve_stream(seed: int, n_requests: int, qps: float, large_pool: List[SignedBipartite],
                 p_large: float = 0.02) -> List[Tuple[float, SignedBipartite]]:
    """Poisson arrivals at `qps`; each request is a batched-mix graph, or with
    probability p_large one graph of `large_pool` (config-2 shaped)."""
    rng = np.random.default_rng([5, seed])
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / qps)
        if large_pool and rng.random() < p_large:
            g = large_pool[int(rng.integers(0, len(large_pool)))]
        else:
            g = config4_graph(rng)
        out.append((t, g))
    return out


# ------------------------------------------------------------------ tiny graphs
def tiny_random(rng: np.random.Generator, max_u: int = 8, max_v: int = 8,
                density: Optional[float] = None, p_pos: Optional[float] = None) -> SignedBipartite:
    n_u = int(rng.integers(0, max_u + 1))
    n_v = int(rng.integers(0, max_v + 1))
    d = float(rng.choice([0.2, 0.4, 0.6, 0.8, 1.0])) if density is None else density
    pp = float(rng.choice([0.0, 0.3, 0.5, 0.7, 1.0])) if p_pos is None else p_pos
    u, v = er_edges(rng, n_u, n_v, d) if n_u * n_v else (np.zeros(0), np.zeros(0))
    s = iid_signs(rng, len(u), pp)
    return _finish(n_u, n_v, u, v, s)


def from_rows(rows: List[str]) -> SignedBipartite:
    """Build a graph from strings of '+', '-', '.' (row = U vertex, column = V
    vertex, '.' = no edge)."""
    n_u = len(rows)
    n_v = len(rows[0]) if rows else 0
    u, v, s = [], [], []
    for i, r in enumerate(rows):
        assert len(r) == n_v
        for j, c in enumerate(r):
            if c in "+-":
                u.append(i); v.append(j); s.append(1 if c == "+" else -1)
    return _finish(n_u, n_v, np.array(u, np.int64), np.array(v, np.int64), np.array(s, np.int8))


def concat(graphs: List[SignedBipartite]):
    """Concatenate COO lists: returns (n_u[], n_v[], edge_offsets[n+1], eu, ev, sign)."""
    n_u = np.array([g.n_u for g in graphs], np.uint32)
    n_v = np.array([g.n_v for g in graphs], np.uint32)
    off = np.zeros(len(graphs) + 1, np.uint64)
    off[1:] = np.cumsum([g.m for g in graphs])
    eu = np.concatenate([g.eu for g in graphs]) if graphs else np.zeros(0, np.uint32)
    ev = np.concatenate([g.ev for g in graphs]) if graphs else np.zeros(0, np.uint32)
    sg = np.concatenate([g.sign for g in graphs]) if graphs else np.zeros(0, np.int8)
    return n_u, n_v, off, eu.astype(np.uint32), ev.astype(np.uint32), sg.astype(np.int8)
