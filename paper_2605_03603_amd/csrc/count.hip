// count.hip -- the counting kernels: signed pair table, unit planning and
// triplet intersection, for balanced (3,3)-bicliques.
//
// For an anchor u1 (the lowest-priority vertex of a triple, Definition 4.1
// and the orientation rho(w) > rho(u) of Algorithm 2) and a common neighbour v
// of u1, u2, u3, the wedge type of Section 4.1 is (c_2, c_3) with
// c_i = s(u1,v) s(u_i,v). Lemma 1 (and its converse: if every v has the same
// type then every butterfly of the biclique is balanced) gives, per triple,
//     sum over the 4 types of C(n_type, 3).
// With M_w^c = { v in N(u1) n N(w) : s(u1,v) s(w,v) = c } for c in {+,-}:
//     n_(c2,c3) = | M_u2^c2  n  M_u3^c3 |,
// so the triple's contribution is the sum over the 4 sign choices of
// C(|M_u2^c2 n M_u3^c3|, 3). The kernels therefore work on "virtual
// candidates" (w, c): a class set M_w^c with at least 3 members (a smaller
// one cannot reach C(.,3) > 0 -- this is the pair prune of Algorithm 2 split
// by sign class). Two virtual candidates of the same w never share a member
// (M_w^+ and M_w^- are disjoint), so every unordered pair of virtual
// candidates may be paired without excluding same-w pairs:
//     contribution(u1) = sum over pairs {x, y} of C(|M_x n M_y|, 3).
// M_x is a bitmask over the positions of N(u1); |M_x n M_y| is an AND and a
// popcount per 32-bit word.
//
// k_pair (the signed pair table: Algorithm 2's cnt map split by sign class)
//   one workgroup per anchor: walk the higher-priority part of each
//   neighbour's list (located by s_suf, no search), count (same,
//   different) per partner in an LDS hash table, keep the classes with >= 3,
//   walk again to set the mask bits, emit masks. Three tiers: 4096- and
//   16384-slot LDS tables, then global-memory tables for anchors that
//   overflow them.
// k_plan_* cut every anchor's lower-triangular pair matrix into work units
//   (64 rows x up to a few hundred columns), without atomics.
// k_triplet (Algorithm 2's loop over pairs A of C, T = intersection and the
//   type histogram): one wave per unit; row masks in VGPRs, column masks by
//   scalar loads (wave-uniform addresses), C(n,3) from an LDS table; totals
//   stay in registers until the wave finishes or changes graph.
//
// Work queues are split into 8 slices, one per XCD (workgroup i runs on XCD
// i % 8): a workgroup drains its own slice first, so consecutive anchors
// and the units of one anchor share an L2, then steals from the others.
#include "bbc_count.h"
#include <type_traits>

namespace bbc {

namespace {

#define BBC_CONST __attribute__((address_space(4)))

template <typename T>
__device__ __forceinline__ const BBC_CONST T *as_const(const T *p)
{
    return (const BBC_CONST T *)p;
}

__device__ __forceinline__ Unit load_unit(const Unit *p)
{
    const BBC_CONST uint32_t *q = as_const((const uint32_t *)p);
    Unit u;
    u.anchor = q[0]; u.rb = q[1]; u.c0 = q[2]; u.c1 = q[3];
    return u;
}

__device__ __forceinline__ AnchorRec load_anchor(const AnchorRec *p)
{
    const BBC_CONST uint32_t *q = as_const((const uint32_t *)p);
    AnchorRec a;
    a.rank = q[0]; a.k = q[1]; a.w32 = q[2]; a.graph = q[3];
    a.mask_off = (uint64_t)q[4] | ((uint64_t)q[5] << 32);
    a.cand_off = (uint64_t)q[6] | ((uint64_t)q[7] << 32);
    return a;
}

constexpr uint32_t kEmpty = 0xffffffffu;
constexpr uint32_t kC3Max = 512;       // C(n,3) table covers masks of up to 16 words
constexpr uint32_t kRegW = 16;         // widest mask kept in registers per row
constexpr uint32_t kWideCols = 64;     // unit width (columns) for wider masks
constexpr uint32_t kMfmaMaxW = 16;     // widest mask counted with the rows held in registers
// Output is reserved in chunks (PairArgs::mask_chunk and cand_chunk mask words
// and candidates per workgroup, wv_mask_chunk and wv_cand_chunk per wave of the
// per-wave tier), sized by the host to the set's edge count so that a small
// graph's demand stays small; anchor records 16 at a time.
constexpr uint32_t kRecChunk = 16;
constexpr int kUnroll = 4;              // independent neighbour-list loads per lane
// rank-window tier (k_pair_window): its threads, widest partner window (bytes
// of its table), LDS words, and the wedge count from which tiers A and B hand
// an anchor to it without counting it themselves
constexpr int kRThreads = 1024;
constexpr uint32_t kRWin = 1u << 17;
constexpr uint32_t kRWords = 38912;
constexpr uint32_t kRMinWedges = 16384;
constexpr int kListR = 4;               // index of its anchor list (defer[], n_list[])

__device__ __forceinline__ uint32_t hash_slot(uint32_t x, int log2h)
{
    return (x * 0x9E3779B1u) >> (32 - log2h);
}

// Insert-or-add into an open-addressing table (linear probing). Returns true
// when this call inserted a new key (the caller counts new keys per wave);
// sets *over when the probe run gets too long.
__device__ __forceinline__ bool hash_add(uint32_t *keys, uint32_t *vals, uint32_t H, int log2h,
                                         uint32_t x, uint32_t inc, volatile uint32_t *over)
{
    uint32_t h = hash_slot(x, log2h);
    // a probe run this long means the table is (nearly) full: the anchor
    // moves to a bigger tier
    const uint32_t max_probe = H < 256 ? H : 256;
    for (uint32_t probe = 0; probe < max_probe; probe++) {
        uint32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
        if (k == x) { atomicAdd(&vals[h], inc); return false; }
        if (k == kEmpty) {
            uint32_t old = atomicCAS(&keys[h], kEmpty, x);
            if (old == kEmpty) { atomicAdd(&vals[h], inc); return true; }
            if (old == x) { atomicAdd(&vals[h], inc); return false; }
        }
        h = (h + 1) & (H - 1);
    }
    *over = 1;
    return false;
}

// Columns per work unit for masks of w32 words.
__host__ __device__ __forceinline__ uint32_t unit_cols(uint32_t w32, uint32_t base)
{
    if (w32 > kRegW) return kWideCols;
    uint32_t c = base / w32;
    c = c < 32 ? 32 : c;
    return (c + 15) & ~15u;   // whole 16-column matrix-core tiles
}

// Whether every partner of anchor r (ranked in (r, end of r's graph)) lies in
// a window the rank-window tier can index.
__device__ __forceinline__ bool window_fits(const CsrView &g, uint32_t r)
{
    const GraphDesc &gd = g.desc[g.s_graph[r]];
    return gd.s_base + gd.n_s - r - 1 <= kRWin;
}

__device__ __forceinline__ uint32_t slice_lo(uint32_t n, uint32_t s)
{
    return (uint32_t)(((uint64_t)n * s) / kXcd);
}

// Next chunk [*lo, *hi) of a work range [0, n) split into kXcd slices; the
// caller starts at its home slice and moves on when a slice is drained.
// Returns false when every slice is drained.
__device__ __forceinline__ bool queue_take(Cursor *cur, uint32_t n, uint32_t chunk,
                                           uint32_t *slice, uint32_t *tried, uint32_t *lo,
                                           uint32_t *hi)
{
    while (*tried < kXcd) {
        const uint32_t s = *slice;
        const uint32_t a = slice_lo(n, s), b = slice_lo(n, s + 1);
        const uint32_t t = atomicAdd(&cur[s].v, chunk);
        if (t < b - a) {
            *lo = a + t;
            *hi = min(a + t + chunk, b);
            return true;
        }
        *slice = (s + 1) % kXcd;
        (*tried)++;
    }
    return false;
}

// Units of one anchor record: row blocks of 64 rows, each cut into column
// ranges of unit_cols() columns of the lower triangle.
__device__ __forceinline__ uint32_t anchor_units(uint32_t k, uint32_t w32, uint32_t base)
{
    if (k < 2) return 0;
    const uint32_t CH = unit_cols(w32, base);
    const uint32_t nb = (k + kWave - 1) / kWave;
    uint32_t tot = 0;
    for (uint32_t b = 0; b < nb; b++) {
        const uint32_t ncols = min(kWave * (b + 1), k) - 1;
        tot += (ncols + CH - 1) / CH;
    }
    return tot;
}

struct PairShared {
    uint32_t item, over, used, nv, skip, wedges;
    uint32_t qlo, qhi, qslice, qtried;
    uint32_t aidx, arec_end;
    unsigned long long top1, top2;               // (suffix length << 32) | position
    unsigned long long moff, mres_end, coff, cres_end;
    unsigned long long bm, bc;                   // own reservations of large outputs
    uint32_t big_m, big_c;
    unsigned long long vm, vm_end, vc, vc_end;   // chunk use as if room were unlimited
    unsigned long long need_m, need_c, need_r, need_u;   // this workgroup's demand
};

// Storage of one tier. `region` (2H words) holds the counting table (keys,
// vals) while partners are counted; once the candidate classes are known it
// is reused for a compact table of the selected partners (ckeys, cidx: 2HC
// words) followed by the mask staging area (maskw words).
struct PairMem {
    uint32_t *region;
    uint32_t H;
    int log2h;
    uint32_t HC;
    int log2hc;
    uint32_t maskw;
    uint32_t *pst, *pln;   // per position: suffix start, suffix length | sign << 31
    uint32_t maxd;
    uint32_t *vc;          // per virtual candidate: partner rank | class << 31
    uint32_t kmax;
};

// Increment an existing key; absent keys are ignored.
__device__ __forceinline__ void hash_inc(const uint32_t *keys, uint32_t *vals, uint32_t H,
                                         int log2h, uint32_t x, uint32_t inc)
{
    uint32_t h = hash_slot(x, log2h);
    for (uint32_t probe = 0; probe < H; probe++) {
        const uint32_t k = keys[h];
        if (k == x) { atomicAdd(&vals[h], inc); return; }
        if (k == kEmpty) return;
        h = (h + 1) & (H - 1);
    }
}

// Packed counting slots (graphs with fewer than 2^24 - 1 anchor-side
// vertices): one 32-bit word per partner, key in bits 0..23, then for each
// sign class a 3-bit thermometer (bits 24..26 same, 27..29 different): hit i
// (i = 1, 2, 3) sets bit i-1 of the class, further hits change nothing.
// Selection only needs "at least 3", so the table holds twice the partners
// of the (key, count) layout in the same memory.
constexpr uint32_t kKeyMask = 0xffffffu;

// Visit the wedges of the anchor's positions in [p0, p1): the ordinary
// positions one wave per position, the two longest suffixes spread over the
// whole workgroup. f(e2, pos, sg) receives kUnroll wedges per lane at once
// (entry, position, sign of (anchor, v); entry kEmpty for an idle slot), so
// that it can issue their first hash probes together. The loads are clamped
// to valid entries and all in flight together.
template <int THREADS, typename F>
__device__ __forceinline__ void walk_positions(const CsrView &g, const PairMem &m, uint32_t d,
                                               uint32_t t1, uint32_t t2, bool ordinary,
                                               bool top, F &&f, uint32_t p0 = 0,
                                               uint32_t p1 = 0xffffffffu)
{
    constexpr int NW = THREADS / kWave;
    const int tid = threadIdx.x, lane = __lane_id(), wv = tid / kWave;
    if (p1 > d) p1 = d;
    uint32_t e2[kUnroll], pp[kUnroll], sg[kUnroll];
    if (ordinary) {
        // The suffixes are cut into pieces of kPiece wedges, dealt round-robin
        // to the waves by their global index; each wave finds its pieces from
        // a prefix sum of piece counts over 64 positions at a time.
        constexpr uint32_t kPiece = kWave * kUnroll;
        uint32_t cum_base = 0;
        for (uint32_t c0 = p0; c0 < p1; c0 += kWave) {
            const uint32_t p = c0 + lane;
            uint32_t len = 0, st = 0, ln = 0;
            if (p < p1 && p != t1 && p != t2) {
                ln = m.pln[p];
                len = ln & 0x7fffffffu;
                st = m.pst[p];
            }
            const uint32_t np = (len + kPiece - 1) / kPiece;
            const uint32_t incl = wave_incl_scan(np);
            const uint32_t cum = cum_base + incl - np;          // first piece of position p
            const uint32_t first = cum + (uint32_t)((wv + NW - (int)(cum % NW)) % NW);
            uint64_t todo = ballot64(first < cum + np);
            while (todo) {
                const uint32_t l = (uint32_t)__builtin_ctzll(todo);
                todo &= todo - 1;
                const uint32_t pl = c0 + l;
                const uint32_t stl = __shfl(st, l, kWave), lenl = __shfl(len, l, kWave);
                const uint32_t sgl = __shfl(ln, l, kWave) >> 31;
                const uint32_t cuml = __shfl(cum, l, kWave), endl = cuml + __shfl(np, l, kWave);
                for (uint32_t q = __shfl(first, l, kWave); q < endl; q += NW) {
                    const uint32_t j0 = (q - cuml) * kPiece;
#pragma unroll
                    for (int u = 0; u < kUnroll; u++) {
                        const uint32_t j = j0 + u * kWave + lane;
                        const uint32_t e = g.o_adj[stl + min(j, lenl - 1)];
                        e2[u] = j < lenl ? e : kEmpty;
                        pp[u] = pl;
                        sg[u] = sgl;
                    }
                    f(e2, pp, sg);
                }
            }
            cum_base += __shfl(incl, kWave - 1, kWave);
        }
    }
    if (top) {
        const uint32_t l1 = (t1 >= p0 && t1 < p1) ? (m.pln[t1] & 0x7fffffffu) : 0;
        const uint32_t l2 = (t2 >= p0 && t2 < p1) ? (m.pln[t2] & 0x7fffffffu) : 0;
        const uint32_t tot = l1 + l2;
        const uint32_t s1 = l1 ? m.pst[t1] : 0, s2 = l2 ? m.pst[t2] : 0;
        const uint32_t g1 = l1 ? m.pln[t1] >> 31 : 0, g2 = l2 ? m.pln[t2] >> 31 : 0;
        for (uint32_t j0 = 0; j0 < tot; j0 += THREADS * kUnroll) {
#pragma unroll
            for (int u = 0; u < kUnroll; u++) {
                const uint32_t j = j0 + u * THREADS + tid;
                const uint32_t jc = min(j, tot - 1);
                const bool first = jc < l1;
                const uint32_t e = g.o_adj[first ? s1 + jc : s2 + (jc - l1)];
                e2[u] = j < tot ? e : kEmpty;
                pp[u] = first ? t1 : t2;
                sg[u] = first ? g1 : g2;
            }
            f(e2, pp, sg);
        }
    }
}

// Thermometer update of one class in a packed slot whose value was seen as
// `cur`: set the lowest bit of the class not yet set (a concurrent hit that
// took it moves this one to the next bit). b0 is the class's first bit.
__device__ __forceinline__ void therm_from(uint32_t *slot, uint32_t cur, uint32_t b0)
{
    uint32_t bit = b0;
#pragma unroll
    for (int i = 0; i < 3; i++, bit <<= 1) {
        if (cur & bit) continue;
        const uint32_t o2 = atomicOr(slot, bit);
        if (!(o2 & bit)) return;
        cur = o2;
    }
}

// Probe runs continued after a first probe at slot h that met another key.
__device__ __forceinline__ bool phash_add_from(uint32_t *slots, uint32_t H, uint32_t h, uint32_t x,
                                               uint32_t b0, volatile uint32_t *over)
{
    const uint32_t max_probe = H < 256 ? H : 256;
    for (uint32_t probe = 1; probe < max_probe; probe++) {
        h = (h + 1) & (H - 1);
        uint32_t v = __atomic_load_n(&slots[h], __ATOMIC_RELAXED);
        if (v == kEmpty) {
            const uint32_t old = atomicCAS(&slots[h], kEmpty, x | b0);
            if (old == kEmpty) return true;
            v = old;
        }
        if ((v & kKeyMask) == x) { therm_from(&slots[h], v, b0); return false; }
    }
    *over = 1;
    return false;
}

__device__ __forceinline__ void phash_inc_from(uint32_t *slots, uint32_t H, uint32_t h, uint32_t x,
                                               uint32_t b0)
{
    for (uint32_t probe = 1; probe < H; probe++) {
        h = (h + 1) & (H - 1);
        const uint32_t v = __atomic_load_n(&slots[h], __ATOMIC_RELAXED);
        if (v == kEmpty) return;
        if ((v & kKeyMask) == x) { therm_from(&slots[h], v, b0); return; }
    }
}

__device__ __forceinline__ uint32_t compact_find_from(const uint32_t *ckeys, const uint32_t *cidx,
                                                      uint32_t HC, uint32_t h, uint32_t x)
{
    for (uint32_t probe = 1; probe < HC; probe++) {
        h = (h + 1) & (HC - 1);
        const uint32_t k = ckeys[h];
        if (k == x) return cidx[h];
        if (k == kEmpty) return 0;
    }
    return 0;
}

// The per-anchor procedure shared by all tiers (LDS storage for tiers A and
// B, global memory for tier C).
template <int THREADS, bool PACKED>
__device__ __forceinline__ void pair_loop(const PairArgs &P, const PairMem &m, PairShared &sh)
{
    const int tid = threadIdx.x, lane = __lane_id();
    const CsrView &g = P.g;
    Counters *C = P.ws.ctr;
    uint32_t *keys = m.region, *vals = m.region + m.H;
    uint32_t *ckeys = m.region, *cidx = m.region + m.HC;
    uint32_t *mstage = m.region + 2 * m.HC;
    const uint32_t H = m.H;
    // counting slots: H (key, counts) pairs, or 2H packed words
    const uint32_t HS = PACKED ? 2 * m.H : m.H;
    const int log2hs = PACKED ? m.log2h + 1 : m.log2h;
    const uint32_t limit = HS - HS / 4;
    uint64_t my_wedges = 0;

    // tier t (1..4) takes the anchors listed for it and hands the ones it
    // cannot hold to tier t + 1
    const uint32_t n_items =
        (uint32_t)min((uint64_t)__atomic_load_n(&C->n_list[P.tier - 1], __ATOMIC_RELAXED),
                      P.ws.cap_defer);
    if (n_items == 0) return;
    const uint32_t *list = P.ws.defer[P.tier - 1];
    uint32_t *next_list = P.tier < 4 ? P.ws.defer[P.tier] : nullptr;

    auto clear_region = [&]() {
        if (PACKED) {
            for (uint32_t i = tid; i < 2 * H; i += THREADS) m.region[i] = kEmpty;
        } else {
            for (uint32_t i = tid; i < H; i += THREADS) { keys[i] = kEmpty; vals[i] = 0; }
        }
    };
    clear_region();
    if (tid == 0) {
        sh.qlo = sh.qhi = 0; sh.qslice = blockIdx.x % kXcd; sh.qtried = 0;
        sh.moff = sh.mres_end = 0; sh.coff = sh.cres_end = 0;
        sh.aidx = sh.arec_end = 0;
        sh.need_m = sh.need_c = sh.need_r = sh.need_u = 0;
        sh.vm = sh.vm_end = sh.vc = sh.vc_end = 0;
    }

    // tier B hands anchors whose partner window fits to the rank-window tier,
    // the others to tier C
    auto defer_anchor = [&](uint32_t r) {
        if (next_list) {
            const int li = (P.tier == 2 && !(P.flags & kPairNoWindow) && window_fits(g, r)) ? kListR
                                                                                          : P.tier;
            uint32_t t = atomicAdd(&C->n_list[li], 1u);
            if (t < P.ws.cap_defer) P.ws.defer[li][t] = r; else atomicOr(&C->over_cap, 1u);
        } else {
            atomicOr(&C->over_cap, 4u);
        }
    };

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            if (sh.qlo >= sh.qhi) {
                uint32_t lo = 0, hi = 0, s = sh.qslice, tr = sh.qtried;
                if (!queue_take(C->q_pair[P.tier], n_items, 1, &s, &tr, &lo, &hi)) lo = hi = n_items;
                sh.qslice = s; sh.qtried = tr; sh.qlo = lo; sh.qhi = hi;
            }
            sh.item = sh.qlo < sh.qhi ? sh.qlo++ : n_items;
            sh.over = 0; sh.used = 0; sh.nv = 0; sh.skip = 0; sh.wedges = 0;
            sh.top1 = 0; sh.top2 = 0;
        }
        __syncthreads();
        const uint32_t item = sh.item;
        if (item >= n_items) break;
        // the list from its end: the anchors deferred last (the later ranks of
        // each slice of the previous tier) start first
        const uint32_t r = list[n_items - 1 - item];
        const uint64_t s0 = g.s_off[r];
        const uint32_t d = (uint32_t)(g.s_off[r + 1] - s0);
        if (d < 3) continue;
        if (d > m.maxd) {
            if (tid == 0) defer_anchor(r);
            continue;
        }
        // phase 0: the part of each neighbour's list ranked above the anchor,
        // and the position with the longest such suffix
        {
            // per-wave sum and maximum, then one LDS atomic per wave
            uint32_t wsum = 0;
            uint64_t wtop = 0;
            for (uint32_t p = tid; p < d; p += THREADS) {
                const uint2 sf = g.s_suf[s0 + p];
                const uint32_t len = sf.y & 0x7fffffffu;
                m.pst[p] = sf.x;
                m.pln[p] = sf.y;
                wsum += len;
                const uint64_t key = len ? ((uint64_t)len << 32) | p : 0;
                wtop = key > wtop ? key : wtop;
            }
            wsum = wave_sum<uint32_t>(wsum);
            wtop = wave_max64(wtop);
            if (lane == 0 && wsum) {
                atomicAdd(&sh.wedges, wsum);
                atomicMax(&sh.top1, (unsigned long long)wtop);
            }
        }
        __syncthreads();
        if (sh.wedges < 6) continue;   // fewer than 2 classes of 3 are impossible
        if (P.tier <= 2 && !(P.flags & kPairNoWindow) && sh.wedges >= kRMinWedges &&
            window_fits(g, r)) {
            // heavy anchor near the top of the order: the rank-window tier
            if (tid == 0) {
                uint32_t t = atomicAdd(&C->n_list[kListR], 1u);
                if (t < P.ws.cap_defer) P.ws.defer[kListR][t] = r; else atomicOr(&C->over_cap, 1u);
            }
            continue;
        }
        const uint32_t t1 = sh.top1 ? (uint32_t)sh.top1 : kEmpty;
        {
            uint64_t wtop = 0;
            for (uint32_t p = tid; p < d; p += THREADS) {
                const uint32_t len = m.pln[p] & 0x7fffffffu;
                const uint64_t key = (len && p != t1) ? ((uint64_t)len << 32) | p : 0;
                wtop = key > wtop ? key : wtop;
            }
            wtop = wave_max64(wtop);
            if (lane == 0 && wtop) atomicMax(&sh.top2, (unsigned long long)wtop);
        }
        __syncthreads();
        const uint32_t t2 = sh.top2 ? (uint32_t)sh.top2 : kEmpty;
        // phase 1: (same, different) counts per higher-priority partner. A
        // class needs 3 hits at distinct positions, so every partner that can
        // qualify is hit at a position other than the two longest suffixes:
        // only those positions insert keys, the two longest only add to them.
        {
            uint32_t fresh = 0;
            walk_positions<THREADS>(g, m, d, t1, t2, true, false,
                                    [&](const uint32_t (&e2)[kUnroll], const uint32_t (&)[kUnroll],
                                        const uint32_t (&sg)[kUnroll]) {
                                        if (PACKED) {
                                            // first probes together: a CAS that inserts or
                                            // returns the slot's value
                                            uint32_t hs[kUnroll], old[kUnroll];
#pragma unroll
                                            for (int u = 0; u < kUnroll; u++) {
                                                const uint32_t b0 = 1u << (24 + 3 * ((e2[u] & 1u) ^ sg[u]));
                                                hs[u] = hash_slot(e2[u] >> 1, log2hs);
                                                old[u] = e2[u] != kEmpty
                                                             ? atomicCAS(&m.region[hs[u]], kEmpty, (e2[u] >> 1) | b0)
                                                             : 0u;
                                            }
#pragma unroll
                                            for (int u = 0; u < kUnroll; u++) {
                                                if (e2[u] == kEmpty) continue;
                                                my_wedges++;
                                                const uint32_t x = e2[u] >> 1;
                                                const uint32_t b0 = 1u << (24 + 3 * ((e2[u] & 1u) ^ sg[u]));
                                                if (old[u] == kEmpty) fresh++;
                                                else if ((old[u] & kKeyMask) == x) therm_from(&m.region[hs[u]], old[u], b0);
                                                else fresh += phash_add_from(m.region, HS, hs[u], x, b0, &sh.over);
                                            }
                                        } else {
#pragma unroll
                                            for (int u = 0; u < kUnroll; u++) {
                                                if (e2[u] == kEmpty) continue;
                                                my_wedges++;
                                                const uint32_t cls = (e2[u] & 1u) ^ sg[u];
                                                fresh += hash_add(keys, vals, H, m.log2h, e2[u] >> 1,
                                                                  cls ? 0x10000u : 1u, &sh.over);
                                            }
                                        }
                                    });
            const uint32_t nf = wave_sum<uint32_t>(fresh);
            if (lane == 0 && nf && atomicAdd(&sh.used, nf) + nf > limit) sh.over = 1;
        }
        __syncthreads();
        bool defer = sh.over != 0;
        if (!defer) {
            walk_positions<THREADS>(g, m, d, t1, t2, false, true,
                                    [&](const uint32_t (&e2)[kUnroll], const uint32_t (&)[kUnroll],
                                        const uint32_t (&sg)[kUnroll]) {
                                        if (PACKED) {
                                            uint32_t hs[kUnroll], v[kUnroll];
#pragma unroll
                                            for (int u = 0; u < kUnroll; u++) {
                                                hs[u] = hash_slot(e2[u] >> 1, log2hs);
                                                v[u] = e2[u] != kEmpty ? __atomic_load_n(&m.region[hs[u]], __ATOMIC_RELAXED)
                                                                       : kEmpty;
                                            }
#pragma unroll
                                            for (int u = 0; u < kUnroll; u++) {
                                                if (e2[u] == kEmpty) continue;
                                                my_wedges++;
                                                if (v[u] == kEmpty) continue;
                                                const uint32_t x = e2[u] >> 1;
                                                const uint32_t b0 = 1u << (24 + 3 * ((e2[u] & 1u) ^ sg[u]));
                                                if ((v[u] & kKeyMask) == x) therm_from(&m.region[hs[u]], v[u], b0);
                                                else phash_inc_from(m.region, HS, hs[u], x, b0);
                                            }
                                        } else {
#pragma unroll
                                            for (int u = 0; u < kUnroll; u++) {
                                                if (e2[u] == kEmpty) continue;
                                                my_wedges++;
                                                const uint32_t cls = (e2[u] & 1u) ^ sg[u];
                                                hash_inc(keys, vals, H, m.log2h, e2[u] >> 1, cls ? 0x10000u : 1u);
                                            }
                                        }
                                    });
            __syncthreads();
            // phase 2: classes with >= 3 members become virtual candidates
            // (packed slots are read four at a time)
            auto select = [&](uint32_t k, bool same3, bool diff3) {
                if (same3) {
                    const uint32_t t = atomicAdd(&sh.nv, 1u);
                    if (t < m.kmax) m.vc[t] = k;
                }
                if (diff3) {
                    const uint32_t t = atomicAdd(&sh.nv, 1u);
                    if (t < m.kmax) m.vc[t] = k | 0x80000000u;
                }
            };
            if (PACKED) {
                // count this thread's classes, reserve once per wave, then
                // read the same slots again and write them out
                const uint4 *R4 = reinterpret_cast<const uint4 *>(m.region);
                uint32_t cnt = 0;
                for (uint32_t q = tid; q < HS / 4; q += THREADS) {
                    const uint4 v4 = R4[q];
                    const uint32_t vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        if (vv[e] != kEmpty) cnt += ((vv[e] >> 26) & 1u) + ((vv[e] >> 29) & 1u);
                }
                const uint32_t incl = wave_incl_scan(cnt);
                uint32_t base = 0;
                if (lane == kWave - 1 && incl) base = atomicAdd(&sh.nv, incl);
                uint32_t t = __shfl(base, kWave - 1, kWave) + incl - cnt;
                for (uint32_t q = tid; cnt && q < HS / 4; q += THREADS) {
                    const uint4 v4 = R4[q];
                    const uint32_t vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        if (vv[e] == kEmpty) continue;
                        const uint32_t k = vv[e] & kKeyMask;
                        if ((vv[e] >> 26) & 1u) { if (t < m.kmax) m.vc[t] = k; t++; }
                        if ((vv[e] >> 29) & 1u) { if (t < m.kmax) m.vc[t] = k | 0x80000000u; t++; }
                    }
                }
            }
            for (uint32_t slot = tid; !PACKED && slot < HS; slot += THREADS) {
                uint32_t k;
                bool same3, diff3;
                {
                    k = keys[slot];
                    if (k == kEmpty) continue;
                    const uint32_t v = vals[slot];
                    same3 = (v & 0xffffu) >= 3;
                    diff3 = (v >> 16) >= 3;
                }
                select(k, same3, diff3);
            }
            __syncthreads();
            defer = sh.nv > m.kmax;
        }
        if (defer) {
            if (tid == 0) defer_anchor(r);
            clear_region();
            continue;
        }
        const uint32_t k = sh.nv;
        if (k < 2) {
            clear_region();
            continue;
        }
        // compact table: partner -> (same index + 1) | (different index + 1) << 16
        for (uint32_t i = tid; i < 2 * m.HC; i += THREADS) m.region[i] = i < m.HC ? kEmpty : 0u;
        __syncthreads();
        for (uint32_t t = tid; t < k; t += THREADS) {
            const uint32_t x = m.vc[t] & 0x7fffffffu;
            const uint32_t bits = (t + 1) << ((m.vc[t] >> 31) ? 16 : 0);
            uint32_t h = hash_slot(x, m.log2hc);
            for (uint32_t probe = 0; probe < m.HC; probe++) {
                const uint32_t old = atomicCAS(&ckeys[h], kEmpty, x);
                if (old == kEmpty || old == x) { atomicOr(&cidx[h], bits); break; }
                h = (h + 1) & (m.HC - 1);
            }
        }
        const uint32_t W = (d + 31) >> 5;
        const uint64_t words = (uint64_t)k * W;
        if (tid == 0) {
            // workgroup-local bump reservations (few global atomics)
            // demand: what the reservations below consume with unlimited room
            sh.big_m = words > P.mask_chunk / 4;
            sh.big_c = k > P.cand_chunk / 4;
            if (sh.big_m) {
                sh.need_m += words;
            } else {
                if (sh.vm + words > sh.vm_end) { sh.need_m += P.mask_chunk; sh.vm = 0; sh.vm_end = P.mask_chunk; }
                sh.vm += words;
            }
            if (sh.big_c) {
                sh.need_c += k;
            } else {
                if (sh.vc + k > sh.vc_end) { sh.need_c += P.cand_chunk; sh.vc = 0; sh.vc_end = P.cand_chunk; }
                sh.vc += k;
            }
            sh.need_r += 1;
            sh.need_u += anchor_units(k, W, P.chunk_base);
            bool bad = (__atomic_load_n(&C->over_cap, __ATOMIC_RELAXED) & 2u) != 0;
            if (!bad) {
                // large outputs get a reservation of their own; small ones come
                // from the workgroup's chunk, whose abandoned tail counts as demand
                if (sh.big_m) {
                    uint64_t o = atomicAdd(&C->mask_cursor, (unsigned long long)words);
                    sh.bm = o;
                    if (o + words > P.ws.cap_mask_words) bad = true;
                } else if (sh.moff + words > sh.mres_end) {
                    uint64_t o = atomicAdd(&C->mask_cursor, (unsigned long long)P.mask_chunk);
                    sh.moff = o; sh.mres_end = o + P.mask_chunk;
                    if (o + P.mask_chunk > P.ws.cap_mask_words) bad = true;
                }
                if (sh.big_c) {
                    uint64_t o = atomicAdd(&C->cand_cursor, (unsigned long long)k);
                    sh.bc = o;
                    if (o + k > P.ws.cap_cands) bad = true;
                } else if (sh.coff + k > sh.cres_end) {
                    uint64_t o = atomicAdd(&C->cand_cursor, (unsigned long long)P.cand_chunk);
                    sh.coff = o; sh.cres_end = o + P.cand_chunk;
                    if (o + P.cand_chunk > P.ws.cap_cands) bad = true;
                }
                if (sh.aidx >= sh.arec_end) {
                    uint32_t o = atomicAdd(&C->n_anchor, kRecChunk);
                    sh.aidx = o; sh.arec_end = o + kRecChunk;
                    if ((uint64_t)o + kRecChunk > P.ws.cap_anchors) bad = true;
                }
            }
            sh.skip = bad;
            if (bad) {
                atomicOr(&C->over_cap, 2u);
                sh.moff = sh.mres_end = sh.coff = sh.cres_end = 0;
                sh.aidx = sh.arec_end = 0;
            }
        }
        __syncthreads();
        if (sh.skip) {
            clear_region();
            continue;
        }
        const uint64_t moff = sh.big_m ? sh.bm : sh.moff, coff = sh.big_c ? sh.bc : sh.coff;
        const uint32_t aidx = sh.aidx;
        // phase 3: bit p of M_(w,c) for every higher-priority wedge through
        // position p, built in the staging area in slabs of whole mask words
        // (k x sw words each); a slab walks only the positions of its words,
        // so every wedge is visited once and every mask word written once.
        const uint32_t sw = min(W, max(1u, m.maskw / k));
        for (uint32_t w0 = 0; w0 < W; w0 += sw) {
            const uint32_t nw = min(sw, W - w0);
            const uint32_t slab = k * nw;
            for (uint32_t i = tid; i < slab; i += THREADS) mstage[i] = 0;
            __syncthreads();
            walk_positions<THREADS>(g, m, d, t1, t2, true, true,
                                    [&](const uint32_t (&e2)[kUnroll], const uint32_t (&pp)[kUnroll],
                                        const uint32_t (&sg)[kUnroll]) {
                                        uint32_t hc[kUnroll], kk[kUnroll], ci[kUnroll];
#pragma unroll
                                        for (int u = 0; u < kUnroll; u++) {
                                            hc[u] = hash_slot(e2[u] >> 1, m.log2hc);
                                            kk[u] = ckeys[hc[u]];
                                            ci[u] = cidx[hc[u]];
                                        }
#pragma unroll
                                        for (int u = 0; u < kUnroll; u++) {
                                            if (e2[u] == kEmpty || kk[u] == kEmpty) continue;
                                            const uint32_t x = e2[u] >> 1;
                                            const uint32_t v = kk[u] == x ? ci[u]
                                                                          : compact_find_from(ckeys, cidx, m.HC, hc[u], x);
                                            const uint32_t idx = ((e2[u] & 1u) ^ sg[u]) ? (v >> 16) : (v & 0xffffu);
                                            const uint32_t p = pp[u];
                                            if (idx)
                                                atomicOr(&mstage[(idx - 1) * nw + (p >> 5) - w0], 1u << (p & 31));
                                        }
                                    },
                                    32 * w0, 32 * (w0 + nw));
            __syncthreads();
            if (nw == W) {
                for (uint32_t i = tid; i < slab; i += THREADS) P.ws.masks[moff + i] = mstage[i];
            } else {
                for (uint32_t i = tid; i < slab; i += THREADS) {
                    const uint32_t c = i / nw;
                    P.ws.masks[moff + (uint64_t)c * W + w0 + (i - c * nw)] = mstage[i];
                }
            }
            __syncthreads();
        }
        for (uint32_t i = tid; i < k; i += THREADS) P.ws.cands[coff + i] = m.vc[i] & 0x7fffffffu;
        if (tid == 0) {
            AnchorRec a;
            a.rank = r; a.k = k; a.w32 = W; a.graph = g.s_graph[r];
            a.mask_off = moff; a.cand_off = coff;
            P.ws.anchors[aidx] = a;
            if (!sh.big_m) sh.moff = moff + words;
            if (!sh.big_c) sh.coff = coff + k;
            sh.aidx = aidx + 1;
        }
        __syncthreads();
        clear_region();
    }
    if (tid == 0) {
        if (sh.need_m) atomicAdd(&C->need_masks, sh.need_m);
        if (sh.need_c) atomicAdd(&C->need_cands, sh.need_c);
        if (sh.need_r) atomicAdd(&C->need_recs, sh.need_r);
        if (sh.need_u) atomicAdd(&C->need_units, sh.need_u);
        // unused reserved anchor records are marked empty
        for (uint32_t i = sh.aidx; i < sh.arec_end; i++) {
            AnchorRec a;
            a.rank = 0; a.k = 0; a.w32 = 0; a.graph = 0; a.mask_off = 0; a.cand_off = 0;
            P.ws.anchors[i] = a;
        }
    }
    my_wedges = wave_sum<uint64_t>(my_wedges);
    if (lane == 0 && my_wedges) atomicAdd(&C->wedges, (unsigned long long)my_wedges);
}

__host__ __device__ constexpr int ilog2(uint32_t x) { return x <= 1 ? 0 : 1 + ilog2(x >> 1); }
__host__ __device__ constexpr uint32_t compact_slots(uint32_t kmax, uint32_t H)
{
    uint32_t c = 1;
    while (c < 2 * kmax) c <<= 1;
    return c < H / 2 ? c : H / 2;
}

template <int THREADS, int H, int MAXD, int KMAX, bool PACKED>
__global__ void __launch_bounds__(THREADS, 2048 / THREADS) k_pair_lds(PairArgs P)
{
    __shared__ __align__(16) uint32_t region[2 * H];
    __shared__ uint32_t pst[MAXD], pln[MAXD], vc[KMAX];
    __shared__ PairShared sh;
    constexpr uint32_t HC = compact_slots(KMAX, H);
    PairMem m;
    m.region = region; m.H = H; m.log2h = ilog2(H);
    m.HC = HC; m.log2hc = ilog2(HC); m.maskw = 2 * H - 2 * HC;
    m.pst = pst; m.pln = pln; m.maxd = MAXD; m.vc = vc; m.kmax = KMAX;
    pair_loop<THREADS, PACKED>(P, m, sh);
}

// Tier B: LDS table, position lists in global memory (any degree below 2^16).
template <int THREADS, int H, int KMAX, bool PACKED>
__global__ void __launch_bounds__(THREADS) k_pair_big(PairArgs P)
{
    __shared__ __align__(16) uint32_t region[2 * H];
    __shared__ uint32_t vc[KMAX];
    __shared__ PairShared sh;
    constexpr uint32_t HC = compact_slots(KMAX, H);
    PairMem m;
    m.region = region; m.H = H; m.log2h = ilog2(H);
    m.HC = HC; m.log2hc = ilog2(HC); m.maskw = 2 * H - 2 * HC;
    m.pst = P.ws.bscr + (uint64_t)blockIdx.x * P.ws.bscr_words_per_block;
    m.pln = m.pst + P.ws.bscr_words_per_block / 2;
    m.maxd = min(P.gmaxd, (uint32_t)(P.ws.bscr_words_per_block / 2));
    m.vc = vc; m.kmax = KMAX;
    pair_loop<THREADS, PACKED>(P, m, sh);
}

constexpr int kGThreads = 1024;

// Tiers C and D: every table in global memory (C: bounded tables on many
// blocks; D: tables sized for the whole anchor side on a few blocks).
template <bool PACKED>
__global__ void __launch_bounds__(kGThreads) k_pair_global(PairArgs P)
{
    __shared__ PairShared sh;
    const bool d = P.tier == 4;
    uint32_t *base = (d ? P.ws.dtab : P.ws.gtab) +
                     (uint64_t)blockIdx.x * (d ? P.ws.dtab_words_per_block : P.ws.gtab_words_per_block);
    const uint32_t H = d ? P.dH : P.gH;
    PairMem m;
    m.region = base; m.H = H; m.log2h = d ? P.dlog2h : P.glog2h;
    m.HC = compact_slots(P.gkmax, H); m.log2hc = ilog2(m.HC);
    m.maskw = 2 * m.H - 2 * m.HC;
    m.pst = base + 2ull * H;
    m.pln = m.pst + P.gmaxd;
    m.maxd = P.gmaxd;
    m.vc = m.pln + P.gmaxd;
    m.kmax = P.gkmax;
    pair_loop<kGThreads, PACKED>(P, m, sh);
}

// --------------------------------------------------- rank-window tier (R)
// Every partner of anchor r is ranked in (r, end of r's graph), so for an
// anchor near the top of the priority order the partner keys form a short
// window. Such anchors are the heavy ones (high degree, long suffix lists,
// often thousands of candidate classes): their counting table is indexed by
// rank - r - 1 directly, one byte per partner holding a 3-bit thermometer per
// sign class, with no keys, no probing and no overflow. The classes with >= 3
// hits become the virtual candidates, numbered by a rank structure (one bitmap
// per class and per-word prefix counts) built in place of the table, so the
// mask pass finds a wedge's candidate with two LDS reads and a popcount.

// One hit on a 3-bit thermometer whose lowest bit is b0 (bits b0, 2 b0, 4 b0
// set by the first, second and third hit; later hits change nothing). A hit
// that finds a bit taken by a concurrent one moves on to the next bit.
__device__ __forceinline__ void win_hit(uint32_t *w, uint32_t b0)
{
    const uint32_t b1 = b0 << 1, b2 = b0 << 2;
    const uint32_t o = atomicOr(w, b0);
    if (!(o & b0) || (o & b2)) return;
    if (!(o & b1)) {
        const uint32_t o2 = atomicOr(w, b1);
        if (!(o2 & b1) || (o2 & b2)) return;
    }
    atomicOr(w, b2);
}

// Exclusive prefix over the workgroup's threads (thread order) of two values;
// also returns both totals. Contains barriers: every thread must call it.
template <int THREADS>
__device__ __forceinline__ void block_excl_scan2(uint32_t &a, uint32_t &b, uint32_t *tmp,
                                                 uint32_t &tot_a, uint32_t &tot_b)
{
    constexpr int NW = THREADS / kWave;
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    const uint32_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
    if (lane == kWave - 1) { tmp[wv] = ia; tmp[NW + wv] = ib; }
    __syncthreads();
    uint32_t pa = 0, pb = 0;
    tot_a = 0; tot_b = 0;
    for (int i = 0; i < NW; i++) {
        const uint32_t ta = tmp[i], tb = tmp[NW + i];
        if (i < wv) { pa += ta; pb += tb; }
        tot_a += ta; tot_b += tb;
    }
    a = pa + ia - a;
    b = pb + ib - b;
    __syncthreads();
}

__global__ void __launch_bounds__(kRThreads) k_pair_window(PairArgs P)
{
    __shared__ __align__(16) uint32_t lds[kRWords];
    __shared__ PairShared sh;
    __shared__ uint32_t scan_tmp[2 * (kRThreads / kWave)];
    __shared__ uint32_t s_k0, s_k1;
    constexpr int THREADS = kRThreads;
    constexpr uint32_t kPerThread = kRWin / 32 / THREADS;   // bitmap words per thread and class
    const int tid = threadIdx.x, lane = __lane_id();
    const CsrView &g = P.g;
    Counters *C = P.ws.ctr;
    uint64_t my_wedges = 0;
    const uint32_t n_items =
        (uint32_t)min((uint64_t)__atomic_load_n(&C->n_list[P.tier - 1], __ATOMIC_RELAXED),
                      P.ws.cap_defer);
    if (n_items == 0) return;
    const uint32_t *list = P.ws.defer[P.tier - 1];
    PairMem m{};
    m.pst = P.ws.bscr + (uint64_t)blockIdx.x * P.ws.bscr_words_per_block;
    m.pln = m.pst + P.ws.bscr_words_per_block / 2;
    m.maxd = min(P.gmaxd, (uint32_t)(P.ws.bscr_words_per_block / 2));
    if (tid == 0) {
        sh.qlo = sh.qhi = 0; sh.qslice = blockIdx.x % kXcd; sh.qtried = 0;
        sh.moff = sh.mres_end = 0; sh.coff = sh.cres_end = 0;
        sh.aidx = sh.arec_end = 0;
        sh.need_m = sh.need_c = sh.need_r = sh.need_u = 0;
        sh.vm = sh.vm_end = sh.vc = sh.vc_end = 0;
    }
    // anchors this tier cannot take go to the bounded global-memory tier
    auto to_global = [&](uint32_t r) {
        const uint32_t t = atomicAdd(&C->n_list[2], 1u);
        if (t < P.ws.cap_defer) P.ws.defer[2][t] = r; else atomicOr(&C->over_cap, 1u);
    };
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            if (sh.qlo >= sh.qhi) {
                uint32_t lo = 0, hi = 0, s = sh.qslice, tr = sh.qtried;
                if (!queue_take(C->q_pair[P.tier], n_items, 1, &s, &tr, &lo, &hi)) lo = hi = n_items;
                sh.qslice = s; sh.qtried = tr; sh.qlo = lo; sh.qhi = hi;
            }
            sh.item = sh.qlo < sh.qhi ? sh.qlo++ : n_items;
            sh.wedges = 0;
        }
        __syncthreads();
        const uint32_t item = sh.item;
        if (item >= n_items) break;
        const uint32_t r = list[n_items - 1 - item];
        const uint64_t s0 = g.s_off[r];
        const uint32_t d = (uint32_t)(g.s_off[r + 1] - s0);
        if (d < 3) continue;
        const GraphDesc &gd = g.desc[g.s_graph[r]];
        const uint32_t win = gd.s_base + gd.n_s - r - 1;
        if (d > m.maxd || win > kRWin) {
            if (tid == 0) to_global(r);
            continue;
        }
        // phase 0: suffix starts and lengths of the positions
        {
            uint32_t wsum = 0;
            for (uint32_t p = tid; p < d; p += THREADS) {
                const uint2 sf = g.s_suf[s0 + p];
                m.pst[p] = sf.x;
                m.pln[p] = sf.y;
                wsum += sf.y & 0x7fffffffu;
            }
            wsum = wave_sum<uint32_t>(wsum);
            if (lane == 0 && wsum) atomicAdd(&sh.wedges, wsum);
        }
        // the table: 8 words (32 partners) per bitmap word of the rank structure
        const uint32_t nbw = (win + 31) / 32;
        for (uint32_t i = tid; i < 8 * nbw; i += THREADS) lds[i] = 0;
        __syncthreads();
        if (sh.wedges < 6) continue;
        // phase 1: thermometer hits of every wedge
        walk_positions<THREADS>(g, m, d, kEmpty, kEmpty, true, false,
                                [&](const uint32_t (&e2)[kUnroll], const uint32_t (&)[kUnroll],
                                    const uint32_t (&sg)[kUnroll]) {
#pragma unroll
                                    for (int u = 0; u < kUnroll; u++) {
                                        if (e2[u] == kEmpty) continue;
                                        my_wedges++;
                                        const uint32_t idx = (e2[u] >> 1) - r - 1;
                                        const uint32_t cls = (e2[u] & 1u) ^ sg[u];
                                        win_hit(&lds[idx >> 2], 1u << (8 * (idx & 3) + 3 * cls));
                                    }
                                });
        __syncthreads();
        // phase 2: candidate bitmaps (bit 2 of a class's thermometer) and their
        // prefix counts; thread t owns bitmap words kPerThread t .. + kPerThread
        uint32_t b0[kPerThread], b1[kPerThread];
        uint32_t c0 = 0, c1 = 0;
#pragma unroll
        for (uint32_t i = 0; i < kPerThread; i++) {
            const uint32_t j = kPerThread * tid + i;
            uint32_t x0 = 0, x1 = 0;
            if (j < nbw) {
                const uint4 *T4 = reinterpret_cast<const uint4 *>(lds + 8 * j);
                const uint4 lo4 = T4[0], hi4 = T4[1];
                const uint32_t tw[8] = {lo4.x, lo4.y, lo4.z, lo4.w, hi4.x, hi4.y, hi4.z, hi4.w};
#pragma unroll
                for (int q = 0; q < 8; q++) {
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        x0 |= ((tw[q] >> (8 * e + 2)) & 1u) << (4 * q + e);
                        x1 |= ((tw[q] >> (8 * e + 5)) & 1u) << (4 * q + e);
                    }
                }
            }
            b0[i] = x0; b1[i] = x1;
            c0 += __popc(x0); c1 += __popc(x1);
        }
        uint32_t k0 = 0, k1 = 0;
        block_excl_scan2<THREADS>(c0, c1, scan_tmp, k0, k1);
        // (every table word has been read: the scan's barriers order the reads
        // before these writes)
#pragma unroll
        for (uint32_t i = 0; i < kPerThread; i++) {
            const uint32_t j = kPerThread * tid + i;
            if (j < nbw) {
                lds[j] = b0[i];
                lds[nbw + j] = b1[i];
                lds[2 * nbw + j] = c0;
                lds[3 * nbw + j] = c1;
            }
            c0 += __popc(b0[i]);
            c1 += __popc(b1[i]);
        }
        if (tid == 0) { s_k0 = k0; s_k1 = k1; }
        __syncthreads();
        const uint32_t K0 = s_k0, k = s_k0 + s_k1;
        if (k < 2) continue;
        const uint32_t W = (d + 31) >> 5;
        const uint32_t stage_cap = kRWords - 4 * nbw;   // >= kRWords - kRWin / 8 > 0
        if (k > P.gkmax) {
            if (tid == 0) to_global(r);
            continue;
        }
        uint32_t *stage = lds + 4 * nbw;
        const uint64_t words = (uint64_t)k * W;
        if (tid == 0) {
            // output reservations as in the hash tiers (workgroup-local chunks
            // for small outputs, a reservation of its own for a large one)
            sh.big_m = words > P.mask_chunk / 4;
            sh.big_c = k > P.cand_chunk / 4;
            if (sh.big_m) {
                sh.need_m += words;
            } else {
                if (sh.vm + words > sh.vm_end) { sh.need_m += P.mask_chunk; sh.vm = 0; sh.vm_end = P.mask_chunk; }
                sh.vm += words;
            }
            if (sh.big_c) {
                sh.need_c += k;
            } else {
                if (sh.vc + k > sh.vc_end) { sh.need_c += P.cand_chunk; sh.vc = 0; sh.vc_end = P.cand_chunk; }
                sh.vc += k;
            }
            sh.need_r += 1;
            sh.need_u += anchor_units(k, W, P.chunk_base);
            bool bad = (__atomic_load_n(&C->over_cap, __ATOMIC_RELAXED) & 2u) != 0;
            if (!bad) {
                if (sh.big_m) {
                    uint64_t o = atomicAdd(&C->mask_cursor, (unsigned long long)words);
                    sh.bm = o;
                    if (o + words > P.ws.cap_mask_words) bad = true;
                } else if (sh.moff + words > sh.mres_end) {
                    uint64_t o = atomicAdd(&C->mask_cursor, (unsigned long long)P.mask_chunk);
                    sh.moff = o; sh.mres_end = o + P.mask_chunk;
                    if (o + P.mask_chunk > P.ws.cap_mask_words) bad = true;
                }
                if (sh.big_c) {
                    uint64_t o = atomicAdd(&C->cand_cursor, (unsigned long long)k);
                    sh.bc = o;
                    if (o + k > P.ws.cap_cands) bad = true;
                } else if (sh.coff + k > sh.cres_end) {
                    uint64_t o = atomicAdd(&C->cand_cursor, (unsigned long long)P.cand_chunk);
                    sh.coff = o; sh.cres_end = o + P.cand_chunk;
                    if (o + P.cand_chunk > P.ws.cap_cands) bad = true;
                }
                if (sh.aidx >= sh.arec_end) {
                    uint32_t o = atomicAdd(&C->n_anchor, kRecChunk);
                    sh.aidx = o; sh.arec_end = o + kRecChunk;
                    if ((uint64_t)o + kRecChunk > P.ws.cap_anchors) bad = true;
                }
            }
            sh.skip = bad;
            if (bad) {
                atomicOr(&C->over_cap, 2u);
                sh.moff = sh.mres_end = sh.coff = sh.cres_end = 0;
                sh.aidx = sh.arec_end = 0;
            }
        }
        __syncthreads();
        if (sh.skip) continue;
        const uint64_t moff = sh.big_m ? sh.bm : sh.moff, coff = sh.big_c ? sh.bc : sh.coff;
        const uint32_t aidx = sh.aidx;
        // candidate ids: class 0 (same sign product) in rank order, then class 1
        for (uint32_t j = tid; j < nbw; j += THREADS) {
#pragma unroll
            for (uint32_t c = 0; c < 2; c++) {
                uint32_t bm = lds[c * nbw + j];
                uint64_t o = coff + (c ? K0 : 0u) + lds[(2 + c) * nbw + j];
                while (bm) {
                    const uint32_t b = (uint32_t)__builtin_ctz(bm);
                    bm &= bm - 1;
                    P.ws.cands[o++] = r + 1 + 32 * j + b;
                }
            }
        }
        // phase 3: bit p of the candidate's mask for every wedge through
        // position p, staged in slabs of whole mask words (a slab walks only
        // the positions of its words); when k words do not fit the staging
        // area, the candidates are taken in ranges and the words walked again
        // per range
        const uint32_t cr = min(k, stage_cap);
        const uint32_t sw = min(W, stage_cap / cr);
        for (uint32_t c0 = 0; c0 < k; c0 += cr) {
            const uint32_t nc = min(cr, k - c0);
            for (uint32_t w0 = 0; w0 < W; w0 += sw) {
                const uint32_t nw = min(sw, W - w0);
                const uint32_t slab = nc * nw;
                for (uint32_t i = tid; i < slab; i += THREADS) stage[i] = 0;
                __syncthreads();
                walk_positions<THREADS>(
                    g, m, d, kEmpty, kEmpty, true, false,
                    [&](const uint32_t (&e2)[kUnroll], const uint32_t (&pp)[kUnroll],
                        const uint32_t (&sg)[kUnroll]) {
                        uint32_t bmv[kUnroll], pre[kUnroll];
#pragma unroll
                        for (int u = 0; u < kUnroll; u++) {
                            const uint32_t idx = (e2[u] >> 1) - r - 1;
                            const uint32_t cls = (e2[u] & 1u) ^ sg[u];
                            const uint32_t j = e2[u] == kEmpty ? 0u : idx >> 5;
                            bmv[u] = lds[cls * nbw + j];
                            pre[u] = lds[(2 + cls) * nbw + j];
                        }
#pragma unroll
                        for (int u = 0; u < kUnroll; u++) {
                            if (e2[u] == kEmpty) continue;
                            const uint32_t idx = (e2[u] >> 1) - r - 1;
                            const uint32_t b = idx & 31;
                            if (!((bmv[u] >> b) & 1u)) continue;
                            const uint32_t cls = (e2[u] & 1u) ^ sg[u];
                            const uint32_t ci = (cls ? K0 : 0u) + pre[u] +
                                                __popc(bmv[u] & ((1u << b) - 1u)) - c0;
                            if (ci >= nc) continue;
                            const uint32_t p = pp[u];
                            atomicOr(&stage[ci * nw + (p >> 5) - w0], 1u << (p & 31));
                        }
                    },
                    32 * w0, 32 * (w0 + nw));
                __syncthreads();
                for (uint32_t i = tid; i < slab; i += THREADS) {
                    const uint32_t c = i / nw;
                    P.ws.masks[moff + (uint64_t)(c0 + c) * W + w0 + (i - c * nw)] = stage[i];
                }
                __syncthreads();
            }
        }
        if (tid == 0) {
            AnchorRec a;
            a.rank = r; a.k = k; a.w32 = W; a.graph = g.s_graph[r];
            a.mask_off = moff; a.cand_off = coff;
            P.ws.anchors[aidx] = a;
            if (!sh.big_m) sh.moff = moff + words;
            if (!sh.big_c) sh.coff = coff + k;
            sh.aidx = aidx + 1;
        }
    }
    if (tid == 0) {
        if (sh.need_m) atomicAdd(&C->need_masks, sh.need_m);
        if (sh.need_c) atomicAdd(&C->need_cands, sh.need_c);
        if (sh.need_r) atomicAdd(&C->need_recs, sh.need_r);
        if (sh.need_u) atomicAdd(&C->need_units, sh.need_u);
        for (uint32_t i = sh.aidx; i < sh.arec_end; i++) {
            AnchorRec a;
            a.rank = 0; a.k = 0; a.w32 = 0; a.graph = 0; a.mask_off = 0; a.cand_off = 0;
            P.ws.anchors[i] = a;
        }
    }
    my_wedges = wave_sum<uint64_t>(my_wedges);
    if (lane == 0 && my_wedges) atomicAdd(&C->wedges, (unsigned long long)my_wedges);
}

// ----------------------------------------------------- per-wave tier
// Anchors of degree <= 32 (masks of one word): the kWvWaves waves of a
// workgroup take one anchor at a time together, with a table in LDS that
// holds, per partner w, the key and both class masks M_w^+ and M_w^- (bit p
// set by the wedge through position p). The masks of the classes with >= 3
// members are copied out as they stand, so the wedges are walked once. A
// table per workgroup rather than per wave lets twice the waves share the
// LDS; the waves take alternate wedge chunks. Lane i takes the (j0 + i)-th wedge
// of the concatenated suffix lists and finds its position by a binary
// search over the lanes that hold the positions' prefix offsets. The two
// longest suffixes only update partners found elsewhere, as in the
// workgroup tiers; anchors of higher degree, or with more partners than the
// table holds, are listed for tier A.
constexpr uint32_t kWvMaxD = 32;
constexpr int kWvUnroll = 2;              // loads in flight per lane, non-top positions
constexpr int kWvTopUnroll = 16;          // and along the two longest suffixes
constexpr uint32_t kWvProbe = 64;
constexpr uint32_t kWvGrab = 2;           // anchors taken from the queue at a time
// non-top wedges (and so partners) of an anchor the per-wave tier takes, for
// a table of S slots
__host__ __device__ constexpr uint32_t wave_tier_limit(uint32_t S) { return S - S / 4; }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t bcast32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t bcast64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}


template <int S, int NWC>
__global__ void __launch_bounds__(NWC * kWave) k_pair_wave(PairArgs P)
{
    // per workgroup: S keys, 2S class masks and the list of occupied slots,
    // shared by its NWC waves, which take each anchor together
    constexpr uint32_t kLimit = wave_tier_limit(S);
    constexpr uint32_t NT = NWC * kWave;
    __shared__ uint32_t tab[3 * S + kLimit];
    __shared__ uint32_t sh_ok, sh_lo, sh_hi, sh_nkeys, sh_over, sh_k, sh_wpos, sh_bad, sh_aidx;
    __shared__ unsigned long long sh_mo, sh_co;
    constexpr int kLog2S = ilog2(S);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = __lane_id();
    const uint32_t wv = tid / kWave;
    uint32_t *keys = tab;
    uint32_t *msk = tab + S;         // msk[2 slot + class]
    uint32_t *used = tab + 3 * S;    // slots holding a key, in insertion order
    const CsrView &g = P.g;
    Counters *C = P.ws.ctr;
    const uint32_t n_items = P.a1 - P.a0;

    auto clear = [&]() {
        for (uint32_t i = tid; i < 3u * S; i += NT) tab[i] = i < (uint32_t)S ? kEmpty : 0u;
        __syncthreads();
    };
    auto clear_used = [&](uint32_t n) {
        for (uint32_t i = tid; i < n; i += NT) {
            const uint32_t sl = used[i];
            keys[sl] = kEmpty; msk[2 * sl] = 0; msk[2 * sl + 1] = 0;
        }
    };
    // called by wave 0 only, so that every anchor is listed once
    auto to_tier_a = [&](bool mine, uint32_t r) {
        const uint64_t b = ballot64(mine);
        if (!b) return;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&C->n_list[0], (uint32_t)__popcll(b));
        base = bcast32(base);
        if (mine) {
            const uint32_t t = base + (uint32_t)__popcll(b & lanemask_lt());
            if (t < P.ws.cap_defer) P.ws.defer[0][t] = r; else atomicOr(&C->over_cap, 1u);
        }
    };
    // continue a probe run after a first probe at slot h that met another key
    auto insert_from = [&](uint32_t x, uint32_t h, bool &fresh) -> uint32_t {
        for (uint32_t probe = 1; probe < kWvProbe; probe++) {
            h = (h + 1) & (S - 1);
            uint32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
            if (k == kEmpty) {
                k = atomicCAS(&keys[h], kEmpty, x);
                if (k == kEmpty) { fresh = true; return h; }
            }
            if (k == x) return h;
        }
        return kEmpty;
    };
    auto find_from = [&](uint32_t x, uint32_t h) -> uint32_t {
        for (uint32_t probe = 1; probe < kWvProbe; probe++) {
            h = (h + 1) & (S - 1);
            const uint32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
            if (k == x) return h;
            if (k == kEmpty) return kEmpty;
        }
        return kEmpty;
    };
    // the end of one anchor: table and shared counters back to idle
    auto finish_anchor = [&](uint32_t nkeys) {
        clear_used(nkeys);
        __syncthreads();
        if (tid == 0) { sh_nkeys = 0; sh_k = 0; sh_wpos = 0; sh_over = 0; }
        __syncthreads();
    };

    if (tid == 0) { sh_nkeys = 0; sh_k = 0; sh_wpos = 0; sh_over = 0; }
    clear();
    // reservation and demand state, kept by wave 0 (wave-uniform)
    uint64_t moff = 0, mres_end = 0, coff = 0, cres_end = 0;
    uint32_t aidx = 0, arec_end = 0;
    uint64_t need_m = 0, need_c = 0, need_r = 0, need_u = 0;
    uint64_t vm = 0, vm_end = 0, vcn = 0, vc_end = 0;
    uint64_t my_wedges = 0;
    uint32_t slice = blockIdx.x % kXcd, tried = 0;   // queue state of thread 0

    for (;;) {
        if (tid == 0) {
            uint32_t lo = 0, hi = 0;
            sh_ok = queue_take(C->q_pair[0], n_items, kWvGrab, &slice, &tried, &lo, &hi) ? 1u : 0u;
            sh_lo = lo; sh_hi = hi;
        }
        __syncthreads();
        const uint32_t ok = bcast32(sh_ok), lo = bcast32(sh_lo), hi = bcast32(sh_hi);
        __syncthreads();
        if (!ok) break;
        const uint32_t item = lo + lane;
        const uint32_t rl = P.a0 + item;
        uint32_t dl = 0;
        uint64_t sl0 = 0;
        if (item < hi) {
            sl0 = g.s_off[rl];
            dl = (uint32_t)(g.s_off[rl + 1] - sl0);
        }
        if (wv == 0) to_tier_a(item < hi && dl > kWvMaxD, rl);
        uint64_t todo = ballot64(item < hi && dl >= 3 && dl <= kWvMaxD);
        while (todo) {
            const uint32_t l = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const uint32_t r = P.a0 + lo + l;
            const uint64_t s0 = bcast64(__shfl(sl0, l, kWave));
            const uint32_t d = bcast32(__shfl(dl, l, kWave));
            // the part of each neighbour's list ranked above the anchor (every
            // wave reads it, so that all take the same decisions below)
            uint32_t st = 0, len = 0, sg = 0;
            if (lane < d) {
                const uint2 sf = g.s_suf[s0 + lane];
                st = sf.x;
                len = sf.y & 0x7fffffffu;
                sg = sf.y >> 31;
            }
            if (wave_sum<uint64_t>(len) < 6) continue;
            const uint64_t key1 = len ? ((uint64_t)len << 6) | lane : 0;
            const uint64_t k1 = wave_max64(key1);
            const uint64_t k2 = wave_max64(lane == (uint32_t)(k1 & 63) ? 0 : key1);
            const uint32_t t1 = (uint32_t)(k1 & 63), l1 = (uint32_t)(k1 >> 6);
            const uint32_t t2 = (uint32_t)(k2 & 63), l2 = (uint32_t)(k2 >> 6);   // l2 = 0: no second
            const uint32_t len1 = (lane == t1 || (l2 && lane == t2)) ? 0 : len;
            // every non-top wedge inserts at most one partner: with T1 <= kLimit
            // the table cannot fill up
            const uint64_t T1 = wave_sum<uint64_t>(len1);
            if (T1 > kLimit) {
                if (wv == 0) to_tier_a(lane == 0, r);
                continue;
            }
            const uint32_t incl = wave_incl_scan(len1);
            const uint32_t pre = lane < d ? incl - len1 : 0xffffffffu;
            const uint32_t info = (incl - len1) | (sg << 31);
            // walk the other positions: insert partners, set mask bits. The
            // waves take alternate chunks of kWave * kWvUnroll wedges.
            bool over = false;
            // Lanes past the end repeat the last wedge: a repeated wedge sets a
            // bit that is already set, so no lane needs a branch, and the
            // searches, loads and first probes of all kWvUnroll wedges issue
            // together.
            for (uint32_t j0 = wv * kWave * kWvUnroll; j0 < (uint32_t)T1 && !over; j0 += NT * kWvUnroll) {
                uint32_t jj[kWvUnroll], p[kWvUnroll], e2[kWvUnroll], pp[kWvUnroll];
#pragma unroll
                for (int u = 0; u < kWvUnroll; u++) {
                    jj[u] = min(j0 + u * kWave + lane, (uint32_t)T1 - 1);
                    p[u] = 0;
                }
#pragma unroll
                for (uint32_t step = 16; step; step >>= 1) {
                    uint32_t v[kWvUnroll];
#pragma unroll
                    for (int u = 0; u < kWvUnroll; u++) v[u] = __shfl(pre, p[u] + step, kWave);
#pragma unroll
                    for (int u = 0; u < kWvUnroll; u++) p[u] += v[u] <= jj[u] ? step : 0u;
                }
#pragma unroll
                for (int u = 0; u < kWvUnroll; u++) {
                    const uint32_t stp = __shfl(st, p[u], kWave);
                    const uint32_t inf = __shfl(info, p[u], kWave);
                    e2[u] = g.o_adj[stp + (jj[u] - (inf & 0x7fffffffu))];
                    pp[u] = p[u] | (inf & 0x80000000u);
                }
                // first probes of all partners at once (a CAS that returns the
                // slot's key); the few longer probe runs follow one by one
                uint32_t hs[kWvUnroll], old[kWvUnroll];
#pragma unroll
                for (int u = 0; u < kWvUnroll; u++) {
                    hs[u] = hash_slot(e2[u] >> 1, kLog2S);
                    old[u] = atomicCAS(&keys[hs[u]], kEmpty, e2[u] >> 1);
                }
                bool bad = false;
#pragma unroll
                for (int u = 0; u < kWvUnroll; u++) {
                    const uint32_t x = e2[u] >> 1;
                    const uint32_t cls = (e2[u] & 1u) ^ (pp[u] >> 31);
                    bool fresh = old[u] == kEmpty;
                    uint32_t h = hs[u];
                    if (!fresh && old[u] != x) h = insert_from(x, h, fresh);
                    if (h == kEmpty) bad = true;
                    else atomicOr(&msk[2 * h + cls], 1u << (pp[u] & 31u));
                    const uint64_t b = ballot64(fresh);
                    if (b) {
                        uint32_t base = 0;
                        if (lane == 0) base = atomicAdd(&sh_nkeys, (uint32_t)__popcll(b));
                        base = bcast32(base);
                        if (fresh) used[base + (uint32_t)__popcll(b & lanemask_lt())] = h;
                    }
                }
                over = ballot64(bad) != 0;
            }
            if (over && lane == 0) sh_over = 1;
            __syncthreads();
            if (sh_over) {   // a probe run longer than kWvProbe
                __syncthreads();
                if (tid == 0) { sh_nkeys = 0; sh_k = 0; sh_wpos = 0; sh_over = 0; }
                clear();
                if (wv == 0) to_tier_a(lane == 0, r);
                continue;
            }
            // the two longest suffixes: existing partners only
            const uint32_t ltop = l1 + l2;
            const uint32_t st1 = __shfl(st, t1, kWave), sg1 = __shfl(sg, t1, kWave);
            const uint32_t st2 = __shfl(st, t2, kWave), sg2 = __shfl(sg, t2, kWave);
            for (uint32_t j0 = wv * kWave * kWvTopUnroll; j0 < ltop; j0 += NT * kWvTopUnroll) {
                uint32_t e2[kWvTopUnroll], hs[kWvTopUnroll], kk[kWvTopUnroll];
                bool first[kWvTopUnroll];
#pragma unroll
                for (int u = 0; u < kWvTopUnroll; u++) {
                    const uint32_t j = min(j0 + u * kWave + lane, ltop - 1);   // repeats are harmless
                    first[u] = j < l1;
                    e2[u] = g.o_adj[first[u] ? st1 + j : st2 + (j - l1)];
                }
#pragma unroll
                for (int u = 0; u < kWvTopUnroll; u++) {
                    hs[u] = hash_slot(e2[u] >> 1, kLog2S);
                    kk[u] = __atomic_load_n(&keys[hs[u]], __ATOMIC_RELAXED);
                }
#pragma unroll
                for (int u = 0; u < kWvTopUnroll; u++) {
                    if (kk[u] == kEmpty) continue;
                    const uint32_t x = e2[u] >> 1;
                    const uint32_t cls = (e2[u] & 1u) ^ (first[u] ? sg1 : sg2);
                    const uint32_t h = kk[u] == x ? hs[u] : find_from(x, hs[u]);
                    if (h != kEmpty) atomicOr(&msk[2 * h + cls], 1u << (first[u] ? t1 : t2));
                }
            }
            __syncthreads();
            const uint32_t nkeys = sh_nkeys;
            // classes with >= 3 members
            uint32_t cnt = 0;
            for (uint32_t i = tid; i < nkeys; i += NT) {
                const uint32_t sl = used[i];
                cnt += (__popc(msk[2 * sl]) >= 3) + (__popc(msk[2 * sl + 1]) >= 3);
            }
            cnt = wave_sum<uint32_t>(cnt);
            if (lane == 0 && cnt) atomicAdd(&sh_k, cnt);
            __syncthreads();
            const uint32_t k = sh_k;
            if (k < 2) {
                finish_anchor(nkeys);
                continue;
            }
            if (wv == 0) {
                my_wedges += (uint64_t)T1 + ltop;
                // reservations: wave-local bump allocation, large outputs apart;
                // the demand counts what they consume with unlimited room
                const bool big_m = k > P.wv_mask_chunk / 4, big_c = k > P.wv_cand_chunk / 4;
                if (big_m) {
                    need_m += k;
                } else {
                    if (vm + k > vm_end) { need_m += P.wv_mask_chunk; vm = 0; vm_end = P.wv_mask_chunk; }
                    vm += k;
                }
                if (big_c) {
                    need_c += k;
                } else {
                    if (vcn + k > vc_end) { need_c += P.wv_cand_chunk; vcn = 0; vc_end = P.wv_cand_chunk; }
                    vcn += k;
                }
                need_r += 1;
                need_u += anchor_units(k, 1, P.chunk_base);
                bool bad = false;
                uint64_t mo = moff, co = coff;
                if (big_m || moff + k > mres_end) {
                    const uint64_t want = big_m ? k : P.wv_mask_chunk;
                    uint64_t o = 0;
                    if (lane == 0) o = atomicAdd(&C->mask_cursor, (unsigned long long)want);
                    o = bcast64(o);
                    mo = o;
                    if (!big_m) { moff = o; mres_end = o + want; }
                    if (o + want > P.ws.cap_mask_words) bad = true;
                }
                if (big_c || coff + k > cres_end) {
                    const uint64_t want = big_c ? k : P.wv_cand_chunk;
                    uint64_t o = 0;
                    if (lane == 0) o = atomicAdd(&C->cand_cursor, (unsigned long long)want);
                    o = bcast64(o);
                    co = o;
                    if (!big_c) { coff = o; cres_end = o + want; }
                    if (o + want > P.ws.cap_cands) bad = true;
                }
                if (aidx >= arec_end) {
                    uint32_t o = 0;
                    if (lane == 0) o = atomicAdd(&C->n_anchor, kRecChunk);
                    o = bcast32(o);
                    aidx = o; arec_end = o + kRecChunk;
                    if ((uint64_t)o + kRecChunk > P.ws.cap_anchors) bad = true;
                }
                if (bad) {
                    if (lane == 0) atomicOr(&C->over_cap, 2u);
                    moff = mres_end = coff = cres_end = 0;
                    aidx = arec_end = 0;
                } else {
                    if (!big_m) moff = mo + k;
                    if (!big_c) coff = co + k;
                }
                if (lane == 0) { sh_bad = bad; sh_mo = mo; sh_co = co; sh_aidx = aidx; }
                if (!bad) aidx++;
            }
            __syncthreads();
            if (sh_bad) {
                finish_anchor(nkeys);
                continue;
            }
            const uint64_t mo = sh_mo, co = sh_co;
            // copy out the selected classes and clear the table; the waves take
            // alternate groups of 64 occupied slots
            for (uint32_t i0 = wv * kWave; i0 < nkeys; i0 += NT) {
                const uint32_t i = i0 + lane;
                const uint32_t sl = i < nkeys ? used[i] : 0u;
                const uint32_t key = i < nkeys ? keys[sl] : kEmpty;
                uint32_t m0 = 0, m1 = 0;
                if (key != kEmpty) { m0 = msk[2 * sl]; m1 = msk[2 * sl + 1]; }
                const bool a0 = __popc(m0) >= 3, a1 = __popc(m1) >= 3;
                const uint64_t b0 = ballot64(a0), b1 = ballot64(a1);
                const uint32_t n01 = (uint32_t)__popcll(b0) + (uint32_t)__popcll(b1);
                uint32_t base = 0;
                if (n01) {
                    if (lane == 0) base = atomicAdd(&sh_wpos, n01);
                    base = bcast32(base);
                }
                const uint64_t lt = lanemask_lt();
                uint32_t idx = base + (uint32_t)__popcll(b0 & lt) + (uint32_t)__popcll(b1 & lt);
                if (a0) { P.ws.cands[co + idx] = key; P.ws.masks[mo + idx] = m0; idx++; }
                if (a1) { P.ws.cands[co + idx] = key; P.ws.masks[mo + idx] = m1; }
            }
            if (tid == 0) {
                AnchorRec a;
                a.rank = r; a.k = k; a.w32 = 1; a.graph = g.s_graph[r];
                a.mask_off = mo; a.cand_off = co;
                P.ws.anchors[sh_aidx] = a;
            }
            __syncthreads();
            finish_anchor(nkeys);
        }
    }
    if (wv == 0 && lane == 0) {
        if (need_m) atomicAdd(&C->need_masks, (unsigned long long)need_m);
        if (need_c) atomicAdd(&C->need_cands, (unsigned long long)need_c);
        if (need_r) atomicAdd(&C->need_recs, (unsigned long long)need_r);
        if (need_u) atomicAdd(&C->need_units, (unsigned long long)need_u);
        if (my_wedges) atomicAdd(&C->wedges, (unsigned long long)my_wedges);
    }
    // unused reserved anchor records are marked empty
    if (wv == 0) {
        for (uint32_t i = aidx + lane; i < arec_end; i += kWave) {
            AnchorRec a;
            a.rank = 0; a.k = 0; a.w32 = 0; a.graph = 0; a.mask_off = 0; a.cand_off = 0;
            P.ws.anchors[i] = a;
        }
    }
}

// ------------------------------------------------------------- planning
// Unit classes, each counted by a kernel of its own so that the register
// needs of wide masks do not lower the occupancy for narrow ones: 0 = masks
// of up to kSmallW words, 1 = up to kRegW words, 2 = wider.
constexpr uint32_t kSmallW = 4;
__device__ __forceinline__ uint32_t unit_class(uint32_t w32)
{
    return w32 > kRegW ? 2u : (w32 > kSmallW ? 1u : 0u);
}

// Units per anchor record, in the slice of its class.
// p is the number of vertices on the anchor side. p = 4: every candidate x
// of a record opens the triangle of the candidates after it (units with x + 1
// in the upper half of Unit::rb); p = 5: every pair x < y opens the triangle
// after y (x in the upper half of rb, c0 | c1 << 16 in c0, y + 1 in c1).
__global__ void __launch_bounds__(256) k_plan_count(Workspace ws, uint32_t chunk_base, uint32_t p)
{
    // after a capacity overflow the records are incomplete: plan nothing
    const uint32_t n_rec = ws.ctr->over_cap ? 0u
                                            : (uint32_t)min((uint64_t)ws.ctr->n_anchor, ws.cap_anchors);
    for (uint64_t a = (uint64_t)blockIdx.x * 256 + threadIdx.x; a < ws.cap_anchors;
         a += (uint64_t)gridDim.x * 256) {
        uint32_t c = 0, cls = 0;
        if (a < n_rec) {
            const AnchorRec &r = ws.anchors[a];
            if (r.k <= 65535u) {
                uint64_t c64 = 0;
                if (p == 4) {
                    for (uint32_t x = 0; x + 2 < r.k; x++) c64 += anchor_units(r.k - x - 1, r.w32, chunk_base);
                } else if (p == 5) {
                    // y pairs (x, y) for every y, each with the triangle after y
                    for (uint32_t y = 1; y + 2 < r.k; y++)
                        c64 += (uint64_t)y * anchor_units(r.k - y - 1, r.w32, chunk_base);
                } else {
                    c64 = anchor_units(r.k, r.w32, chunk_base);
                }
                // units are numbered in 32 bits: a larger plan is reported, not cut
                if (c64 > 0xffffffffull) atomicOr(&ws.ctr->over_cap, 32u);
                c = c64 > 0xffffffffull ? 0u : (uint32_t)c64;
            }
            cls = unit_class(r.w32);
        }
#pragma unroll
        for (uint32_t x = 0; x < 3; x++) ws.ucnt[x * ws.cap_anchors + a] = x == cls ? c : 0u;
    }
}

// One wave per anchor record writes its units.
__global__ void __launch_bounds__(256) k_plan_write(Workspace ws, uint32_t chunk_base, uint32_t p)
{
    Counters *C = ws.ctr;
    const uint32_t n_rec = C->over_cap ? 0u : (uint32_t)min((uint64_t)C->n_anchor, ws.cap_anchors);
    const uint64_t total = ws.uoff[3 * ws.cap_anchors];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        C->n_units = (uint32_t)min(total, ws.cap_units);
        C->n_cls_end[0] = (uint32_t)min(ws.uoff[ws.cap_anchors], ws.cap_units);
        C->n_cls_end[1] = (uint32_t)min(ws.uoff[2 * ws.cap_anchors], ws.cap_units);
        if (total > 0xffffffffull) atomicOr(&C->over_cap, 32u);   // units are numbered in 32 bits
        else if (total > ws.cap_units) {
            atomicOr(&C->over_cap, 2u);
            if (total > C->need_units) C->need_units = total;   // the exact demand
        }
    }
    const uint32_t lane = __lane_id();
    const uint32_t wave = (blockIdx.x * 256 + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * 256 / kWave;
    for (uint32_t a = wave; a < n_rec; a += nwaves) {
        const AnchorRec r = ws.anchors[a];
        if (r.k < 2 || r.k > 65535u) continue;
        const uint64_t base = ws.uoff[unit_class(r.w32) * ws.cap_anchors + a];
        const uint32_t CH = unit_cols(r.w32, chunk_base);
        uint32_t u0 = 0;
        // p = 3: one triangle; p = 4: the triangle after every candidate x;
        // p = 5: the triangle after y for every pair x < y
        const uint32_t ny = p == 3 ? 1 : (r.k >= 3 ? r.k - 2 : 0);
        for (uint32_t y = p == 5 ? 1 : 0; y < ny; y++) {
            const uint32_t kk = p == 3 ? r.k : r.k - y - 1;
            const uint32_t nx = p == 5 ? y : 1;
            for (uint32_t x = 0; x < nx; x++) {
                const uint32_t nb = (kk + kWave - 1) / kWave;
                for (uint32_t b = 0; b < nb; b++) {
                    const uint32_t ncols = min(kWave * (b + 1), kk) - 1;
                    const uint32_t nu = (ncols + CH - 1) / CH;
                    for (uint32_t c = lane; c < nu; c += kWave) {
                        const uint64_t idx = base + u0 + c;
                        if (idx < ws.cap_units) {
                            const uint32_t c0 = c * CH, c1 = min(c0 + CH, ncols);
                            Unit un;
                            un.anchor = a;
                            if (p == 5) {
                                un.rb = b | (x << 16); un.c0 = c0 | (c1 << 16); un.c1 = y + 1;
                            } else {
                                un.rb = b | (p == 4 ? (y + 1) << 16 : 0u); un.c0 = c0; un.c1 = c1;
                            }
                            ws.units[idx] = un;
                        }
                    }
                    u0 += nu;
                }
            }
        }
    }
}

// ------------------------------------------------------------ triplets
// C(n, q) for the general-q totals. After step i, c = C(n, i + 1), computed
// as (c div d) (n - i) + (c mod d) (n - i) / d with d = i + 1, which is exact
// because d divides c (n - i); `ovf` is set when C(n, q) needs more than 64
// bits.
__host__ __device__ __forceinline__ uint64_t choose_q(uint32_t n, uint32_t q, bool &ovf)
{
    if (n < q) return 0;
    uint64_t c = 1;
    for (uint32_t i = 0; i < q; i++) {
        const uint64_t d = i + 1, f = n - i;
        uint64_t hi;
        if (__builtin_mul_overflow(c / d, f, &hi)) { ovf = true; return 0; }
        const uint64_t lo = (c % d) * f / d;
        if (__builtin_add_overflow(hi, lo, &c)) { ovf = true; return 0; }
    }
    return c;
}

// Rows in lanes, masks of W <= 16 words in registers; columns through
// scalar loads, 8 at a time.
template <int W, int MODE>
__device__ __forceinline__ uint64_t tri_rows(const Unit &un, const AnchorRec &a,
                                             const uint32_t *__restrict__ masks,
                                             const uint32_t *c3, const uint64_t *cq,
                                             uint64_t *colacc, const TriArgs &T)
{
    const uint32_t lane = __lane_id();
    const uint32_t i = un.rb * kWave + lane;
    const bool vi = i < a.k;
    const uint32_t *M = masks + a.mask_off;
    const BBC_CONST uint32_t *MS = as_const(M);
    uint32_t row[W];
#pragma unroll
    for (int w = 0; w < W; w++) row[w] = vi ? M[(uint64_t)i * W + w] : 0u;
    const bool diag = un.c1 > un.rb * kWave;
    uint64_t acc = 0;
    uint32_t j = un.c0;
    if (MODE == 3) {
        // totals with C(n, q) from the 64-bit table cq
        for (; j < un.c1; j++) {
            const BBC_CONST uint32_t *cp = MS + (uint64_t)j * W;
            uint32_t n = 0;
#pragma unroll
            for (int w = 0; w < W; w++) n += __popc(row[w] & cp[w]);
            acc += (!diag || j < i) ? cq[n] : 0ull;
        }
        return acc;
    }
    if (MODE == 0) {
        // 8 columns = 8*W consecutive words: one pointer, immediate offsets.
        // Only units that reach the diagonal need the j < i test.
        if (!diag) {
            for (; j + 8 <= un.c1; j += 8) {
                const BBC_CONST uint32_t *cp = MS + (uint64_t)j * W;
                uint32_t s = 0;
#pragma unroll
                for (int jj = 0; jj < 8; jj++) {
                    uint32_t n = 0;
#pragma unroll
                    for (int w = 0; w < W; w++) n += __popc(row[w] & cp[jj * W + w]);
                    s += c3[n];
                }
                acc += s;
            }
        } else {
            for (; j + 8 <= un.c1; j += 8) {
                const BBC_CONST uint32_t *cp = MS + (uint64_t)j * W;
                uint32_t s = 0;
#pragma unroll
                for (int jj = 0; jj < 8; jj++) {
                    uint32_t n = 0;
#pragma unroll
                    for (int w = 0; w < W; w++) n += __popc(row[w] & cp[jj * W + w]);
                    const uint32_t t = c3[n];
                    s += (j + jj < i) ? t : 0u;
                }
                acc += s;
            }
        }
        for (; j < un.c1; j++) {
            const BBC_CONST uint32_t *cp = MS + (uint64_t)j * W;
            uint32_t n = 0;
#pragma unroll
            for (int w = 0; w < W; w++) n += __popc(row[w] & cp[w]);
            uint32_t t = c3[n];
            if (diag) t = (j < i) ? t : 0u;
            acc += t;
        }
        return acc;
    }
    for (; j < un.c1; j++) {
        uint32_t cw[W];
        uint32_t n = 0;
        const BBC_CONST uint32_t *cp = MS + (uint64_t)j * W;
#pragma unroll
        for (int w = 0; w < W; w++) {
            cw[w] = cp[w];
            n += __popc(row[w] & cw[w]);
        }
        uint32_t t = c3[n];
        if (diag) t = (j < i) ? t : 0u;
        acc += t;
        if (t) {
            if (MODE == 1) {
                atomicAdd((unsigned long long *)&colacc[j - un.c0], (unsigned long long)t);
            } else {
                // every member of the common class lies in C(n-1, 2) of these
                // bicliques: summed per anchor position in the wave's LDS array
                // (colacc here), scattered to the vertices once per unit
                const uint64_t each = choose2(n - 1);
#pragma unroll
                for (int w = 0; w < W; w++) {
                    uint32_t m = row[w] & cw[w];
                    while (m) {
                        const uint32_t b = __ffs(m) - 1;
                        m &= m - 1;
                        atomicAdd((unsigned long long *)&colacc[w * 32 + b], (unsigned long long)each);
                    }
                }
            }
        }
    }
    return acc;
}

// Masks wider than 16 words: up to 32 columns per unit, taken 8 at a time
// with one counter per column in registers; row words are streamed 16 at a
// time (re-read per column group from L1/L2), column words by scalar loads.
template <int MODE>
__device__ uint64_t tri_rows_wide(const Unit &un, const AnchorRec &a,
                                  const uint32_t *__restrict__ masks, uint64_t *colacc,
                                  const TriArgs &T, const uint32_t *xm = nullptr,
                                  const uint32_t *ym = nullptr)
{
    const uint32_t lane = __lane_id();
    const uint32_t i = un.rb * kWave + lane;
    const bool vi = i < a.k;
    const uint32_t W = a.w32;
    const uint32_t *M = masks + a.mask_off;
    const BBC_CONST uint32_t *MS = as_const(M);
    const uint32_t ncol = un.c1 - un.c0;
    uint64_t acc = 0;
    for (uint32_t cg = 0; cg < ncol; cg += 8) {
        uint32_t n[8];
#pragma unroll
        for (int c = 0; c < 8; c++) n[c] = 0;
        for (uint32_t w0 = 0; w0 < W; w0 += kRegW) {
            const uint32_t wn = min(kRegW, W - w0);
            uint32_t row[kRegW];
#pragma unroll
            for (int w = 0; w < (int)kRegW; w++) {
                row[w] = (vi && (uint32_t)w < wn) ? M[(uint64_t)i * W + w0 + w] : 0u;
                if (MODE >= 4 && (uint32_t)w < wn) row[w] &= xm[w0 + w] & ym[w0 + w];   // rows meet x (and y)
            }
#pragma unroll
            for (int c = 0; c < 8; c++) {
                if (cg + c < ncol) {
                    const BBC_CONST uint32_t *col = MS + (uint64_t)(un.c0 + cg + c) * W + w0;
                    uint32_t s = 0;
#pragma unroll
                    for (int w = 0; w < (int)kRegW; w++)
                        if ((uint32_t)w < wn) s += __popc(row[w] & col[w]);
                    n[c] += s;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const uint32_t j = un.c0 + cg + c;
            uint64_t t = 0;
            if (cg + c < ncol && j < i) {
                if (MODE >= 3) {
                    bool ovf = false;
                    t = choose_q(n[c], T.q, ovf);
                    if (ovf) atomicOr(&T.ws.ctr->over_cap, 16u);
                } else {
                    t = choose3(n[c]);
                }
            }
            acc += t;
            if ((MODE == 1 || MODE == 2) && t) {
                if (MODE == 1) {
                    atomicAdd((unsigned long long *)&colacc[cg + c], (unsigned long long)t);
                } else {
                    // every member of the common class lies in C(n-1, 2) of these bicliques
                    const uint64_t each = choose2(n[c] - 1);
                    const uint64_t s0 = T.g.s_off[a.rank];
                    for (uint32_t w = 0; w < W; w++) {
                        uint32_t m = M[(uint64_t)i * W + w] & M[(uint64_t)j * W + w];
                        while (m) {
                            const uint32_t b = __ffs(m) - 1;
                            m &= m - 1;
                            const uint32_t o = T.g.s_adj[s0 + w * 32 + b] >> 1;
                            atomicAdd(&T.ws.pv_o[o], (unsigned long long)each);
                        }
                    }
                }
            }
        }
    }
    return acc;
}

constexpr int kTThreads = 256;
constexpr uint32_t kMaxChunk = 2048;
constexpr uint32_t kUnitGrab = 4;   // units per queue take of a triplet wave

// ---------------------------------------------- matrix-core triplet path
// The counts |M_x n M_y| of one unit form an integer matrix product of
// 0/1 matrices (rows x mask bits times mask bits x columns), which runs on
// the fp4 matrix cores (below). The totals need n (n - 1) (n - 2) =
// D (D^2 - 1) with D = n - 1, zero for n <= 2 (also for padding rows and
// columns, whose masks are zero, and for masked pairs, set to D = -1). Each
// term is 6 C(n, 3), so a lane's sum is divided by 6 once.
typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

// a * b + c with a and b taken as 24-bit signed integers (full rate)
__device__ __forceinline__ uint32_t mad_i24(int a, int b, uint32_t c)
{
    uint32_t r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Sum of D (D^2 - 1) over N pairs of packed 16-bit D, each -1 (0xffff) or
// 0 <= D < 256: D^2 - 1 wraps to 0 for 0xffff and fits 16 bits for the
// others, so one packed multiply-add and one two-term dot product serve two
// pairs. All squares are formed before the first product that reads one.
template <int N>
__device__ __forceinline__ uint32_t cubic_sum_u16(const u16x2 (&p)[N][2])
{
    u16x2 e[N][2];
    uint32_t s[N];
#pragma unroll
    for (int n = 0; n < N; n++)
#pragma unroll
        for (int h = 0; h < 2; h++) e[n][h] = p[n][h] * p[n][h] + (u16x2){0xffff, 0xffff};
#pragma unroll
    for (int n = 0; n < N; n++) s[n] = __builtin_amdgcn_udot2(p[n][0], e[n][0], 0u, false);
#pragma unroll
    for (int n = 0; n < N; n++) s[n] = __builtin_amdgcn_udot2(p[n][1], e[n][1], s[n], false);
    uint32_t t = 0;
#pragma unroll
    for (int n = 0; n < N; n++) t += s[n];
    return t;
}

// Sum of D (D^2 - 1) over N accumulators, D = n - 1 with n <= 32 W: packed
// for W <= 8 (n <= 256; converted to 16 bits with clamping, -1 becomes
// 0xffff), 24-bit multiply-adds above (-1 <= D < 512: both products fit,
// which the compiler cannot prove). Every accumulator has a partial sum of
// its own, so that consecutive instructions do not depend on each other.
// With MASKED set, element k of accumulator n (row i0 + 16 n + k, column j)
// counts only for j < i0 + 16 n + k, the others are taken as D = -1.
template <int W, int N, bool MASKED>
__device__ __forceinline__ uint32_t cubic_sum(const v4i32 (&acc)[N], uint32_t j, uint32_t i0)
{
    auto D = [&](int n, int k) -> int {
        return !MASKED || j < i0 + 16 * n + k ? acc[n][k] : -1;
    };
    uint32_t s[N];
    if constexpr (W <= 8) {
        u16x2 p[N][2];
#pragma unroll
        for (int n = 0; n < N; n++)
#pragma unroll
            for (int h = 0; h < 2; h++)
                p[n][h] = __builtin_bit_cast(
                    u16x2, __builtin_amdgcn_cvt_pk_u16((uint32_t)D(n, 2 * h), (uint32_t)D(n, 2 * h + 1)));
        return cubic_sum_u16<N>(p);
    } else {
#pragma unroll
        for (int n = 0; n < N; n++) s[n] = 0;
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
            for (int n = 0; n < N; n++) {
                const int d = D(n, k);
                s[n] = mad_i24(d, mad_i24(d, d, -1), s[n]);
            }
    }
    uint32_t t = 0;
#pragma unroll
    for (int n = 0; n < N; n++) t += s[n];
    return t;
}

// The fp32 accumulators of the C(n, 3) totals start at 2^23 + 2^16 - 1
// instead of -1. Every partial sum is an integer below 2^24 (n < 2^16), so
// the sums are exact and each ends at 2^23 + 2^16 + D (D = n - 1 >= -1),
// whose encoding is kDBits + D: its low 16 bits are D mod 2^16 (0xffff for
// n = 0) with no conversion, and D is one integer subtraction away.
constexpr float kDInit = 8454143.0f;       // 2^23 + 2^16 - 1
constexpr uint32_t kDBits = 0x4b010000u;   // encoding of 2^23 + 2^16

__device__ __forceinline__ int enc_d(float x) { return (int)(__float_as_uint(x) - kDBits); }

// cubic_sum of encoded accumulators, every D <= 255: one byte permutation
// packs the low halves of two encodings
template <int N>
__device__ __forceinline__ uint32_t cubic_sum_enc(const v4f32 (&acc)[N])
{
    u16x2 p[N][2];
#pragma unroll
    for (int n = 0; n < N; n++)
#pragma unroll
        for (int h = 0; h < 2; h++)
            p[n][h] = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(__float_as_uint(acc[n][2 * h + 1]),
                                                                     __float_as_uint(acc[n][2 * h]),
                                                                     0x05040100u));
    return cubic_sum_u16<N>(p);
}

// largest accumulator of N, compared with the encoding of D = 255
template <int N>
__device__ __forceinline__ bool enc_over_255(const v4f32 (&acc)[N])
{
    float m = acc[0][0];
#pragma unroll
    for (int n = 0; n < N; n++)
#pragma unroll
        for (int k = 0; k < 4; k++) m = fmaxf(m, acc[n][k]);
    return m > kDInit + 256.f;
}

// fp4 operands: v_mfma_scale_f32_16x16x128_f8f6f4 with both operands in e2m1
// (and unit scales) multiplies 16 x 128 by 128 x 16; lane l supplies row (or
// column) l % 16, elements 32 (l / 16) .. + 31, eight per register. One
// 32-bit mask word fills a lane's four registers: element i of register q is
// bit 4 i + q, for rows and columns alike. A set bit becomes a power of two
// whose e2m1 code is that bit, moved within its nibble only where needed:
// column registers 0 to 3 hold 0.5, 1.0, 2.0, 2.0 (codes 0b0001, 0b0010,
// 0b0100; bit 3 is the sign, so register 3 is shifted) and row registers
// 2.0, 1.0, 0.5, 0.5. Every product of two set bits is then exactly 1 and
// the fp32 sums are exact integers (n <= 32 W < 2^24). Columns are spread
// once per tile and cost five instructions per word (one shift, four ands);
// rows are spread once per unit.
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));
typedef int v8i32 __attribute__((ext_vector_type(8)));
constexpr int kFp4 = 4;       // operand format code of e2m1 (A and B)
constexpr int kScale1 = 127;  // e8m0 scale 2^0

typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));
typedef __amdgpu_buffer_rsrc_t Rsrc;

// a buffer range of `bytes` bytes from p (p and bytes wave-uniform); raw
// loads past it return 0
__device__ __forceinline__ Rsrc mask_rsrc(const uint32_t *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(p), 0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ v8i32 spread_col(uint32_t x)
{
    v8i32 r = {0, 0, 0, 0, 0, 0, 0, 0};
    r[0] = (int)(x & 0x11111111u);
    r[1] = (int)(x & 0x22222222u);
    r[2] = (int)(x & 0x44444444u);
    r[3] = (int)((x >> 1) & 0x44444444u);
    return r;
}

__device__ __forceinline__ v8i32 spread_row(uint32_t x)
{
    v8i32 r = {0, 0, 0, 0, 0, 0, 0, 0};
    r[0] = (int)((x << 2) & 0x44444444u);
    r[1] = (int)(x & 0x22222222u);
    r[2] = (int)((x >> 2) & 0x11111111u);
    r[3] = (int)((x >> 3) & 0x11111111u);
    return r;
}

__device__ __forceinline__ v4f32 mfma_fp4(const v8i32 &a, const v8i32 &b, const v4f32 &c)
{
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, kFp4, kFp4, 0, kScale1, 0, kScale1);
}

// The same sum on the fp4 matrix cores. Lane group g holds words
// NC g .. NC g + NC - 1 of its row or column (NC = ceil(W / 4), one load of
// NC consecutive words, at most NC - 1 of them past the row) and chunk t takes
// word NC g + t, the same placement for rows and columns; words past the mask
// width are dropped by the spread. The rows of all four blocks stay in
// registers (4 NC x 4), so every unit is one pass. MODE 0 sums C(n, 3) (the
// cubic of D = n - 1, divided by 6 once) from encoded accumulators; the
// other modes start them at -1 and convert D to an integer. MODE 3 sums C(n, q) from the workgroup's table
// cq (n <= 32 W <= 512). MODE 1 (per vertex of the anchor side) takes C(n, 3)
// per pair from the table c3, adds each column's total to the wave's colacc
// (one lane per column) and keeps 16 row totals per lane, which are summed
// over the lane group at the end of the unit and handed out so that lane L
// returns the total of row 64 rb + L (a row total is at most C(512, 3) x 128
// < 2^32 for W <= 16, as the unit has at most 2048 / W columns).
template <int W, int MODE>
__device__ uint64_t tri_rows_fp4(const Unit &un, const AnchorRec &a,
                                 const uint32_t *__restrict__ masks, const uint64_t *cq,
                                 const uint32_t *c3, uint64_t *colacc, const uint32_t *xm,
                                 const uint32_t *ym)
{
    constexpr int NC = (W + 3) / 4;          // 128-bit K-chunks
    constexpr int SB = 4;
    const uint32_t lane = __lane_id();
    const uint32_t g = lane >> 4, r16 = lane & 15u;
    const uint32_t *M = masks + a.mask_off;
    const uint32_t rbase = un.rb * kWave;
    const uint32_t wf = g * NC;                           // first word of the lane's piece
    const uint32_t ws = wf < (uint32_t)W ? wf : (uint32_t)W - 1;
    // The anchor's masks as two buffer ranges from M, rows below a.k and
    // columns below un.c1 (k W < 2^22 bytes): a load past its range returns
    // 0, so rows and columns past the candidates take no test. A lane reads
    // words wf .. wf + NC - 1 of its row, in one load where W is a multiple
    // of 4 (all of them then lie in the row); otherwise word by word, and kw
    // clears the words at W or past it (another row's, or 0).
    const Rsrc rrow = mask_rsrc(M, a.k * (uint32_t)W * 4u);
    const Rsrc rcol = mask_rsrc(M, un.c1 * (uint32_t)W * 4u);
    const uint32_t lofs = (r16 * (uint32_t)W + wf) * 4u;
    uint32_t kw[NC];
#pragma unroll
    for (int t = 0; t < NC; t++) kw[t] = W % 4 == 0 || wf + t < (uint32_t)W ? ~0u : 0u;
    auto words = [&](const Rsrc &r, uint32_t row0, uint32_t (&raw)[NC]) {
        const int off = (int)(row0 * ((uint32_t)W * 4u) + lofs);
        if constexpr (W % 4 == 0 && NC == 4) {
            const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
            raw[0] = v.x; raw[1] = v.y; raw[2] = v.z; raw[3] = v.w;
        } else if constexpr (W % 4 == 0 && NC == 2) {
            const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
            raw[0] = v.x; raw[1] = v.y;
        } else {
#pragma unroll
            for (int t = 0; t < NC; t++) raw[t] = __builtin_amdgcn_raw_buffer_load_b32(r, off + 4 * t, 0, 0);
        }
    };
    // MODE 4 and 5: the rows meet the masks xm and ym of the candidates
    // chosen before them (the same mask for MODE 4; same word layout)
    uint32_t xw[NC];
#pragma unroll
    for (int t = 0; t < NC; t++) xw[t] = (MODE >= 4 ? xm[ws + t] & ym[ws + t] : ~0u) & kw[t];
    v8i32 A[SB][NC];
    uint32_t pmax = 0;   // most set bits in one of the lane's row pieces
#pragma unroll
    for (int sb = 0; sb < SB; sb++) {
        uint32_t raw[NC], pc = 0;
        words(rrow, rbase + 16 * sb, raw);
#pragma unroll
        for (int t = 0; t < NC; t++) {
            A[sb][t] = spread_row(raw[t] & xw[t]);
            if constexpr (MODE == 0 && W > 8) pc += __popc(raw[t] & xw[t]);
        }
        pmax = max(pmax, pc);
    }
    // MODE 0, masks over 8 words: when no row piece has more than 64 bits
    // (no row more than 256), no pair of the unit meets in more than 256
    const bool rows_small = MODE == 0 && W > 8 && !__any(pmax > 64u);
    auto col_words = [&](uint32_t j0, uint32_t (&raw)[NC]) { words(rcol, j0, raw); };
    auto products = [&](const uint32_t (&raw)[NC], uint32_t j0, v4f32 (&acc)[SB]) {
        constexpr float a0 = MODE == 0 ? kDInit : -1.f;
#pragma unroll
        for (int sb = 0; sb < SB; sb++) acc[sb] = (v4f32){a0, a0, a0, a0};
#pragma unroll
        for (int t = 0; t < NC; t++) {
            const v8i32 B = spread_col(W % 4 == 0 ? raw[t] : raw[t] & kw[t]);
#pragma unroll
            for (int sb = 0; sb < SB; sb++) acc[sb] = mfma_fp4(A[sb][t], B, acc[sb]);
        }
    };
    uint32_t rs[SB][4];   // MODE 1: row totals of the lane's 16 rows over its columns
#pragma unroll
    for (int sb = 0; sb < SB; sb++)
#pragma unroll
        for (int e = 0; e < 4; e++) rs[sb][e] = 0;
    auto epilogue = [&](const v4f32 (&acc)[SB], uint32_t j0) -> uint64_t {
        if constexpr (MODE == 1) {
            const bool diag = j0 + 16 > rbase;
            const uint32_t j = j0 + r16, i0 = rbase + 4 * g;
            uint32_t cs = 0;
#pragma unroll
            for (int sb = 0; sb < SB; sb++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const uint32_t n = (uint32_t)((int)acc[sb][e] + 1);
                    const uint32_t t = (!diag || j < i0 + 16 * sb + e) ? c3[n] : 0u;
                    rs[sb][e] += t;
                    cs += t;
                }
            cs += __shfl_xor(cs, 16, kWave);
            cs += __shfl_xor(cs, 32, kWave);
            if (g == 0 && j < un.c1 && cs) colacc[j - un.c0] += cs;
            return 0;
        } else if constexpr (MODE >= 3) {
            // element e of block sb: row rbase + 16 sb + 4 g + e, column j0 + r16
            const bool diag = j0 + 16 > rbase;
            const uint32_t j = j0 + r16, i0 = rbase + 4 * g;
            uint64_t t = 0;
#pragma unroll
            for (int sb = 0; sb < SB; sb++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const uint32_t n = (uint32_t)((int)acc[sb][e] + 1);
                    if (!diag || j < i0 + 16 * sb + e) t += cq[n];
                }
            return t;
        } else {
            // encoded accumulators; masks over 9 to 16 words take the packed
            // form in a unit whose rows have at most 256 bits, else in a tile
            // whose pairs all meet in at most 256 bits (wave-uniform tests),
            // as do masks up to 8 words always
            const bool full = __builtin_expect(j0 + 16 <= rbase, 1);   // every column before every row
            if (full && (W <= 8 || rows_small || !__any(enc_over_255<SB>(acc)))) return cubic_sum_enc<SB>(acc);
            v4i32 d[SB];
#pragma unroll
            for (int sb = 0; sb < SB; sb++)
#pragma unroll
                for (int e = 0; e < 4; e++) d[sb][e] = enc_d(acc[sb][e]);
            if (full) return cubic_sum<W, SB, false>(d, 0, 0);
            return cubic_sum<W, SB, true>(d, j0 + r16, rbase + 4 * g);
        }
    };
    // Columns past un.c1 read as 0 (their buffer range ends there), so the
    // words of the tile after next are loaded without a test.
    uint64_t sum = 0;
    uint32_t w0[NC], w1[NC];
    v4f32 acc0[SB], acc1[SB];
    uint32_t j0 = un.c0;
    col_words(j0, w0);
    col_words(j0 + 16, w1);
    products(w0, j0, acc0);
    for (;;) {
        bool more = j0 + 16 < un.c1;
        col_words(j0 + 32, w0);
        if (more) products(w1, j0 + 16, acc1);
        sum += epilogue(acc0, j0);
        if (!more) break;
        j0 += 16;
        more = j0 + 16 < un.c1;
        col_words(j0 + 32, w1);
        if (more) products(w0, j0 + 16, acc0);
        sum += epilogue(acc1, j0);
        if (!more) break;
        j0 += 16;
    }
    if constexpr (MODE == 1) {
        // row totals over the 16 lanes of the group (their columns), then lane
        // L takes row 64 rb + L: block L / 16, group (L / 4) % 4, element L % 4
#pragma unroll
        for (int sb = 0; sb < SB; sb++)
#pragma unroll
            for (int e = 0; e < 4; e++)
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) rs[sb][e] += __shfl_xor(rs[sb][e], o, kWave);
        const uint32_t src = 16 * ((lane >> 2) & 3u), want = 4 * (lane >> 4) + (lane & 3u);
        uint32_t mine = 0;
#pragma unroll
        for (int sb = 0; sb < SB; sb++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t v = __shfl(rs[sb][e], src, kWave);
                mine = (uint32_t)(4 * sb + e) == want ? v : mine;
            }
        return mine;
    }
    return MODE >= 3 ? sum : sum / 6;
}

// Masks wider than 16 words (totals): 64 rows x up to 64 columns per unit,
// on the fp4 matrix cores. The products of all four column tiles stay in
// accumulators while the mask words go by in K-blocks of 16 words: lane
// group g holds words 4 g .. 4 g + 3 of its row or column (one 16-byte load)
// and chunk t takes word 4 g + t, the same placement for rows and columns.
// The last W mod 16 words go by chunks of four consecutive words (chunk t,
// group g: word 4 t + g), so that no chunk past the mask is issued; a word
// past the row is cleared. n can reach 32 W, so the epilogue is 64-bit:
// n (n - 1) (n - 2) = n ((n^2 + 2) - 3 n), which is 0 for n = 0, 1, 2 with
// unsigned wrap-around. MODE 3-5 take C(n, q) instead (the table, or the
// exact 64-bit product above its end), and MODE 4-5 meet the row words with
// the masks of the candidates chosen before the rows. MODE 1 returns lane L's
// row total (row 64 rb + L) and adds the column totals to colacc.
template <int MODE>
__device__ uint64_t tri_rows_mfma_wide(const Unit &un, const AnchorRec &a,
                                       const uint32_t *__restrict__ masks, const uint64_t *cq,
                                       uint64_t *colacc, const TriArgs &T, const uint32_t *xm,
                                       const uint32_t *ym)
{
    static_assert(MODE != 2, "no per-vertex counts of the other side");
    constexpr uint32_t KW = 16;              // words per K-block
    const uint32_t lane = __lane_id();
    const uint32_t g = lane >> 4, r16 = lane & 15u;
    const uint32_t W = a.w32;
    const uint32_t *M = masks + a.mask_off;
    const uint32_t rbase = un.rb * kWave;
    const uint32_t nt = (un.c1 - un.c0 + 15) / 16;   // column tiles (<= 4)
    // The anchor's masks as buffer ranges from the K-block's first word on,
    // rows below a.k and columns below un.c1 (k W < 2^32 bytes): a load past
    // its range returns 0, so rows and columns past the candidates take no
    // test. ro and co: byte offsets of word 4 g of the lane's rows and
    // columns. A full K-block reads words w0 + 4 g .. + 3, all in the row.
    uint32_t ro[4], co[4];
#pragma unroll
    for (int sb = 0; sb < 4; sb++) {
        ro[sb] = ((rbase + 16 * sb + r16) * W + 4 * g) * 4u;
        co[sb] = ((un.c0 + 16 * sb + r16) * W + 4 * g) * 4u;
    }
    const uint32_t rbytes = a.k * W * 4u, cbytes = un.c1 * W * 4u;
    v4f32 acc[4][4];
#pragma unroll
    for (int tt = 0; tt < 4; tt++)
#pragma unroll
        for (int sb = 0; sb < 4; sb++)
            acc[tt][sb] = MODE == 0 ? (v4f32){kDInit, kDInit, kDInit, kDInit} : (v4f32){0.f, 0.f, 0.f, 0.f};
    const uint32_t Wf = W & ~(KW - 1);
    // One K-block of 16 words. NTC is the number of column tiles when it is
    // known at compile time (4: a full unit, the common case, whose K-block
    // then has no branches), else 0 and the unit's nt is tested per tile.
    auto kblock = [&](uint32_t w0, auto ntc) {
        constexpr int NTC = decltype(ntc)::value;
        const Rsrc rr = mask_rsrc(M + w0, rbytes - 4u * w0), rc_ = mask_rsrc(M + w0, cbytes - 4u * w0);
        uint32_t ra[4][4], rc[4][4];
#pragma unroll
        for (int sb = 0; sb < 4; sb++) {
            const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(rr, (int)ro[sb], 0, 0);
            ra[sb][0] = v.x; ra[sb][1] = v.y; ra[sb][2] = v.z; ra[sb][3] = v.w;
        }
        if constexpr (MODE >= 4) {
            // the rows meet the masks of the candidates chosen before them
            const uint32_t wl = w0 + 4 * g;
            const u32x4a4 x = *reinterpret_cast<const u32x4a4 *>(xm + wl);
            const u32x4a4 y = *reinterpret_cast<const u32x4a4 *>(ym + wl);
            const uint32_t xy[4] = {x.x & y.x, x.y & y.y, x.z & y.z, x.w & y.w};
#pragma unroll
            for (int sb = 0; sb < 4; sb++)
#pragma unroll
                for (int t = 0; t < 4; t++) ra[sb][t] &= xy[t];
        }
#pragma unroll
        for (int tt = 0; tt < 4; tt++) {
            if (NTC == 0 && (uint32_t)tt >= nt) break;
            const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(rc_, (int)co[tt], 0, 0);
            rc[tt][0] = v.x; rc[tt][1] = v.y; rc[tt][2] = v.z; rc[tt][3] = v.w;
        }
#pragma unroll
        for (int t = 0; t < 4; t++) {
            v8i32 A[4];
#pragma unroll
            for (int sb = 0; sb < 4; sb++) A[sb] = spread_row(ra[sb][t]);
#pragma unroll
            for (int tt = 0; tt < 4; tt++) {
                if (NTC == 0 && (uint32_t)tt >= nt) break;
                const v8i32 B = spread_col(rc[tt][t]);
#pragma unroll
                for (int sb = 0; sb < 4; sb++) acc[tt][sb] = mfma_fp4(A[sb], B, acc[tt][sb]);
            }
        }
    };
    if (nt == 4) {
        for (uint32_t w0 = 0; w0 < Wf; w0 += KW) kblock(w0, std::integral_constant<int, 4>{});
    } else {
        for (uint32_t w0 = 0; w0 < Wf; w0 += KW) kblock(w0, std::integral_constant<int, 0>{});
    }
    // the last W mod 16 words by chunks of four: lane group g takes word
    // w + g, at byte offset ro - 12 g from the chunk's first word; a word at
    // W or past it (another row's, or 0) is cleared
    for (uint32_t w = Wf; w < W; w += 4) {
        const Rsrc rr = mask_rsrc(M + w, rbytes - 4u * w), rc_ = mask_rsrc(M + w, cbytes - 4u * w);
        const uint32_t wg = w + g;
        const bool kw = wg < W;
        const uint32_t xy = MODE >= 4 ? xm[kw ? wg : W - 1] & ym[kw ? wg : W - 1] : ~0u;
        v8i32 A[4];
#pragma unroll
        for (int sb = 0; sb < 4; sb++) {
            const uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(rr, (int)(ro[sb] - 12u * g), 0, 0) & xy;
            A[sb] = spread_row(kw ? x : 0u);
        }
#pragma unroll
        for (int tt = 0; tt < 4; tt++) {
            if ((uint32_t)tt >= nt) break;
            const uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(rc_, (int)(co[tt] - 12u * g), 0, 0);
            const v8i32 B = spread_col(kw ? x : 0u);
#pragma unroll
            for (int sb = 0; sb < 4; sb++) acc[tt][sb] = mfma_fp4(A[sb], B, acc[tt][sb]);
        }
    }
    if constexpr (MODE == 1) {
        // C(n, 3) per pair (64-bit: n can pass 512), summed per column into
        // the wave's column totals and per row into the lane's 16 rows
        uint64_t rs[4][4];
#pragma unroll
        for (int sb = 0; sb < 4; sb++)
#pragma unroll
            for (int e = 0; e < 4; e++) rs[sb][e] = 0;
#pragma unroll
        for (int tt = 0; tt < 4; tt++) {
            if ((uint32_t)tt >= nt) break;
            const uint32_t j = un.c0 + 16 * tt + r16;
            uint64_t cs = 0;
#pragma unroll
            for (int sb = 0; sb < 4; sb++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const uint64_t n = j < rbase + 16 * sb + 4 * g + e ? (uint32_t)acc[tt][sb][e] : 0u;
                    const uint64_t t = n >= 3 ? n * (n - 1) * (n - 2) / 6 : 0;
                    rs[sb][e] += t;
                    cs += t;
                }
            cs += __shfl_xor(cs, 16, kWave);
            cs += __shfl_xor(cs, 32, kWave);
            if (g == 0 && j < un.c1 && cs) colacc[j - un.c0] += cs;
        }
        // row totals over the 16 lanes of the group, then lane L takes row
        // 64 rb + L: block L / 16, group (L / 4) % 4, element L % 4
#pragma unroll
        for (int sb = 0; sb < 4; sb++)
#pragma unroll
            for (int e = 0; e < 4; e++)
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) rs[sb][e] += __shfl_xor(rs[sb][e], o, kWave);
        const uint32_t src = 16 * ((lane >> 2) & 3u), want = 4 * (lane >> 4) + (lane & 3u);
        uint64_t mine = 0;
#pragma unroll
        for (int sb = 0; sb < 4; sb++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint64_t v = __shfl(rs[sb][e], src, kWave);
                mine = (uint32_t)(4 * sb + e) == want ? v : mine;
            }
        return mine;
    }
    uint64_t sum = 0;
    bool ovf = false;
    if constexpr (MODE == 0) {
        // The accumulators are encoded (D = n - 1). Masks this wide still
        // meet in at most 256 bits in nearly every tile (their members are
        // sparse): a column tile whose 1024 pairs all have D <= 255 takes the
        // packed 16-bit cubic of the narrow masks (exact there), any other
        // tile the 64-bit one. The test is wave-uniform.
#pragma unroll
        for (int tt = 0; tt < 4; tt++) {
            if ((uint32_t)tt >= nt) break;
            const uint32_t j = un.c0 + 16 * tt + r16;
            const bool diag = un.c0 + 16 * tt + 16 > rbase;   // some column j >= some row
            const bool small = !__any(enc_over_255<4>(acc[tt]));
            if (small && !diag) {
                sum += cubic_sum_enc<4>(acc[tt]);
                continue;
            }
            v4i32 d[4];
#pragma unroll
            for (int sb = 0; sb < 4; sb++)
#pragma unroll
                for (int e = 0; e < 4; e++) d[sb][e] = enc_d(acc[tt][sb][e]);
            if (small) {
                sum += cubic_sum<8, 4, true>(d, j, rbase + 4 * g);
            } else {
#pragma unroll
                for (int sb = 0; sb < 4; sb++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        const uint32_t n = j < rbase + 16 * sb + 4 * g + e ? (uint32_t)(d[sb][e] + 1) : 0u;
                        const uint32_t t2 = n * n + 2u - 3u * n;   // (n - 1)(n - 2) mod 2^32, n < 2^16
                        sum += (uint64_t)n * t2;
                    }
            }
        }
        return sum / 6;
    }
#pragma unroll
    for (int tt = 0; tt < 4; tt++) {
        if ((uint32_t)tt >= nt) break;
        const uint32_t j = un.c0 + 16 * tt + r16;
#pragma unroll
        for (int sb = 0; sb < 4; sb++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t n = j < rbase + 16 * sb + 4 * g + e ? (uint32_t)acc[tt][sb][e] : 0u;
                // C(n, q): the table up to kC3Max, computed above it
                sum += n <= kC3Max ? cq[n] : choose_q(n, T.q, ovf);
            }
    }
    if (ovf) atomicOr(&T.ws.ctr->over_cap, 16u);
    return sum;
}

// Two kernels per mode: CLS 0 takes the units of class 0, CLS 1 those of
// classes 1 and 2 (one kernel for the two saves a tail). Waves per SIMD:
// totals of masks up to kSmallW words 4, other totals 3 (both measured
// faster than 3 and 2 in spite of a few spilled registers, reloaded once per
// column tile; the same for totals with q > 3), per-vertex counts of the
// anchor side 2, per-vertex counts of the other side 5.
__host__ __device__ constexpr int tri_waves(int mode, int cls)
{
    return (mode == 0 || mode >= 3) ? (cls == 0 ? 4 : 3) : (mode == 1 ? 2 : 5);
}

template <int MODE, int CLS>
__global__ void __launch_bounds__(kTThreads, tri_waves(MODE, CLS)) k_triplet(TriArgs T)
{
    __shared__ uint32_t c3[kC3Max + 1];
    __shared__ uint64_t cq[MODE >= 3 ? kC3Max + 1 : 1];   // C(n, q), n <= 32 kRegW
    // per wave: column totals of a unit (MODE 1) or totals per anchor position,
    // masks up to kRegW words (MODE 2)
    constexpr uint32_t kLacc = MODE == 1 ? kMaxChunk : (MODE == 2 ? 32 * kRegW : 1);
    __shared__ unsigned long long colacc_all[MODE == 1 || MODE == 2 ? kTThreads / kWave : 1][kLacc];
    for (uint32_t i = threadIdx.x; i <= kC3Max; i += kTThreads) c3[i] = (uint32_t)choose3(i);
    if (MODE >= 3) {
        bool ovf = false;   // C(512, 7) < 2^51
        for (uint32_t i = threadIdx.x; i <= kC3Max; i += kTThreads) cq[i] = choose_q(i, T.q, ovf);
    }
    if (MODE == 1 || MODE == 2)
        for (uint32_t i = threadIdx.x; i < (kTThreads / kWave) * kLacc; i += kTThreads)
            (&colacc_all[0][0])[i] = 0;
    __syncthreads();
    Counters *C = T.ws.ctr;
    if (__atomic_load_n(&C->over_cap, __ATOMIC_RELAXED)) return;
    // class 0, or classes 1 and 2
    const uint32_t u_base = CLS == 0 ? 0u : __atomic_load_n(&C->n_cls_end[0], __ATOMIC_RELAXED);
    const uint32_t u_end = CLS == 0 ? __atomic_load_n(&C->n_cls_end[0], __ATOMIC_RELAXED)
                                    : __atomic_load_n(&C->n_units, __ATOMIC_RELAXED);
    const uint32_t n_units = u_end - u_base;
    Cursor *queue = C->q_tri[CLS];
    const uint32_t lane = __lane_id();
    uint64_t *colacc = (uint64_t *)colacc_all[MODE == 1 || MODE == 2 ? threadIdx.x / kWave : 0];
    uint64_t examined = 0, exwords = 0;
    uint64_t total = 0;
    uint32_t cur_graph = 0xffffffffu;
    uint32_t slice = blockIdx.x % kXcd, tried = 0, qlo = 0, qhi = 0;

    auto flush = [&]() {
        const uint64_t tot = wave_sum<uint64_t>(total);
        if (lane == 0 && tot) {
            const unsigned long long old = atomicAdd(&T.ws.count[cur_graph], (unsigned long long)tot);
            if (old + tot < old) atomicAdd(&T.ws.carry[cur_graph], 1u);
        }
        total = 0;
    };

    for (;;) {
        if (qlo >= qhi) {
            // lane 0 takes the next chunk; readfirstlane keeps every value (and
            // so the loop) wave-uniform, which lets the column loads be scalar
            uint32_t lo = 0, hi = 0, ok = 0;
            if (lane == 0)
                ok = queue_take(queue, n_units, kUnitGrab, &slice, &tried, &lo, &hi) ? 1u : 0u;
            ok = __builtin_amdgcn_readfirstlane(ok);
            if (!ok) break;
            qlo = __builtin_amdgcn_readfirstlane(lo);
            qhi = __builtin_amdgcn_readfirstlane(hi);
            slice = __builtin_amdgcn_readfirstlane(slice);
            tried = __builtin_amdgcn_readfirstlane(tried);
        }
        // from the end of the list: the records of the later pair tiers (the
        // widest masks, the heaviest units) start first
        const uint32_t u = u_base + (n_units - 1 - qlo++);
        Unit un = load_unit(T.ws.units + u);
        AnchorRec a = load_anchor(T.ws.anchors + un.anchor);
        const uint32_t *xm = nullptr, *ym = nullptr;
        if constexpr (MODE == 4) {
            // the triangle of the candidates after x = base - 1, whose mask
            // every row meets: a record of k - base candidates from base on
            const uint32_t base = un.rb >> 16;
            un.rb &= 0xffffu;
            xm = ym = T.ws.masks + a.mask_off + (uint64_t)(base - 1) * a.w32;
            a.k -= base;
            a.mask_off += (uint64_t)base * a.w32;
        } else if constexpr (MODE == 5) {
            // the triangle after y = base - 1, rows meeting the masks of x and y
            const uint32_t base = un.c1, x = un.rb >> 16;
            un.rb &= 0xffffu;
            un.c1 = un.c0 >> 16;
            un.c0 &= 0xffffu;
            xm = T.ws.masks + a.mask_off + (uint64_t)x * a.w32;
            ym = T.ws.masks + a.mask_off + (uint64_t)(base - 1) * a.w32;
            a.k -= base;
            a.mask_off += (uint64_t)base * a.w32;
        }
        if (a.graph != cur_graph) {
            if (cur_graph != 0xffffffffu) flush();
            cur_graph = a.graph;
        }
        uint64_t acc = 0;
        const bool wide = CLS != 0 && a.w32 > kRegW;
        if (wide) {
            if constexpr (CLS != 0) {
                if constexpr (MODE != 2)
                    acc = tri_rows_mfma_wide<MODE>(un, a, T.ws.masks, cq, colacc, T, xm, ym);
                else acc = tri_rows_wide<MODE>(un, a, T.ws.masks, colacc, T, xm, ym);
            }
        } else {
            // only the widths of this kernel's class are instantiated; the
            // fp4 matrix cores for all but the per-vertex counts of the other
            // side
            constexpr bool mc = MODE != 2;
            if (mc && a.w32 <= kMfmaMaxW) {
#define BBC_W(n) case n: acc = tri_rows_fp4<n, MODE>(un, a, T.ws.masks, cq, c3, colacc, xm, ym); break;
                if constexpr (CLS == 0) {
                    switch (a.w32) { BBC_W(1) BBC_W(2) BBC_W(3) BBC_W(4) default: break; }
                } else {
                    switch (a.w32) {
                        BBC_W(5) BBC_W(6) BBC_W(7) BBC_W(8) BBC_W(9) BBC_W(10) BBC_W(11) BBC_W(12)
                        BBC_W(13) BBC_W(14) BBC_W(15) BBC_W(16)
                        default: break;
                    }
                }
#undef BBC_W
            } else {
#define BBC_W(n) case n: acc = tri_rows<n, MODE>(un, a, T.ws.masks, c3, cq, colacc, T); break;
                if constexpr (CLS == 0) {
                    switch (a.w32) { BBC_W(1) BBC_W(2) BBC_W(3) BBC_W(4) default: break; }
                } else {
                    switch (a.w32) {
                        BBC_W(5) BBC_W(6) BBC_W(7) BBC_W(8) BBC_W(9) BBC_W(10) BBC_W(11) BBC_W(12)
                        BBC_W(13) BBC_W(14) BBC_W(15) BBC_W(16)
                        default: break;
                    }
                }
#undef BBC_W
            }
        }
        const uint32_t i = un.rb * kWave + lane;
        if (i < a.k && i > un.c0) {
            const uint32_t ex = min(i, un.c1) - un.c0;
            examined += ex;
            exwords += (uint64_t)ex * a.w32;
        }
        total += acc;
        if (MODE == 2 && !wide) {
            // the unit's totals per anchor position to the opposite vertices
            const uint64_t s0 = T.g.s_off[a.rank];
            const uint32_t d = (uint32_t)(T.g.s_off[a.rank + 1] - s0);
            for (uint32_t p = lane; p < d; p += kWave) {
                const uint64_t v = colacc[p];
                if (v) {
                    atomicAdd(&T.ws.pv_o[T.g.s_adj[s0 + p] >> 1], (unsigned long long)v);
                    colacc[p] = 0;
                }
            }
        }
        if (MODE == 1) {
            // this lane's row total, the anchor's total, and the column totals;
            // candidates are summed in their own slots (only the units of one
            // anchor meet there) and scattered to their vertices once at the end
            if (i < a.k && acc) atomicAdd(&T.ws.pv_slot[a.cand_off + i], (unsigned long long)acc);
            const uint64_t tot = wave_sum<uint64_t>(acc);
            if (lane == 0 && tot) atomicAdd(&T.ws.pv[a.rank], (unsigned long long)tot);
            for (uint32_t c = lane; c < un.c1 - un.c0; c += kWave) {
                const uint64_t v = colacc[c];
                if (v) {
                    atomicAdd(&T.ws.pv_slot[a.cand_off + un.c0 + c], (unsigned long long)v);
                    colacc[c] = 0;
                }
            }
        }
    }
    if (cur_graph != 0xffffffffu) flush();
    examined = wave_sum<uint64_t>(examined);
    exwords = wave_sum<uint64_t>(exwords);
    if (lane == 0 && examined) {
        atomicAdd(&C->pairs_examined, (unsigned long long)examined);
        atomicAdd(&C->pair_words, (unsigned long long)exwords);
    }
}

// Anchor-side per-vertex counts: the candidate slots in use (the cursor of
// the pair tables) are cleared before the triplet kernels and scattered to
// their vertices after them, one atomic per slot. A vertex that is a
// candidate of many anchors then takes one update per anchor and class
// instead of one per unit row and column.
__global__ void __launch_bounds__(256) k_pv_slot_clear(Workspace ws)
{
    const uint64_t n = min((uint64_t)__atomic_load_n(&ws.ctr->cand_cursor, __ATOMIC_RELAXED), ws.cap_cands);
    for (uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (uint64_t)gridDim.x * 256)
        ws.pv_slot[t] = 0;
}

__global__ void __launch_bounds__(256) k_pv_slot_scatter(Workspace ws)
{
    if (__atomic_load_n(&ws.ctr->over_cap, __ATOMIC_RELAXED)) return;
    const uint64_t n = min((uint64_t)__atomic_load_n(&ws.ctr->cand_cursor, __ATOMIC_RELAXED), ws.cap_cands);
    for (uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (uint64_t)gridDim.x * 256) {
        const unsigned long long v = ws.pv_slot[t];
        if (v) atomicAdd(&ws.pv[ws.cands[t]], v);
    }
}

// Per-vertex counts into a caller's device array: out[id[i]] = pv[i] (id
// null: out[i] = pv[i]); a value above 2^63 - 1 sets *bad.
__global__ void __launch_bounds__(256) k_pv_out(const unsigned long long *__restrict__ pv,
                                                 const uint32_t *__restrict__ id, uint32_t n,
                                                 int64_t *__restrict__ out, uint32_t *bad)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const unsigned long long v = pv[i];
        if (v > (unsigned long long)INT64_MAX) atomicOr(bad, 1u);
        out[id ? id[i] : i] = (int64_t)v;
    }
}

}  // namespace

hipError_t per_vertex_to_device(const unsigned long long *pv, const uint32_t *id, uint32_t n,
                                int64_t *out, uint32_t *bad, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const uint32_t grid = std::min<uint32_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pv_out, dim3(grid), dim3(256), 0, s, pv, id, n, out, bad);
    return hipGetLastError();
}

// Tier parameters (LDS use per block: tier A ~ 80 KiB, two blocks per CU;
// tier B ~ 144 KiB).
constexpr int kAThreads = 512, kAH = 8192, kAMaxD = 1024, kAKmax = 1984;
constexpr int kBThreads = 1024, kBH = 16384, kBKmax = 4096;
// per-wave tier: 2048 slots (30 KiB with the slot list) per wave
constexpr int kWvSlots = 2048, kWvWaves = 2;   // waves of a workgroup share its table

uint32_t wave_tier_blocks_per_cu()
{
    return (160u * 1024u) / ((3u * kWvSlots + wave_tier_limit(kWvSlots)) * 4u + 64u);
}
uint32_t wave_tier_waves_per_cu() { return wave_tier_blocks_per_cu() * kWvWaves; }

uint32_t tier_c_max_degree() { return 65535; }
uint32_t window_tier_max_window() { return kRWin; }
uint32_t tier_c_max_k() { return 65535; }
uint32_t max_unit_chunk() { return kMaxChunk; }

template <bool PACKED>
static void launch_pairs(const PairArgs &base, const LaunchShape &sh, hipStream_t s)
{
    PairArgs P = base;
    P.tier = 0;
    hipLaunchKernelGGL((k_pair_wave<kWvSlots, kWvWaves>), dim3(sh.grid_w), dim3(kWvWaves * kWave),
                       0, s, P);
    P.tier = 1;
    hipLaunchKernelGGL((k_pair_lds<kAThreads, kAH, kAMaxD, kAKmax, PACKED>), dim3(sh.grid_a),
                       dim3(kAThreads), 0, s, P);
    P.tier = 2;
    hipLaunchKernelGGL((k_pair_big<kBThreads, kBH, kBKmax, PACKED>), dim3(sh.grid_b),
                       dim3(kBThreads), 0, s, P);
    P.tier = kListR + 1;
    hipLaunchKernelGGL(k_pair_window, dim3(sh.grid_b), dim3(kRThreads), 0, s, P);
    P.tier = 3;
    hipLaunchKernelGGL((k_pair_global<PACKED>), dim3(sh.grid_c), dim3(kGThreads), 0, s, P);
    P.tier = 4;
    hipLaunchKernelGGL((k_pair_global<PACKED>), dim3(sh.grid_d), dim3(kGThreads), 0, s, P);
}

hipError_t count_pairs(const PairArgs &base, const LaunchShape &sh, hipStream_t s)
{
    // packed counting slots need anchor ranks below 2^24 - 1
    if (base.g.NS < kKeyMask) launch_pairs<true>(base, sh, s);
    else launch_pairs<false>(base, sh, s);
    return hipGetLastError();
}

hipError_t count_plan(const Workspace &ws, uint32_t chunk_base, void *tmp, size_t tmp_bytes,
                      uint32_t p, hipStream_t s)
{
    uint32_t grid = (uint32_t)std::min<uint64_t>((ws.cap_anchors + 255) / 256, 4096);
    hipLaunchKernelGGL(k_plan_count, dim3(grid), dim3(256), 0, s, ws, chunk_base, p);
    hipError_t e = scan_u32_to_u64(ws.ucnt, ws.uoff, 3 * ws.cap_anchors, tmp, tmp_bytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_plan_write, dim3(1024), dim3(256), 0, s, ws, chunk_base, p);
    return hipGetLastError();
}

hipError_t count_triplets(const TriArgs &T, int mode, uint32_t grid, hipStream_t s)
{
    // masks of up to 4 words, then the wider ones
    switch (mode) {
        case 0:
            hipLaunchKernelGGL((k_triplet<0, 0>), dim3(grid), dim3(kTThreads), 0, s, T);
            hipLaunchKernelGGL((k_triplet<0, 1>), dim3(grid), dim3(kTThreads), 0, s, T);
            break;
        case 1:
            hipLaunchKernelGGL(k_pv_slot_clear, dim3(grid), dim3(256), 0, s, T.ws);
            hipLaunchKernelGGL((k_triplet<1, 0>), dim3(grid), dim3(kTThreads), 0, s, T);
            hipLaunchKernelGGL((k_triplet<1, 1>), dim3(grid), dim3(kTThreads), 0, s, T);
            hipLaunchKernelGGL(k_pv_slot_scatter, dim3(grid), dim3(256), 0, s, T.ws);
            break;
        case 2:
            hipLaunchKernelGGL((k_triplet<2, 0>), dim3(grid), dim3(kTThreads), 0, s, T);
            hipLaunchKernelGGL((k_triplet<2, 1>), dim3(grid), dim3(kTThreads), 0, s, T);
            break;
        case 3:
            hipLaunchKernelGGL((k_triplet<3, 0>), dim3(grid), dim3(kTThreads), 0, s, T);
            hipLaunchKernelGGL((k_triplet<3, 1>), dim3(grid), dim3(kTThreads), 0, s, T);
            break;
        case 4:
            hipLaunchKernelGGL((k_triplet<4, 0>), dim3(grid), dim3(kTThreads), 0, s, T);
            hipLaunchKernelGGL((k_triplet<4, 1>), dim3(grid), dim3(kTThreads), 0, s, T);
            break;
        default:
            hipLaunchKernelGGL((k_triplet<5, 0>), dim3(grid), dim3(kTThreads), 0, s, T);
            hipLaunchKernelGGL((k_triplet<5, 1>), dim3(grid), dim3(kTThreads), 0, s, T);
            break;
    }
    return hipGetLastError();
}

}  // namespace bbc
