// count.hip -- the counting kernels: signed pair table and triplet
// intersection, for balanced (3,3)-bicliques.
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
// C(|M_u2^c2 n M_u3^c3|, 3). This kernel pair therefore works on "virtual
// candidates" (w, c): a class set M_w^c with at least 3 members (a smaller
// one cannot reach C(.,3) > 0 -- this is the pair prune of Algorithm 2 split
// by sign class). Two virtual candidates of the same w never share a member
// (M_w^+ and M_w^- are disjoint), so every unordered pair of virtual
// candidates may be paired without excluding same-w pairs:
//     contribution(u1) = sum over pairs {x, y} of C(|M_x n M_y|, 3).
// M_x is a bitmask over the positions of N(u1); |M_x n M_y| is an AND and a
// popcount per 32-bit word.
//
// k_pair (the signed pair table, Algorithm 2's cnt map split by sign class):
//   per anchor, 2-hop walk over the higher-priority part of each neighbour
//   list, counting (same, different) per partner in an LDS hash table; keep
//   the classes with >= 3; a second walk sets the mask bits; emit masks and
//   work units. Three tiers: LDS tables of 4096 and 16384 slots, then tables
//   in global memory for the anchors that overflow them.
// k_triplet (Algorithm 2's loop over pairs A of C with T = intersection and
//   the type histogram): one wave per work unit of 64 rows x up to a few
//   hundred columns of an anchor's lower-triangular pair matrix; row masks in
//   VGPRs, column masks through scalar loads (wave-uniform), C(n,3) from an
//   LDS table, 64-bit accumulation, one atomic per unit.
#include "bbc_count.h"

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
constexpr uint32_t kC3Max = 512;   // C(n,3) table covers masks of up to 16 words

__device__ __forceinline__ uint32_t hash_slot(uint32_t x, int log2h)
{
    return (x * 0x9E3779B1u) >> (32 - log2h);
}

// Insert-or-add into an open-addressing table (linear probing). Returns
// false when the table is too full (the anchor goes to the next tier).
__device__ __forceinline__ void hash_add(uint32_t *keys, uint32_t *vals, uint32_t H, int log2h,
                                         uint32_t x, uint32_t inc, uint32_t *used, uint32_t limit,
                                         volatile uint32_t *over)
{
    uint32_t h = hash_slot(x, log2h);
    for (uint32_t probe = 0; probe < H; probe++) {
        uint32_t k = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
        if (k == x) { atomicAdd(&vals[h], inc); return; }
        if (k == kEmpty) {
            uint32_t old = atomicCAS(&keys[h], kEmpty, x);
            if (old == kEmpty) {
                if (atomicAdd(used, 1u) >= limit) *over = 1;
                atomicAdd(&vals[h], inc);
                return;
            }
            if (old == x) { atomicAdd(&vals[h], inc); return; }
        }
        h = (h + 1) & (H - 1);
        if (*over) return;
    }
    *over = 1;
}

// Slot of a key known to be present; H if absent (never expected).
__device__ __forceinline__ uint32_t hash_find(const uint32_t *keys, uint32_t H, int log2h,
                                              uint32_t x)
{
    uint32_t h = hash_slot(x, log2h);
    for (uint32_t probe = 0; probe < H; probe++) {
        if (keys[h] == x) return h;
        h = (h + 1) & (H - 1);
    }
    return H;
}

__device__ __forceinline__ uint32_t unit_chunk(uint32_t w32, uint32_t base)
{
    uint32_t c = base / w32;
    c = c < 32 ? 32 : c;
    return (c + 7) & ~7u;
}

struct PairShared {
    uint32_t item, over, used, nv, skip, aidx, uoff, nunits, wedges;
    unsigned long long moff, coff;
};

// The per-anchor procedure shared by all tiers. Table storage is passed as
// pointers (LDS arrays for tiers A and B, global memory for tier C).
template <int THREADS>
__device__ __forceinline__ void pair_loop(const PairArgs &P, uint32_t *keys, uint32_t *vals,
                                          const uint32_t H, const int log2h, uint32_t *pst,
                                          uint32_t *pln, const uint32_t maxd, uint32_t *vc,
                                          const uint32_t kmax, uint32_t *msk,
                                          const uint32_t maskw, uint32_t *bpre, PairShared &sh)
{
    constexpr int NW = THREADS / kWave;
    const int tid = threadIdx.x, lane = __lane_id(), wv = tid / kWave;
    const CsrView &g = P.g;
    Counters *C = P.ws.ctr;
    const uint32_t limit = H - H / 4;
    uint64_t my_wedges = 0;

    for (uint32_t i = tid; i < H; i += THREADS) { keys[i] = kEmpty; vals[i] = 0; }
    const uint32_t n_items =
        P.tier ? (uint32_t)min((uint64_t)__atomic_load_n(&C->n_list[P.tier - 1], __ATOMIC_RELAXED),
                               P.ws.cap_defer)
               : P.a1 - P.a0;
    const uint32_t *list = P.tier ? P.ws.defer[P.tier - 1] : nullptr;
    uint32_t *next_list = P.tier < 2 ? P.ws.defer[P.tier] : nullptr;

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            sh.item = atomicAdd(&C->next[P.tier], 1u);
            sh.over = 0; sh.used = 0; sh.nv = 0; sh.skip = 0; sh.wedges = 0;
        }
        __syncthreads();
        const uint32_t item = sh.item;
        if (item >= n_items) break;
        const uint32_t r = list ? list[item] : P.a0 + item;
        const uint64_t s0 = g.s_off[r];
        const uint32_t d = (uint32_t)(g.s_off[r + 1] - s0);
        if (d < 3) continue;
        if (d > maxd) {
            if (tid == 0) {
                if (next_list) {
                    uint32_t t = atomicAdd(&C->n_list[P.tier], 1u);
                    if (t < P.ws.cap_defer) next_list[t] = r; else atomicOr(&C->over_cap, 1u);
                } else {
                    atomicOr(&C->over_cap, 4u);
                }
            }
            continue;
        }
        // phase 0: the part of each neighbour list above the anchor's rank
        for (uint32_t p = tid; p < d; p += THREADS) {
            const uint32_t e = g.s_adj[s0 + p];
            const uint32_t v = e >> 1;
            uint64_t lo = g.o_off[v];
            const uint64_t hi = g.o_off[v + 1];
            const uint32_t target = (r + 1) << 1;
            uint64_t b = hi;
            while (lo < b) {
                uint64_t mid = (lo + b) >> 1;
                if (g.o_adj[mid] < target) lo = mid + 1; else b = mid;
            }
            uint32_t len = (uint32_t)(hi - lo);
            if (len < 2) len = 0;   // v needs 2 higher partners to lie in any T
            pst[p] = (uint32_t)lo;
            pln[p] = len | ((e & 1u) << 31);
            if (len) atomicAdd(&sh.wedges, len);
        }
        __syncthreads();
        if (sh.wedges < 6) continue;   // fewer than 2 classes of 3 are impossible
        // phase 1: (same, different) counts per higher-priority partner
        for (uint32_t p = wv; p < d; p += NW) {
            const uint32_t ln = pln[p];
            const uint32_t len = ln & 0x7fffffffu;
            if (!len) continue;
            const uint32_t st = pst[p], sg = ln >> 31;
            my_wedges += lane < len ? (len - lane + kWave - 1) / kWave : 0;
            for (uint32_t j = lane; j < len; j += kWave) {
                const uint32_t e2 = g.o_adj[st + j];
                hash_add(keys, vals, H, log2h, e2 >> 1, ((e2 & 1u) ^ sg) ? 0x10000u : 1u,
                         &sh.used, limit, &sh.over);
            }
            if (__atomic_load_n(&sh.over, __ATOMIC_RELAXED)) break;
        }
        __syncthreads();
        bool defer = sh.over != 0;
        // phase 2: classes with >= 3 members become virtual candidates
        if (!defer) {
            for (uint32_t slot = tid; slot < H; slot += THREADS) {
                const uint32_t k = keys[slot];
                if (k == kEmpty) continue;
                const uint32_t v = vals[slot];
                uint32_t is = 0, id = 0;
                if ((v & 0xffffu) >= 3) {
                    uint32_t t = atomicAdd(&sh.nv, 1u);
                    if (t < kmax) vc[t] = k;
                    is = t + 1;
                }
                if ((v >> 16) >= 3) {
                    uint32_t t = atomicAdd(&sh.nv, 1u);
                    if (t < kmax) vc[t] = k;
                    id = t + 1;
                }
                vals[slot] = (is & 0xffffu) | (id << 16);
            }
            __syncthreads();
            defer = sh.nv > kmax;
        }
        if (defer) {
            if (tid == 0) {
                if (next_list) {
                    uint32_t t = atomicAdd(&C->n_list[P.tier], 1u);
                    if (t < P.ws.cap_defer) next_list[t] = r; else atomicOr(&C->over_cap, 1u);
                } else {
                    atomicOr(&C->over_cap, 4u);
                }
            }
            for (uint32_t i = tid; i < H; i += THREADS) { keys[i] = kEmpty; vals[i] = 0; }
            continue;
        }
        const uint32_t k = sh.nv;
        if (k < 2) {
            for (uint32_t i = tid; i < H; i += THREADS) { keys[i] = kEmpty; vals[i] = 0; }
            continue;
        }
        const uint32_t W = (d + 31) >> 5;
        const uint64_t words = (uint64_t)k * W;
        const uint32_t CH = unit_chunk(W, P.chunk_base);
        const uint32_t nb = (k + kWave - 1) / kWave;
        if (tid == 0) {
            uint32_t tot = 0;
            for (uint32_t b = 0; b < nb; b++) {
                bpre[b] = tot;
                uint32_t ncols = min(kWave * (b + 1), k) - 1;
                tot += (ncols + CH - 1) / CH;
            }
            bpre[nb] = tot;
            sh.nunits = tot;
            sh.moff = atomicAdd(&C->mask_cursor, (unsigned long long)words);
            sh.coff = atomicAdd(&C->cand_cursor, (unsigned long long)k);
            sh.aidx = atomicAdd(&C->n_anchor, 1u);
            sh.uoff = atomicAdd(&C->n_units, tot);
            atomicAdd(&C->pairs, (unsigned long long)k * (k - 1) / 2);
            bool bad = sh.moff + words > P.ws.cap_mask_words || sh.coff + k > P.ws.cap_cands ||
                       sh.aidx >= P.ws.cap_anchors || (uint64_t)sh.uoff + tot > P.ws.cap_units;
            sh.skip = bad;
            if (bad) atomicOr(&C->over_cap, 2u);
        }
        __syncthreads();
        if (sh.skip) {
            for (uint32_t i = tid; i < H; i += THREADS) { keys[i] = kEmpty; vals[i] = 0; }
            continue;
        }
        const bool in_lds = words <= maskw;
        uint32_t *mp = in_lds ? msk : P.ws.masks + sh.moff;
        for (uint64_t i = tid; i < words; i += THREADS) mp[i] = 0;
        if (!in_lds) __threadfence();
        __syncthreads();
        // phase 3: bit p of M_(w,c) for every higher-priority wedge through position p
        for (uint32_t p = wv; p < d; p += NW) {
            const uint32_t ln = pln[p];
            const uint32_t len = ln & 0x7fffffffu;
            if (!len) continue;
            const uint32_t st = pst[p], sg = ln >> 31;
            for (uint32_t j = lane; j < len; j += kWave) {
                const uint32_t e2 = g.o_adj[st + j];
                const uint32_t h = hash_find(keys, H, log2h, e2 >> 1);
                if (h == H) { atomicOr(&C->over_cap, 8u); continue; }
                const uint32_t v = vals[h];
                const uint32_t idx = ((e2 & 1u) ^ sg) ? (v >> 16) : (v & 0xffffu);
                if (idx) atomicOr(&mp[(uint64_t)(idx - 1) * W + (p >> 5)], 1u << (p & 31));
            }
        }
        __syncthreads();
        const uint64_t moff = sh.moff, coff = sh.coff;
        if (in_lds)
            for (uint64_t i = tid; i < words; i += THREADS) P.ws.masks[moff + i] = msk[i];
        for (uint32_t i = tid; i < k; i += THREADS) P.ws.cands[coff + i] = vc[i];
        if (tid == 0) {
            AnchorRec a;
            a.rank = r; a.k = k; a.w32 = W; a.graph = g.s_graph[r];
            a.mask_off = moff; a.cand_off = coff;
            P.ws.anchors[sh.aidx] = a;
        }
        const uint32_t nunits = sh.nunits, uoff = sh.uoff, aidx = sh.aidx;
        for (uint32_t u = tid; u < nunits; u += THREADS) {
            uint32_t lo = 0, hi = nb;   // largest b with bpre[b] <= u
            while (hi - lo > 1) {
                uint32_t mid = (lo + hi) >> 1;
                if (bpre[mid] <= u) lo = mid; else hi = mid;
            }
            const uint32_t c = u - bpre[lo];
            const uint32_t ncols = min(kWave * (lo + 1), k) - 1;
            Unit un;
            un.anchor = aidx; un.rb = lo; un.c0 = c * CH; un.c1 = min(un.c0 + CH, ncols);
            P.ws.units[uoff + u] = un;
        }
        for (uint32_t i = tid; i < H; i += THREADS) { keys[i] = kEmpty; vals[i] = 0; }
    }
    my_wedges = wave_sum<uint64_t>(my_wedges);
    if (lane == 0 && my_wedges) atomicAdd(&C->wedges, (unsigned long long)my_wedges);
}

template <int THREADS, int H, int LOG2H, int MAXD, int KMAX, int MASKW>
__global__ void __launch_bounds__(THREADS) k_pair_lds(PairArgs P)
{
    __shared__ uint32_t keys[H], vals[H], pst[MAXD], pln[MAXD], vc[KMAX], msk[MASKW];
    __shared__ uint32_t bpre[KMAX / kWave + 2];
    __shared__ PairShared sh;
    pair_loop<THREADS>(P, keys, vals, H, LOG2H, pst, pln, MAXD, vc, KMAX, msk, MASKW, bpre, sh);
}

constexpr int kGThreads = 1024;

__global__ void __launch_bounds__(kGThreads) k_pair_global(PairArgs P)
{
    __shared__ uint32_t bpre[65536 / kWave + 2];
    __shared__ PairShared sh;
    uint32_t *base = P.ws.gtab + (uint64_t)blockIdx.x * P.ws.gtab_words_per_block;
    const uint32_t H = P.gH;
    uint32_t *keys = base;
    uint32_t *vals = keys + H;
    uint32_t *pst = vals + H;
    uint32_t *pln = pst + P.gmaxd;
    uint32_t *vc = pln + P.gmaxd;
    pair_loop<kGThreads>(P, keys, vals, H, P.glog2h, pst, pln, P.gmaxd, vc, P.gkmax, nullptr, 0,
                         bpre, sh);
}

// ------------------------------------------------------------ triplets
struct TriCtx {
    const uint32_t *masks;
    const uint32_t *c3;
    uint32_t i;        // this lane's row
    bool vi;
};

template <int W>
__device__ __forceinline__ uint64_t tri_rows(const Unit &un, const AnchorRec &a,
                                             const uint32_t *__restrict__ masks,
                                             const uint32_t *c3, uint64_t *colacc, int mode,
                                             const TriArgs &T)
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
    if (mode == 0) {
        for (; j + 8 <= un.c1; j += 8) {
            uint32_t s = 0;
#pragma unroll
            for (int jj = 0; jj < 8; jj++) {
                uint32_t n = 0;
#pragma unroll
                for (int w = 0; w < W; w++) n += __popc(row[w] & MS[(uint64_t)(j + jj) * W + w]);
                uint32_t t = c3[n];
                if (diag) t = (j + jj < i) ? t : 0u;
                s += t;
            }
            acc += s;
        }
        for (; j < un.c1; j++) {
            uint32_t n = 0;
#pragma unroll
            for (int w = 0; w < W; w++) n += __popc(row[w] & MS[(uint64_t)j * W + w]);
            uint32_t t = c3[n];
            if (diag) t = (j < i) ? t : 0u;
            acc += t;
        }
        return acc;
    }
    // per-vertex modes
    for (; j < un.c1; j++) {
        uint32_t cw[W];
        uint32_t n = 0;
#pragma unroll
        for (int w = 0; w < W; w++) {
            cw[w] = MS[(uint64_t)j * W + w];
            n += __popc(row[w] & cw[w]);
        }
        uint32_t t = c3[n];
        if (diag) t = (j < i) ? t : 0u;
        acc += t;
        if (t) {
            if (mode == 1) {
                atomicAdd((unsigned long long *)&colacc[j - un.c0], (unsigned long long)t);
            } else {
                // every member of the common class is in C(n-1, 2) of these bicliques
                const uint64_t each = choose2(n - 1);
                const uint64_t s0 = T.g.s_off[a.rank];
#pragma unroll
                for (int w = 0; w < W; w++) {
                    uint32_t m = row[w] & cw[w];
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
    return acc;
}

// Masks wider than 16 words: row words are re-read per column.
__device__ uint64_t tri_rows_wide(const Unit &un, const AnchorRec &a,
                                  const uint32_t *__restrict__ masks, uint64_t *colacc, int mode,
                                  const TriArgs &T)
{
    const uint32_t lane = __lane_id();
    const uint32_t i = un.rb * kWave + lane;
    const bool vi = i < a.k;
    const uint32_t W = a.w32;
    const uint32_t *M = masks + a.mask_off;
    const BBC_CONST uint32_t *MS = as_const(M);
    const bool diag = un.c1 > un.rb * kWave;
    uint64_t acc = 0;
    for (uint32_t j = un.c0; j < un.c1; j++) {
        uint32_t n = 0;
        if (vi)
            for (uint32_t w = 0; w < W; w++)
                n += __popc(M[(uint64_t)i * W + w] & MS[(uint64_t)j * W + w]);
        uint64_t t = choose3(n);
        if (diag && !(j < i)) t = 0;
        acc += t;
        if (t && mode == 1) atomicAdd((unsigned long long *)&colacc[j - un.c0], (unsigned long long)t);
        if (t && mode == 2) {
            const uint64_t each = choose2(n - 1);
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
    return acc;
}

constexpr int kTThreads = 256;
constexpr uint32_t kMaxChunk = 2048;

template <int MODE>
__global__ void __launch_bounds__(kTThreads) k_triplet(TriArgs T)
{
    __shared__ uint32_t c3[kC3Max + 1];
    __shared__ unsigned long long colacc_all[MODE == 1 ? kTThreads / kWave : 1][MODE == 1 ? kMaxChunk : 1];
    for (uint32_t i = threadIdx.x; i <= kC3Max; i += kTThreads) c3[i] = (uint32_t)choose3(i);
    if (MODE == 1)
        for (uint32_t i = threadIdx.x; i < (kTThreads / kWave) * kMaxChunk; i += kTThreads)
            (&colacc_all[0][0])[i] = 0;
    __syncthreads();
    Counters *C = T.ws.ctr;
    if (__atomic_load_n(&C->over_cap, __ATOMIC_RELAXED)) return;
    const uint32_t n_units = __atomic_load_n(&C->n_units, __ATOMIC_RELAXED);
    const uint32_t lane = __lane_id();
    uint64_t *colacc = (uint64_t *)colacc_all[MODE == 1 ? threadIdx.x / kWave : 0];
    uint64_t examined = 0;
    for (;;) {
        uint32_t u = 0;
        if (lane == 0) u = atomicAdd(&C->unit_next, 1u);
        u = __builtin_amdgcn_readfirstlane(u);
        if (u >= n_units) break;
        const Unit un = load_unit(T.ws.units + u);
        const AnchorRec a = load_anchor(T.ws.anchors + un.anchor);
        uint64_t acc;
        switch (a.w32) {
#define BBC_W(n) case n: acc = tri_rows<n>(un, a, T.ws.masks, c3, colacc, MODE, T); break;
            BBC_W(1) BBC_W(2) BBC_W(3) BBC_W(4) BBC_W(5) BBC_W(6) BBC_W(7) BBC_W(8)
            BBC_W(9) BBC_W(10) BBC_W(11) BBC_W(12) BBC_W(13) BBC_W(14) BBC_W(15) BBC_W(16)
#undef BBC_W
            default: acc = tri_rows_wide(un, a, T.ws.masks, colacc, MODE, T); break;
        }
        {
            const uint32_t i = un.rb * kWave + lane;
            if (i < a.k && i > un.c0) examined += min(i, un.c1) - un.c0;
        }
        if (MODE == 1) {
            // this lane's row total, the anchor's total, and the column totals
            const uint32_t i = un.rb * kWave + lane;
            if (i < a.k && acc)
                atomicAdd(&T.ws.pv[T.ws.cands[a.cand_off + i]], (unsigned long long)acc);
            const uint64_t tot = wave_sum<uint64_t>(acc);
            if (lane == 0 && tot) atomicAdd(&T.ws.pv[a.rank], (unsigned long long)tot);
            for (uint32_t c = lane; c < un.c1 - un.c0; c += kWave) {
                const uint64_t v = colacc[c];
                if (v) {
                    atomicAdd(&T.ws.pv[T.ws.cands[a.cand_off + un.c0 + c]], (unsigned long long)v);
                    colacc[c] = 0;
                }
            }
        }
        const uint64_t tot = wave_sum<uint64_t>(acc);
        if (lane == 0 && tot) {
            const unsigned long long old = atomicAdd(&T.ws.count[a.graph], (unsigned long long)tot);
            if (old + tot < old) atomicAdd(&T.ws.carry[a.graph], 1u);
        }
    }
    examined = wave_sum<uint64_t>(examined);
    if (lane == 0 && examined) atomicAdd(&C->pairs_examined, (unsigned long long)examined);
}

}  // namespace

// Tier parameters (LDS use per block: tier A ~ 64 KiB, tier B ~ 152 KiB).
constexpr int kAThreads = 512, kAH = 4096, kALog = 12, kAMaxD = 1024, kAKmax = 2048, kAMaskW = 4096;
constexpr int kBThreads = 1024, kBH = 16384, kBLog = 14, kBMaxD = 1024, kBKmax = 4096, kBMaskW = 1;

uint32_t tier_c_max_degree() { return 65535; }
uint32_t tier_c_max_k() { return 65535; }

hipError_t count_pairs(const PairArgs &base, const LaunchShape &sh, hipStream_t s)
{
    PairArgs P = base;
    P.tier = 0;
    hipLaunchKernelGGL((k_pair_lds<kAThreads, kAH, kALog, kAMaxD, kAKmax, kAMaskW>),
                       dim3(sh.grid_a), dim3(kAThreads), 0, s, P);
    P.tier = 1;
    hipLaunchKernelGGL((k_pair_lds<kBThreads, kBH, kBLog, kBMaxD, kBKmax, kBMaskW>),
                       dim3(sh.grid_b), dim3(kBThreads), 0, s, P);
    if (sh.grid_c) {
        P.tier = 2;
        hipLaunchKernelGGL(k_pair_global, dim3(sh.grid_c), dim3(kGThreads), 0, s, P);
    }
    return hipGetLastError();
}

hipError_t count_triplets(const TriArgs &T, int mode, uint32_t grid, hipStream_t s)
{
    if (mode == 0) hipLaunchKernelGGL(k_triplet<0>, dim3(grid), dim3(kTThreads), 0, s, T);
    else if (mode == 1) hipLaunchKernelGGL(k_triplet<1>, dim3(grid), dim3(kTThreads), 0, s, T);
    else hipLaunchKernelGGL(k_triplet<2>, dim3(grid), dim3(kTThreads), 0, s, T);
    return hipGetLastError();
}

uint32_t max_unit_chunk() { return kMaxChunk; }

}  // namespace bbc
