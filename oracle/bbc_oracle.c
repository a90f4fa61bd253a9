/*
 * bbc_oracle.c -- plain CPU oracle for balanced (3,3)-biclique counting.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The product path (the
 * HIP library) never calls it, shares no code, header or table with it, and
 * must fail loudly when its own extension is missing.
 *
 * Paper: "Counting Small Balanced (p,q)-bicliques in Signed Bipartite Graphs"
 * (arXiv 2605.03603). Everything here is for p = q = 3 unless a function says
 * otherwise (the _q and _pq variants take a general q, or p and q), in exact
 * integer arithmetic (128-bit accumulators), written as plain loops so that
 * it can be checked against the paper by eye.
 *
 *   orc_butterfly_balanced   Section 1 (Fig. 2): a butterfly is balanced iff it
 *                            has an even number of negative edges.
 *   orc_wedge_type           Section 4.1 (signed p-wedge type, Fig. 3(b)):
 *                            c_i = s iff sign(u1,v) == sign(v,w_i).
 *   orc_count_bruteforce     Section 3 definitions (butterfly, balanced
 *                            biclique, balanced (p,q)-biclique, problem
 *                            statement) taken literally: every 3x3 vertex
 *                            subset, 9 edges present, 9 butterflies balanced.
 *   orc_count_bbvp           Algorithm 2 (BBVP, Section 4.2) with p = q = 3,
 *                            steps in the paper's order: anchor side S, cnt
 *                            over higher-priority 2-hop vertices, candidate
 *                            set C, lists L[w] = Gamma(u) n Gamma(w), pairs
 *                            A of C, T = intersection, type histogram x,
 *                            b += sum_kappa C(x[kappa], 3).
 *   orc_vertex_count         the same per-anchor steps without the priority
 *                            filter: the number of balanced (3,3)-bicliques
 *                            that contain one given vertex.
 *   orc_count_bbvp_q         Algorithm 2 with p = 3 on the anchor side and a
 *                            general q (3..7) on the other: prune cnt >= q,
 *                            skip |T| < q, add C(x[kappa], q).
 *   orc_count_bruteforce_pq  the definitions for general (p, q): every p x q
 *                            vertex subset, all edges present, every butterfly
 *                            balanced (totals only).
 *
 * Readings of points the paper leaves open:
 *   - vertex priority (Definition 4.1): higher degree first, equal degree
 *     broken by the larger input id;
 *   - the anchor side: the caller picks U, V, or the smaller partition as the
 *     paper does (side = -1);
 *   - the pair prune keeps w when cnt[w] >= q (unsigned, as in Algorithm 2).
 * Edge signs are int8 +1 / -1 (the paper's datasets write + as 1 and - as 0).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

/* Planted mistakes for the oracle's own mutation test: the test suite builds
 * this file with -DORC_MUTANT=k (k > 0) and checks that its pins reject every
 * variant. The default build (0) is the oracle. */
#ifndef ORC_MUTANT
#define ORC_MUTANT 0
#endif

/* ------------------------------------------------------------------ basics */

/* Fig. 2: balanced <=> even number of negative edges <=> sign product = +1. */
int orc_butterfly_balanced(int s1, int s2, int s3, int s4)
{
    int neg = (s1 < 0) + (s2 < 0) + (s3 < 0) + (s4 < 0);
#if ORC_MUTANT == 1
    return (neg % 2) == 1;
#endif
    return (neg % 2) == 0;
}

/* Section 4.1: type of the signed 3-wedge <u1, w1, w2, v>. Returns a 2-bit
 * code: bit 1 is c_1, bit 0 is c_2, each 0 for 's' (same sign as (u1,v)) and 1
 * for 'd'. So ss = 0, sd = 1, ds = 2, dd = 3. */
int orc_wedge_type(int s_u1v, int s_w1v, int s_w2v)
{
    int c1 = (s_u1v == s_w1v) ? 0 : 1;
    int c2 = (s_u1v == s_w2v) ? 0 : 1;
#if ORC_MUTANT == 2
    c2 = (s_w1v == s_w2v) ? 0 : 1;
#endif
    return (c1 << 1) | c2;
}

static uint64_t choose3(uint64_t n)
{
    if (n < 3) return 0;
#if ORC_MUTANT == 3
    return (n - 1) * (n - 2) / 2 * (n - 3) / 3;
#endif
    return n * (n - 1) / 2 * (n - 2) / 3;
}

uint64_t orc_choose3(uint64_t n) { return choose3(n); }

/* C(n, k) exactly: after step i, c = C(n, i + 1), and c * (n - i) is always
 * divisible by i + 1. */
static i128 choose_k(uint64_t n, int k)
{
    if ((uint64_t)k > n) return 0;
    i128 c = 1;
    for (int i = 0; i < k; i++) c = c * (i128)(n - (uint64_t)i) / (i + 1);
    return c;
}

/* ----------------------------------------------------- O1: the definition */

/* Count balanced (3,3)-bicliques of a tiny graph straight from the
 * definitions. L has 3 vertices of U, R has 3 vertices of V; (L,R) counts when
 * all 9 edges exist and every butterfly (2 of L x 2 of R) is balanced.
 * Also fills per-vertex counts (number of counted bicliques containing the
 * vertex) when the arrays are non-NULL. Returns -1 if the graph is too big
 * (n_u or n_v above 24) or an edge is repeated or out of range. */
int orc_count_bruteforce(int n_u, int n_v, int64_t m, const uint32_t *eu, const uint32_t *ev,
                         const int8_t *sign, uint64_t *out_total, int64_t *per_u, int64_t *per_v)
{
    if (n_u < 0 || n_v < 0 || n_u > 24 || n_v > 24) return -1;
    int8_t s[24][24];
    memset(s, 0, sizeof(s));
    for (int64_t e = 0; e < m; e++) {
        if (eu[e] >= (uint32_t)n_u || ev[e] >= (uint32_t)n_v) return -1;
        if (s[eu[e]][ev[e]] != 0) return -1;
        s[eu[e]][ev[e]] = sign[e];
    }
    if (per_u) for (int i = 0; i < n_u; i++) per_u[i] = 0;
    if (per_v) for (int i = 0; i < n_v; i++) per_v[i] = 0;
    uint64_t total = 0;
    for (int a = 0; a < n_u; a++)
    for (int b = a + 1; b < n_u; b++)
    for (int c = b + 1; c < n_u; c++) {
        int L[3] = {a, b, c};
        for (int x = 0; x < n_v; x++)
        for (int y = x + 1; y < n_v; y++)
        for (int z = y + 1; z < n_v; z++) {
            int R[3] = {x, y, z};
            int ok = 1;
            for (int i = 0; i < 3 && ok; i++)
                for (int j = 0; j < 3 && ok; j++)
                    if (s[L[i]][R[j]] == 0 && !(ORC_MUTANT == 8 && i == 2 && j == 2))
                        ok = 0;                              /* cohesiveness */
            for (int i = 0; i < 3 && ok; i++)
            for (int i2 = i + 1; i2 < 3 && ok; i2++)
            for (int j = 0; j < 3 && ok; j++)
            for (int j2 = j + 1; j2 < 3 && ok; j2++)
                if (!orc_butterfly_balanced(s[L[i]][R[j]], s[L[i]][R[j2]],
                                            s[L[i2]][R[j]], s[L[i2]][R[j2]]))
                    ok = 0;                                  /* balance */
            if (ok) {
                total++;
                if (per_u) { per_u[a]++; per_u[b]++; per_u[c]++; }
                if (per_v) { per_v[x]++; per_v[y]++; per_v[z]++; }
            }
        }
    }
    *out_total = total;
    return 0;
}

/* The definitions for general (p, q), totals only: every p-subset L of U and
 * q-subset R of V (in lexicographic order) counts when all p*q edges exist and
 * every butterfly of L x R is balanced. Tiny graphs only (sides up to 24, p
 * and q up to 8). Returns -1 on bad input. */
int orc_count_bruteforce_pq(int n_u, int n_v, int64_t m, const uint32_t *eu, const uint32_t *ev,
                            const int8_t *sign, int p, int q, uint64_t *out_total)
{
    if (n_u < 0 || n_v < 0 || n_u > 24 || n_v > 24 || p < 1 || q < 1 || p > 8 || q > 8) return -1;
    int8_t s[24][24];
    memset(s, 0, sizeof(s));
    for (int64_t e = 0; e < m; e++) {
        if (eu[e] >= (uint32_t)n_u || ev[e] >= (uint32_t)n_v) return -1;
        if (s[eu[e]][ev[e]] != 0) return -1;
        s[eu[e]][ev[e]] = sign[e];
    }
    uint64_t total = 0;
    *out_total = 0;
    if (p > n_u || q > n_v) return 0;
    int L[8], R[8];
    for (int i = 0; i < p; i++) L[i] = i;
    for (;;) {
        for (int j = 0; j < q; j++) R[j] = j;
        for (;;) {
            int ok = 1;
            for (int i = 0; i < p && ok; i++)
                for (int j = 0; j < q && ok; j++)
                    if (s[L[i]][R[j]] == 0) ok = 0;                 /* cohesiveness */
            for (int i = 0; i < p && ok; i++)
            for (int i2 = i + 1; i2 < p && ok; i2++)
            for (int j = 0; j < q && ok; j++)
            for (int j2 = j + 1; j2 < q && ok; j2++)
                if (!orc_butterfly_balanced(s[L[i]][R[j]], s[L[i]][R[j2]],
                                            s[L[i2]][R[j]], s[L[i2]][R[j2]]))
                    ok = 0;                                         /* balance */
            total += (uint64_t)ok;
            /* next q-subset of V */
            int j = q - 1;
            while (j >= 0 && R[j] == n_v - q + j) j--;
            if (j < 0) break;
            R[j]++;
            for (int j2 = j + 1; j2 < q; j2++) R[j2] = R[j2 - 1] + 1;
        }
        /* next p-subset of U */
        int i = p - 1;
        while (i >= 0 && L[i] == n_u - p + i) i--;
        if (i < 0) break;
        L[i]++;
        for (int i2 = i + 1; i2 < p; i2++) L[i2] = L[i2 - 1] + 1;
    }
    *out_total = total;
    return 0;
}

/* ------------------------------------------------------- adjacency lists */

typedef struct {
    int64_t n_s, n_o;          /* anchor side S, opposite side */
    int64_t *off_s, *off_o;    /* n+1 offsets */
    uint32_t *adj_s, *adj_o;   /* Gamma(s) as opposite ids (sorted), Gamma(o) as S ids */
    int8_t *sg_s, *sg_o;       /* edge signs aligned with adj_s / adj_o */
    int64_t *deg_s;
} graph_t;

static int cmp_pair(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Build both adjacency orientations; side_is_v selects S = V. Lists are
 * sorted by neighbour id. Returns -1 on a repeated or out-of-range edge. */
static int build_graph(graph_t *g, int64_t n_u, int64_t n_v, int64_t m, const uint32_t *eu,
                       const uint32_t *ev, const int8_t *sign, int side_is_v)
{
    memset(g, 0, sizeof(*g));
    g->n_s = side_is_v ? n_v : n_u;
    g->n_o = side_is_v ? n_u : n_v;
    uint64_t *key = malloc(sizeof(uint64_t) * (m > 0 ? m : 1));
    int64_t *idx = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
    g->off_s = calloc(g->n_s + 1, sizeof(int64_t));
    g->off_o = calloc(g->n_o + 1, sizeof(int64_t));
    g->adj_s = malloc(sizeof(uint32_t) * (m > 0 ? m : 1));
    g->adj_o = malloc(sizeof(uint32_t) * (m > 0 ? m : 1));
    g->sg_s = malloc(m > 0 ? m : 1);
    g->sg_o = malloc(m > 0 ? m : 1);
    g->deg_s = calloc(g->n_s + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) {
        if ((int64_t)eu[e] >= n_u || (int64_t)ev[e] >= n_v) goto fail;
        uint64_t s = side_is_v ? ev[e] : eu[e];
        uint64_t o = side_is_v ? eu[e] : ev[e];
        key[e] = (s << 32) | o;
    }
    /* sort edge keys (S id, opposite id) to get sorted S lists and to find repeats */
    {
        uint64_t *ke = malloc(sizeof(uint64_t) * 2 * (m > 0 ? m : 1));
        for (int64_t e = 0; e < m; e++) { ke[2 * e] = key[e]; ke[2 * e + 1] = (uint64_t)e; }
        qsort(ke, m, 2 * sizeof(uint64_t), cmp_pair);
        for (int64_t e = 0; e < m; e++) idx[e] = (int64_t)ke[2 * e + 1];
        free(ke);
    }
    for (int64_t e = 1; e < m; e++)
        if (key[idx[e]] == key[idx[e - 1]]) goto fail;
    for (int64_t e = 0; e < m; e++) {
        uint64_t s = key[e] >> 32, o = key[e] & 0xffffffffu;
        g->off_s[s + 1]++;
        g->off_o[o + 1]++;
    }
    for (int64_t i = 0; i < g->n_s; i++) { g->deg_s[i] = g->off_s[i + 1]; g->off_s[i + 1] += g->off_s[i]; }
    for (int64_t i = 0; i < g->n_o; i++) g->off_o[i + 1] += g->off_o[i];
    {
        int64_t *fill_o = calloc(g->n_o + 1, sizeof(int64_t));
        /* walking edges in (S id, opposite id) order leaves every opposite
         * list sorted by S id as well */
        for (int64_t t = 0; t < m; t++) {
            int64_t e = idx[t];
            uint64_t s = key[e] >> 32, o = key[e] & 0xffffffffu;
            g->adj_s[t] = (uint32_t)o;
            g->sg_s[t] = sign[e];
            int64_t p = g->off_o[o] + fill_o[o]++;
            g->adj_o[p] = (uint32_t)s;
            g->sg_o[p] = sign[e];
        }
        free(fill_o);
    }
    free(key); free(idx);
    return 0;
fail:
    free(key); free(idx);
    return -1;
}

static void free_graph(graph_t *g)
{
    free(g->off_s); free(g->off_o); free(g->adj_s); free(g->adj_o);
    free(g->sg_s); free(g->sg_o); free(g->deg_s);
}

/* Definition 4.1: rho(a) > rho(b) iff deg(a) > deg(b), or equal degree and
 * id(a) > id(b). */
static int higher_priority(const graph_t *g, uint32_t a, uint32_t b)
{
    if (g->deg_s[a] != g->deg_s[b]) return g->deg_s[a] > g->deg_s[b];
    return a > b;
}

/* --------------------------------------------- O2: Algorithm 2, p = q = 3 */

typedef struct {
    int32_t *cnt;        /* cnt map of Algorithm 2, dense over S, reset after use */
    uint32_t *touched;   /* S vertices with cnt != 0 */
    uint32_t *cand;      /* candidate set C */
    int64_t *l_off;      /* L[w] stored as (position in Gamma(u), sign(u,v), sign(w,v)) */
    int32_t *l_pos;
    int8_t *l_su, *l_sw;
    int64_t l_cap;
    int8_t *mark;        /* per position of Gamma(u): sign(w1,v) while L[w1] is marked, else 0 */
} scratch_t;

typedef struct {
    i128 total;
    uint64_t feasible;   /* pairs A with |T| >= q (survivors of the |T| < q test) */
    uint64_t candidates; /* pairs A enumerated from C */
} tally_t;

/* Optional watch list of opposite-side vertices. A balanced (3,3)-biclique
 * found at anchor u from the pair (w1, w2) takes its three opposite vertices
 * from one wedge-type class of T (Lemma 1), so a watched vertex v of T in the
 * class of x_k members lies in C(x_k - 1, 2) of the C(x_k, 3) bicliques of
 * that class. Summed over all anchors and pairs, this is the number of
 * balanced (3,3)-bicliques that contain v. */
typedef struct {
    const int32_t *idx;  /* per opposite vertex: its index in the watch list, or -1 */
    i128 *tally;         /* per watched vertex (this thread's part) */
    int32_t *hit;        /* scratch: (watch index, wedge type) of the watched members of T */
} watch_t;

/* Optional record of one anchor's intermediate values (for the worked
 * example of Fig. 4): the candidate set C and, for every pair A of C, |T| and
 * the type histogram x. */
typedef struct {
    int64_t cap_c, n_c;
    uint32_t *cand;
    int64_t cap_pairs, n_pairs;
    int64_t *pairs;      /* per pair: w1, w2, |T|, x_ss, x_sd, x_ds, x_dd */
} trace_t;

static void scratch_init(scratch_t *w, const graph_t *g)
{
    w->cnt = calloc(g->n_s + 1, sizeof(int32_t));
    w->touched = malloc(sizeof(uint32_t) * (g->n_s + 1));
    w->cand = malloc(sizeof(uint32_t) * (g->n_s + 1));
    w->l_off = malloc(sizeof(int64_t) * (g->n_s + 2));
    w->l_cap = 1024;
    w->l_pos = malloc(sizeof(int32_t) * w->l_cap);
    w->l_su = malloc(w->l_cap);
    w->l_sw = malloc(w->l_cap);
    int64_t max_d = 0;
    for (int64_t i = 0; i < g->n_s; i++)
        if (g->off_s[i + 1] - g->off_s[i] > max_d) max_d = g->off_s[i + 1] - g->off_s[i];
    w->mark = calloc(max_d + 1, 1);
}

static void scratch_free(scratch_t *w)
{
    free(w->cnt); free(w->touched); free(w->cand); free(w->l_off);
    free(w->l_pos); free(w->l_su); free(w->l_sw); free(w->mark);
}

/* One anchor u of Algorithm 2. With oriented != 0 only partners of higher
 * priority are used (each biclique is then counted at its lowest-priority S
 * vertex); with oriented == 0 every other S vertex is a partner, which counts
 * every balanced biclique containing u exactly once. per_s (optional) gets
 * each counted biclique's contribution added to u, w1 and w2. */
static void bbvp_anchor(const graph_t *g, uint32_t u, int oriented, scratch_t *w, tally_t *t,
                        i128 *per_s, trace_t *tr, int q, watch_t *wt)
{
#if ORC_MUTANT == 4
    const int q_prune = q + 1;
#else
    const int q_prune = q;
#endif
    /* cnt[w] = |Gamma(u) n Gamma(w)| over w in S with rho(w) > rho(u) */
    int64_t n_touched = 0;
    for (int64_t a = g->off_s[u]; a < g->off_s[u + 1]; a++) {
        uint32_t v = g->adj_s[a];
        for (int64_t b = g->off_o[v]; b < g->off_o[v + 1]; b++) {
            uint32_t x = g->adj_o[b];
            if (x == u) continue;
            if (oriented && !higher_priority(g, x, u)) continue;
#if ORC_MUTANT == 9
            if (oriented && g->deg_s[x] == g->deg_s[u]) continue;
#endif
            if (w->cnt[x] == 0) w->touched[n_touched++] = x;
            w->cnt[x]++;
        }
    }
    /* C = { w : cnt[w] >= q } */
    int64_t n_c = 0;
    for (int64_t i = 0; i < n_touched; i++)
        if (w->cnt[w->touched[i]] >= q_prune) w->cand[n_c++] = w->touched[i];
    for (int64_t i = 0; i < n_touched; i++) w->cnt[w->touched[i]] = 0;
    if (tr) {
        tr->n_c = n_c;
        for (int64_t i = 0; i < n_c && i < tr->cap_c; i++) tr->cand[i] = w->cand[i];
    }
    if (n_c < 2) return;      /* |C| < p - 1 */

    /* L[w] = Gamma(u) n Gamma(w), as sorted positions in Gamma(u), by a merge
     * of the two sorted neighbour lists */
    int64_t need = 0;
    for (int64_t i = 0; i < n_c; i++) {
        int64_t du = g->off_s[u + 1] - g->off_s[u];
        int64_t dw = g->off_s[w->cand[i] + 1] - g->off_s[w->cand[i]];
        need += du < dw ? du : dw;
    }
    if (need > w->l_cap) {
        w->l_cap = need;
        w->l_pos = realloc(w->l_pos, sizeof(int32_t) * need);
        w->l_su = realloc(w->l_su, need);
        w->l_sw = realloc(w->l_sw, need);
    }
    int64_t fill = 0;
    for (int64_t i = 0; i < n_c; i++) {
        uint32_t x = w->cand[i];
        w->l_off[i] = fill;
        int64_t a = g->off_s[u], ae = g->off_s[u + 1];
        int64_t b = g->off_s[x], be = g->off_s[x + 1];
        while (a < ae && b < be) {
            if (g->adj_s[a] < g->adj_s[b]) a++;
            else if (g->adj_s[a] > g->adj_s[b]) b++;
            else {
                w->l_pos[fill] = (int32_t)(a - g->off_s[u]);
                w->l_su[fill] = g->sg_s[a];
                w->l_sw[fill] = g->sg_s[b];
                fill++; a++; b++;
            }
        }
    }
    w->l_off[n_c] = fill;

    /* every pair A = (w1, w2) of C: T = L[w1] n L[w2]. The positions of
     * L[w1] are marked (with sign(w1, v)) in an array over Gamma(u); each
     * entry of L[w2] then looks its position up, and a marked one is a common
     * neighbour v with its wedge type. */
    for (int64_t i = 0; i < n_c; i++) {
        for (int64_t a = w->l_off[i]; a < w->l_off[i + 1]; a++) w->mark[w->l_pos[a]] = w->l_sw[a];
        for (int64_t j = i + 1; j < n_c; j++) {
            t->candidates++;
            uint64_t x[4] = {0, 0, 0, 0};
            uint64_t size_t_ = 0;
            int64_t n_hit = 0;
            for (int64_t b = w->l_off[j]; b < w->l_off[j + 1]; b++) {
                const int8_t s_w1v = w->mark[w->l_pos[b]];
                if (!s_w1v) continue;   /* v not in L[w1] */
#if ORC_MUTANT == 6
                int kappa = orc_wedge_type(w->l_su[b], s_w1v, s_w1v);
#else
                int kappa = orc_wedge_type(w->l_su[b], s_w1v, w->l_sw[b]);
#endif
                x[kappa]++;
                size_t_++;
                if (wt) {
                    const int32_t h = wt->idx[g->adj_s[g->off_s[u] + w->l_pos[b]]];
                    if (h >= 0) { wt->hit[2 * n_hit] = h; wt->hit[2 * n_hit + 1] = kappa; n_hit++; }
                }
            }
            if (tr && tr->n_pairs < tr->cap_pairs) {
                int64_t *r = tr->pairs + 7 * tr->n_pairs++;
                r[0] = w->cand[i]; r[1] = w->cand[j]; r[2] = (int64_t)size_t_;
                for (int k = 0; k < 4; k++) r[3 + k] = (int64_t)x[k];
            }
            if (size_t_ < (uint64_t)q) continue;   /* |T| < q */
            t->feasible++;
            i128 add = 0;
#if ORC_MUTANT == 5
            for (int k = 0; k < 3; k++) add += q == 3 ? (i128)choose3(x[k]) : choose_k(x[k], q);
#else
            for (int k = 0; k < 4; k++) add += q == 3 ? (i128)choose3(x[k]) : choose_k(x[k], q);
#endif
            t->total += add;
            for (int64_t h = 0; h < n_hit; h++) {
                const uint64_t r = x[wt->hit[2 * h + 1]] - 1;   /* the other members of v's class */
                wt->tally[wt->hit[2 * h]] += (i128)(r * (r - (r > 0)) / 2);
            }
            if (per_s && add) {
                per_s[u] += add;
                per_s[w->cand[i]] += add;
#if ORC_MUTANT == 7
                per_s[u] += add;
#else
                per_s[w->cand[j]] += add;
#endif
            }
        }
        for (int64_t a = w->l_off[i]; a < w->l_off[i + 1]; a++) w->mark[w->l_pos[a]] = 0;
    }
}

/* One anchor u of Algorithm 2 with p = 4 on the anchor side: the candidate
 * set C and the lists L[w] as for p = 3, then every 3-subset A = {w1, w2, w3}
 * of C (the (p - 1)-subsets of the algorithm): T = L[w1] n L[w2] n L[w3], and
 * each v in T falls in one of the 2^3 classes given by the three products
 * s(u, v) s(wi, v) (the wedge types of the pairs (u, wi) at v); the subset adds
 * C(x_c, q) over the classes. Oriented (partners of higher priority) only. */
static void bbvp_anchor_p4(const graph_t *g, uint32_t u, scratch_t *w, tally_t *t, int q)
{
    int64_t n_touched = 0;
    for (int64_t a = g->off_s[u]; a < g->off_s[u + 1]; a++) {
        uint32_t v = g->adj_s[a];
        for (int64_t b = g->off_o[v]; b < g->off_o[v + 1]; b++) {
            uint32_t x = g->adj_o[b];
            if (x == u || !higher_priority(g, x, u)) continue;
            if (w->cnt[x] == 0) w->touched[n_touched++] = x;
            w->cnt[x]++;
        }
    }
    int64_t n_c = 0;
    for (int64_t i = 0; i < n_touched; i++)
        if (w->cnt[w->touched[i]] >= q) w->cand[n_c++] = w->touched[i];
    for (int64_t i = 0; i < n_touched; i++) w->cnt[w->touched[i]] = 0;
    if (n_c < 3) return;      /* |C| < p - 1 */
    int64_t need = 0;
    for (int64_t i = 0; i < n_c; i++) {
        int64_t du = g->off_s[u + 1] - g->off_s[u];
        int64_t dw = g->off_s[w->cand[i] + 1] - g->off_s[w->cand[i]];
        need += du < dw ? du : dw;
    }
    if (need > w->l_cap) {
        w->l_cap = need;
        w->l_pos = realloc(w->l_pos, sizeof(int32_t) * need);
        w->l_su = realloc(w->l_su, need);
        w->l_sw = realloc(w->l_sw, need);
    }
    int64_t fill = 0;
    for (int64_t i = 0; i < n_c; i++) {
        uint32_t x = w->cand[i];
        w->l_off[i] = fill;
        int64_t a = g->off_s[u], ae = g->off_s[u + 1];
        int64_t b = g->off_s[x], be = g->off_s[x + 1];
        while (a < ae && b < be) {
            if (g->adj_s[a] < g->adj_s[b]) a++;
            else if (g->adj_s[a] > g->adj_s[b]) b++;
            else {
                w->l_pos[fill] = (int32_t)(a - g->off_s[u]);
                w->l_su[fill] = g->sg_s[a];
                w->l_sw[fill] = g->sg_s[b];
                fill++; a++; b++;
            }
        }
    }
    w->l_off[n_c] = fill;
    for (int64_t i = 0; i < n_c; i++)
        for (int64_t j = i + 1; j < n_c; j++)
            for (int64_t k = j + 1; k < n_c; k++) {
                t->candidates++;
                uint64_t x[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                uint64_t size_t_ = 0;
                int64_t a = w->l_off[i], ae = w->l_off[i + 1];
                int64_t b = w->l_off[j], be = w->l_off[j + 1];
                int64_t c = w->l_off[k], ce = w->l_off[k + 1];
                while (a < ae && b < be && c < ce) {
                    const int32_t pa = w->l_pos[a], pb = w->l_pos[b], pc = w->l_pos[c];
                    if (pa == pb && pb == pc) {
                        const int su = w->l_su[a];
                        const int cls = (su * w->l_sw[a] < 0) | ((su * w->l_sw[b] < 0) << 1) |
                                        ((su * w->l_sw[c] < 0) << 2);
                        x[cls]++;
                        size_t_++;
                        a++; b++; c++;
                    } else {
                        const int32_t mx = pa > pb ? (pa > pc ? pa : pc) : (pb > pc ? pb : pc);
                        if (pa < mx) a++;
                        if (pb < mx) b++;
                        if (pc < mx) c++;
                    }
                }
                if (size_t_ < (uint64_t)q) continue;   /* |T| < q */
                t->feasible++;
                for (int cl = 0; cl < 8; cl++) t->total += choose_k(x[cl], q);
            }
}

/* One anchor u of Algorithm 2 with p - 1 = r partners (p = 4 or 5), in the
 * plainest form: the candidate set C as above, then for every candidate w a
 * dense vector over the positions of Gamma(u) holding 0 (w not adjacent) or
 * the product s(u, v) s(w, v); every r-subset A of C walks the positions, and
 * a position where all of A is adjacent falls in the class given by the signs
 * of the r products (2^r classes); the subset adds C(x_c, q) over the
 * classes. Oriented (partners of higher priority) only. */
static void bbvp_anchor_dense(const graph_t *g, uint32_t u, scratch_t *w, tally_t *t, int p, int q)
{
    const int r = p - 1;
    int64_t n_touched = 0;
    for (int64_t a = g->off_s[u]; a < g->off_s[u + 1]; a++) {
        uint32_t v = g->adj_s[a];
        for (int64_t b = g->off_o[v]; b < g->off_o[v + 1]; b++) {
            uint32_t x = g->adj_o[b];
            if (x == u || !higher_priority(g, x, u)) continue;
            if (w->cnt[x] == 0) w->touched[n_touched++] = x;
            w->cnt[x]++;
        }
    }
    int64_t n_c = 0;
    for (int64_t i = 0; i < n_touched; i++)
        if (w->cnt[w->touched[i]] >= q) w->cand[n_c++] = w->touched[i];
    for (int64_t i = 0; i < n_touched; i++) w->cnt[w->touched[i]] = 0;
    if (n_c < r) return;
    const int64_t du = g->off_s[u + 1] - g->off_s[u];
    int8_t *vec = calloc((size_t)(n_c * du + 1), 1);
    for (int64_t i = 0; i < n_c; i++) {
        const uint32_t x = w->cand[i];
        int64_t a = g->off_s[u], ae = g->off_s[u + 1];
        int64_t b = g->off_s[x], be = g->off_s[x + 1];
        while (a < ae && b < be) {
            if (g->adj_s[a] < g->adj_s[b]) a++;
            else if (g->adj_s[a] > g->adj_s[b]) b++;
            else {
                vec[i * du + (a - g->off_s[u])] = (int8_t)(g->sg_s[a] * g->sg_s[b]);
                a++; b++;
            }
        }
    }
    int64_t A[4];
    for (int k = 0; k < r; k++) A[k] = k;
    for (;;) {
        t->candidates++;
        uint64_t x[16];
        memset(x, 0, sizeof(x));
        uint64_t size_t_ = 0;
        for (int64_t pos = 0; pos < du; pos++) {
            int cls = 0, all = 1;
            for (int k = 0; k < r && all; k++) {
                const int8_t e = vec[A[k] * du + pos];
                if (e == 0) all = 0;
                else if (e < 0) cls |= 1 << k;
            }
            if (all) { x[cls]++; size_t_++; }
        }
        if (size_t_ >= (uint64_t)q) {
            t->feasible++;
            for (int c = 0; c < (1 << r); c++) t->total += choose_k(x[c], q);
        }
        /* next r-subset of C */
        int k = r - 1;
        while (k >= 0 && A[k] == n_c - r + k) k--;
        if (k < 0) break;
        A[k]++;
        for (int k2 = k + 1; k2 < r; k2++) A[k2] = A[k2 - 1] + 1;
    }
    free(vec);
}

typedef struct {
    const graph_t *g;
    int64_t next;            /* shared anchor cursor (dynamic chunks) */
    pthread_mutex_t lock;
    int64_t stride;          /* process anchors whose index is residue modulo stride */
    int64_t residue;
    int want_per_vertex;
    int p, q;
    tally_t tally;
    i128 *per_s;             /* shared per-vertex, merged under the lock */
    const int32_t *watch_idx;  /* optional watch list (watch_t), NULL for none */
    int64_t n_watch;
    i128 *watch_tally;       /* merged under the lock */
    const uint8_t *anchor_on;  /* optional: only anchors u with anchor_on[u] != 0 */
} job_t;

static void *worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    const graph_t *g = jb->g;
    scratch_t w;
    scratch_init(&w, g);
    tally_t t = {0, 0, 0};
    i128 *per = NULL;
    if (jb->want_per_vertex) per = calloc(g->n_s + 1, sizeof(i128));
    watch_t wv, *wt = NULL;
    if (jb->watch_idx) {
        wv.idx = jb->watch_idx;
        wv.tally = calloc(jb->n_watch + 1, sizeof(i128));
        wv.hit = malloc(sizeof(int32_t) * 2 * (jb->n_watch + 1));
        wt = &wv;
    }
    const int64_t chunk = 64;
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        int64_t begin = jb->next;
        jb->next += chunk;
        pthread_mutex_unlock(&jb->lock);
        if (begin >= g->n_s) break;
        int64_t end = begin + chunk < g->n_s ? begin + chunk : g->n_s;
        for (int64_t u = begin; u < end; u++) {
            if (u % jb->stride != jb->residue) continue;
            if (jb->anchor_on && !jb->anchor_on[u]) continue;
            if (jb->p == 4) bbvp_anchor_p4(g, (uint32_t)u, &w, &t, jb->q);
            else if (jb->p > 4 || jb->p < 0) bbvp_anchor_dense(g, (uint32_t)u, &w, &t, jb->p < 0 ? -jb->p : jb->p, jb->q);
            else bbvp_anchor(g, (uint32_t)u, 1, &w, &t, per, NULL, jb->q, wt);
        }
    }
    pthread_mutex_lock(&jb->lock);
    jb->tally.total += t.total;
    jb->tally.feasible += t.feasible;
    jb->tally.candidates += t.candidates;
    if (per) for (int64_t i = 0; i < g->n_s; i++) jb->per_s[i] += per[i];
    if (wt) for (int64_t i = 0; i < jb->n_watch; i++) jb->watch_tally[i] += wt->tally[i];
    pthread_mutex_unlock(&jb->lock);
    free(per);
    if (wt) { free(wv.tally); free(wv.hit); }
    scratch_free(&w);
    return NULL;
}

/* Algorithm 2 (BBVP) with p = 3 on the anchor side and q (3..7) on the other
 * (orc_count_bbvp: q = 3). A balanced (p, 3)-biclique of G is a balanced
 * (3, p)-biclique of G with the sides exchanged, so side = 1 with q = p counts
 * (p, 3).
 *   side: 0 anchors on U, 1 on V, -1 on the smaller partition (the paper's
 *         choice; U when equal).
 *   n_threads: worker threads over anchors (dynamic chunks of 64).
 *   anchor_stride: 1 for the whole count; k > 1 keeps only anchors whose id is
 *         a multiple of k (a bounded sample for timing).
 *   (orc_count_bbvp_shard takes a residue r as well and keeps the anchors
 *   whose id is r modulo k: the k shards r = 0..k-1 partition the anchors, so
 *   their totals, statistics and per-vertex arrays add up to the whole count.)
 *   out_total: the count as a 128-bit integer, little-endian words lo, hi.
 *   out_stats: [feasible triples (|T| >= 3), candidate pairs of C, side used].
 *   per_vertex: optional int64 per vertex of the side used.
 * Returns 0, -1 on a bad edge list or q, -2 if a per-vertex value exceeds int64. */
static int count_bbvp_part(int64_t n_u, int64_t n_v, int64_t m, const uint32_t *eu,
                           const uint32_t *ev, const int8_t *sign, int side, int n_threads,
                           int64_t anchor_stride, int64_t residue, int q, uint64_t *out_total,
                           uint64_t *out_stats, int64_t *per_vertex, int64_t n_watch,
                           const uint32_t *watch, const uint8_t *anchor_on, uint64_t *watch_out)
{
    if (q < 3 || q > 7) return -1;
    if (anchor_stride < 1) anchor_stride = 1;
    if (residue < 0 || residue >= anchor_stride) return -1;
    if (side < 0) side = (n_v < n_u) ? 1 : 0;
    graph_t g;
    if (build_graph(&g, n_u, n_v, m, eu, ev, sign, side) != 0) { free_graph(&g); return -1; }
    if (n_threads < 1) n_threads = 1;
    job_t jb;
    memset(&jb, 0, sizeof(jb));
    jb.g = &g;
    jb.stride = anchor_stride;
    jb.residue = residue;
    jb.want_per_vertex = per_vertex != NULL;
    jb.p = 3;
    jb.q = q;
    pthread_mutex_init(&jb.lock, NULL);
    if (per_vertex) jb.per_s = calloc(g.n_s + 1, sizeof(i128));
    int32_t *widx = NULL;
    if (watch && n_watch > 0) {
        widx = malloc(sizeof(int32_t) * (g.n_o + 1));
        for (int64_t i = 0; i < g.n_o; i++) widx[i] = -1;
        for (int64_t i = 0; i < n_watch; i++) {
            if ((int64_t)watch[i] >= g.n_o || widx[watch[i]] >= 0) { free(widx); free(jb.per_s); free_graph(&g); return -1; }
            widx[watch[i]] = (int32_t)i;
        }
        jb.watch_idx = widx;
        jb.n_watch = n_watch;
        jb.watch_tally = calloc(n_watch, sizeof(i128));
    }
    jb.anchor_on = anchor_on;
    pthread_t *th = malloc(sizeof(pthread_t) * n_threads);
    for (int i = 0; i < n_threads; i++) pthread_create(&th[i], NULL, worker, &jb);
    for (int i = 0; i < n_threads; i++) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&jb.lock);
    int rc = 0;
    if (widx) {
        for (int64_t i = 0; i < n_watch; i++) {
            watch_out[2 * i] = (uint64_t)jb.watch_tally[i];
            watch_out[2 * i + 1] = (uint64_t)(jb.watch_tally[i] >> 64);
        }
        free(jb.watch_tally);
        free(widx);
    }
    out_total[0] = (uint64_t)jb.tally.total;
    out_total[1] = (uint64_t)(jb.tally.total >> 64);
    if (out_stats) {
        out_stats[0] = jb.tally.feasible;
        out_stats[1] = jb.tally.candidates;
        out_stats[2] = (uint64_t)side;
    }
    if (per_vertex) {
        for (int64_t i = 0; i < g.n_s; i++) {
            if (jb.per_s[i] > (i128)INT64_MAX) rc = -2;
            per_vertex[i] = (int64_t)jb.per_s[i];
        }
        free(jb.per_s);
    }
    free_graph(&g);
    return rc;
}

/* Algorithm 2 with p = 4 or 5 on the anchor side and q (3..7) on the other
 * (side 0: balanced (p, q)-bicliques, anchored on U; side 1: balanced
 * (q, p)-bicliques, anchored on V). p = 4 intersects the L lists by merges,
 * p = 5 (and p = -4, the same count as p = 4) walks dense sign vectors.
 * out_total: 128-bit count, words lo, hi; out_stats: [subsets with |T| >= q,
 * (p - 1)-subsets of C enumerated]. Returns 0, or -1 on a bad edge list, p
 * or q. */
int orc_count_bbvp_pk(int64_t n_u, int64_t n_v, int64_t m, const uint32_t *eu,
                      const uint32_t *ev, const int8_t *sign, int side, int n_threads, int p,
                      int q, uint64_t *out_total, uint64_t *out_stats)
{
    if (q < 3 || q > 7 || (side != 0 && side != 1)) return -1;
    if (p != 4 && p != 5 && p != -4) return -1;
    graph_t g;
    if (build_graph(&g, n_u, n_v, m, eu, ev, sign, side) != 0) { free_graph(&g); return -1; }
    if (n_threads < 1) n_threads = 1;
    job_t jb;
    memset(&jb, 0, sizeof(jb));
    jb.g = &g;
    jb.stride = 1;
    jb.p = p;
    jb.q = q;
    pthread_mutex_init(&jb.lock, NULL);
    pthread_t *th = malloc(sizeof(pthread_t) * n_threads);
    for (int i = 0; i < n_threads; i++) pthread_create(&th[i], NULL, worker, &jb);
    for (int i = 0; i < n_threads; i++) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&jb.lock);
    out_total[0] = (uint64_t)jb.tally.total;
    out_total[1] = (uint64_t)(jb.tally.total >> 64);
    if (out_stats) {
        out_stats[0] = jb.tally.feasible;
        out_stats[1] = jb.tally.candidates;
    }
    free_graph(&g);
    return 0;
}

int orc_count_bbvp_q(int64_t n_u, int64_t n_v, int64_t m, const uint32_t *eu,
                     const uint32_t *ev, const int8_t *sign, int side, int n_threads,
                     int64_t anchor_stride, int q, uint64_t *out_total, uint64_t *out_stats,
                     int64_t *per_vertex)
{
    return count_bbvp_part(n_u, n_v, m, eu, ev, sign, side, n_threads, anchor_stride, 0, q,
                           out_total, out_stats, per_vertex, 0, NULL, NULL, NULL);
}

int orc_count_bbvp_shard(int64_t n_u, int64_t n_v, int64_t m, const uint32_t *eu,
                         const uint32_t *ev, const int8_t *sign, int side, int n_threads,
                         int64_t n_shards, int64_t shard, uint64_t *out_total,
                         uint64_t *out_stats, int64_t *per_vertex)
{
    return count_bbvp_part(n_u, n_v, m, eu, ev, sign, side, n_threads, n_shards, shard, 3,
                           out_total, out_stats, per_vertex, 0, NULL, NULL, NULL);
}

/* orc_count_bbvp_shard with a watch list of n_watch distinct opposite-side
 * vertices (watch_t): watch_out gets, per watched vertex, the number of
 * balanced (3,3)-bicliques that contain it and whose anchor is in this shard
 * (128-bit, words lo, hi). anchor_on (optional, one byte per anchor-side
 * vertex) skips the anchors it marks 0; a biclique that contains a watched
 * vertex v is anchored at a neighbour of v, so keeping the neighbours of the
 * watched vertices keeps every contribution to watch_out. Returns 0, or -1
 * on a bad edge list, shard or watch list. */
int orc_count_bbvp_watch(int64_t n_u, int64_t n_v, int64_t m, const uint32_t *eu,
                         const uint32_t *ev, const int8_t *sign, int side, int n_threads,
                         int64_t n_shards, int64_t shard, int64_t n_watch, const uint32_t *watch,
                         const uint8_t *anchor_on, uint64_t *out_total, uint64_t *out_stats,
                         uint64_t *watch_out)
{
    if (side != 0 && side != 1) return -1;
    if (n_watch < 1 || !watch || !watch_out) return -1;
    return count_bbvp_part(n_u, n_v, m, eu, ev, sign, side, n_threads, n_shards, shard, 3,
                           out_total, out_stats, NULL, n_watch, watch, anchor_on, watch_out);
}

int orc_count_bbvp(int64_t n_u, int64_t n_v, int64_t m, const uint32_t *eu, const uint32_t *ev,
                   const int8_t *sign, int side, int n_threads, int64_t anchor_stride,
                   uint64_t *out_total, uint64_t *out_stats, int64_t *per_vertex)
{
    return orc_count_bbvp_q(n_u, n_v, m, eu, ev, sign, side, n_threads, anchor_stride, 3,
                            out_total, out_stats, per_vertex);
}

/* Number of balanced (3,3)-bicliques that contain vertex x of the given side
 * (0 = U, 1 = V): the per-anchor steps of Algorithm 2 with every other vertex
 * of the side as a partner. out_count gets lo, hi words of the 128-bit value.
 * Builds the adjacency once per call; xs lists n_x vertices to evaluate. */
int orc_vertex_counts(int64_t n_u, int64_t n_v, int64_t m, const uint32_t *eu, const uint32_t *ev,
                      const int8_t *sign, int side, int64_t n_x, const uint32_t *xs,
                      uint64_t *out_counts)
{
    graph_t g;
    if (build_graph(&g, n_u, n_v, m, eu, ev, sign, side) != 0) { free_graph(&g); return -1; }
    scratch_t w;
    scratch_init(&w, &g);
    int rc = 0;
    for (int64_t i = 0; i < n_x; i++) {
        if ((int64_t)xs[i] >= g.n_s) { rc = -1; break; }
        tally_t t = {0, 0, 0};
        bbvp_anchor(&g, xs[i], 0, &w, &t, NULL, NULL, 3, NULL);
        out_counts[2 * i] = (uint64_t)t.total;
        out_counts[2 * i + 1] = (uint64_t)(t.total >> 64);
    }
    scratch_free(&w);
    free_graph(&g);
    return rc;
}

/* Intermediate values of Algorithm 2 at one anchor u (side 0 = U, 1 = V):
 * fills the candidate set C (sorted by vertex id is not guaranteed; the order
 * is the order of first discovery) and, for every pair of C, the record
 * (w1, w2, |T|, x_ss, x_sd, x_ds, x_dd). oriented selects the priority filter
 * rho(w) > rho(u). Returns 0 or -1. */
int orc_anchor_detail(int64_t n_u, int64_t n_v, int64_t m, const uint32_t *eu, const uint32_t *ev,
                      const int8_t *sign, int side, uint32_t u, int oriented,
                      int64_t cap_c, uint32_t *cand, int64_t *n_cand,
                      int64_t cap_pairs, int64_t *pairs, int64_t *n_pairs, uint64_t *out_total)
{
    graph_t g;
    if (build_graph(&g, n_u, n_v, m, eu, ev, sign, side) != 0) { free_graph(&g); return -1; }
    if ((int64_t)u >= g.n_s) { free_graph(&g); return -1; }
    scratch_t w;
    scratch_init(&w, &g);
    trace_t tr = {cap_c, 0, cand, cap_pairs, 0, pairs};
    tally_t t = {0, 0, 0};
    bbvp_anchor(&g, u, oriented, &w, &t, NULL, &tr, 3, NULL);
    *n_cand = tr.n_c;
    *n_pairs = tr.n_pairs;
    out_total[0] = (uint64_t)t.total;
    out_total[1] = (uint64_t)(t.total >> 64);
    scratch_free(&w);
    free_graph(&g);
    return 0;
}
