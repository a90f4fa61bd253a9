/*
 * bbc.h -- C ABI of libbbc: exact counting of balanced (3,3)-bicliques in
 * signed bipartite graphs on an AMD MI355X (gfx950) GPU.
 *
 * Problem (Section 3 of "Counting Small Balanced (p,q)-bicliques in Signed
 * Bipartite Graphs", arXiv 2605.03603): G = (U, V, E) with E a subset of
 * U x V and a sign +1 or -1 on every edge. A (p,q)-biclique (L, R) has
 * |L| = p vertices of one side and |R| = q of the other, all p*q edges
 * present; it is balanced when none of its butterflies (2x2 sub-bicliques)
 * has an odd number of negative edges (Section 1, Fig. 2). The library
 * returns the number of balanced (p,q)-bicliques: (3,3) everywhere, and for
 * global counts 3, 4 or 5 vertices on the graph's anchor side with 3..7 on
 * the other (bbc_count_global).
 *
 * Method (Section 4, Lemma 1 and Algorithm 2): every same-side triple
 * {u1,u2,u3} is visited once, from its lowest-priority vertex (priority:
 * higher degree first, ties by the larger id; Definition 4.1); each common
 * neighbour v is put in one of 4 classes by (s(u1,v)s(u2,v), s(u1,v)s(u3,v));
 * the triple adds sum over classes of C(n_class, 3).
 *
 * Conventions for every call:
 *   - Every call returns a bbc_status; out-parameters are written only on
 *     BBC_OK.
 *   - Input arrays are borrowed for the duration of the call; the library
 *     copies what it keeps. With BBC_IN_DEVICE_PTRS they are device pointers
 *     on the context's device, otherwise host pointers.
 *   - Validation errors are reported before any count is produced. A HIP
 *     runtime failure returns BBC_E_HIP and bbc_last_error() holds the detail.
 *   - A context is used by one thread at a time, except bbc_submit*,
 *     bbc_poll and bbc_wait, which may be called from any thread.
 *   - Degenerate inputs (fewer than 3 vertices on a side, no edges, isolated
 *     vertices) are valid and count 0.
 */
#ifndef BBC_H
#define BBC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BBC_OK = 0,
    BBC_E_INVAL = 1,         /* null pointer, bad flag combination or size */
    BBC_E_RANGE = 2,         /* an edge endpoint u >= n_u or v >= n_v */
    BBC_E_SIGN = 3,          /* a sign that is not +1 / -1 (or 1 / 0 with BBC_SIGNS_01) */
    BBC_E_DUP_EDGE = 4,      /* the same (u, v) pair twice (E is a set) */
    BBC_E_NOMEM = 5,         /* device memory, or the context's memory cap */
    BBC_E_OVERFLOW = 6,      /* a count does not fit in int64 */
    BBC_E_UNSUPPORTED = 7,   /* a (p, q) or size the call does not support */
    BBC_E_NOT_READY = 8,     /* bbc_poll: the request is still queued or running */
    BBC_E_UNKNOWN_TICKET = 9,
    BBC_E_HIP = 10           /* HIP runtime error; see bbc_last_error */
} bbc_status;

typedef struct bbc_ctx bbc_ctx;
typedef struct bbc_graph bbc_graph;
typedef uint64_t bbc_ticket;

/* Flags of bbc_build_csr / bbc_build_csr_batch / bbc_submit_coo. */
#define BBC_IN_DEVICE_PTRS    (1u << 0)  /* eu, ev, sign are device pointers */
#define BBC_SIGNS_2BIT_PACKED (1u << 1)  /* sign holds 2-bit codes, 4 per byte, edge e in
                                            bits 2*(e%4)..: 01 = +1, 11 = -1 (00, 10 invalid) */
#define BBC_SIGNS_01          (1u << 2)  /* int8 signs 1 = +, 0 = - (the paper's dataset
                                            encoding, Section 5) instead of +1 / -1 */
#define BBC_ANCHOR_U          (1u << 4)  /* anchor triples on U (default: chosen per graph
                                            from degree statistics) */
#define BBC_ANCHOR_V          (1u << 5)  /* anchor triples on V */
#define BBC_ANCHOR_SMALLER    (1u << 6)  /* the paper's rule: the smaller side */

/* Context on one device. hip_stream: a hipStream_t to run on (e.g. torch's
 * current stream), or NULL for a stream the context creates. mem_cap_bytes
 * bounds the device memory the context allocates (0 = no cap); exceeding it
 * returns BBC_E_NOMEM. */
bbc_status bbc_ctx_create(int device, void *hip_stream, uint64_t mem_cap_bytes, bbc_ctx **out);
/* Destroys the context and every graph, request and buffer it owns. */
void bbc_ctx_destroy(bbc_ctx *ctx);

/* Validate a COO edge list and build the device CSR of one graph (Section 3
 * input model; degree ordering of Definition 4.1).
 *   eu[e] < n_u, ev[e] < n_v (uint32), sign[e] per flags; n_edges edges.
 * The graph stays resident on the device and is owned by the context until
 * bbc_graph_free. Errors: BBC_E_INVAL, BBC_E_RANGE, BBC_E_SIGN,
 * BBC_E_DUP_EDGE, BBC_E_NOMEM, BBC_E_HIP. */
bbc_status bbc_build_csr(bbc_ctx *ctx, uint32_t n_u, uint32_t n_v, uint64_t n_edges,
                         const uint32_t *eu, const uint32_t *ev, const void *sign,
                         uint32_t flags, bbc_graph **out);

/* Build n_graphs graphs from one concatenated COO in a single device pass.
 *   n_u[i], n_v[i]: host arrays; edge_offsets: host array of n_graphs+1
 *   offsets into eu/ev/sign (graph i owns edges [edge_offsets[i],
 *   edge_offsets[i+1])), vertex ids local to each graph.
 * out_graphs receives n_graphs handles sharing one device allocation (freed
 * when the last of them is freed). On error no handle is returned; the
 * status is the first error found over all graphs. */
bbc_status bbc_build_csr_batch(bbc_ctx *ctx, uint32_t n_graphs, const uint32_t *n_u,
                               const uint32_t *n_v, const uint64_t *edge_offsets,
                               const uint32_t *eu, const uint32_t *ev, const void *sign,
                               uint32_t flags, bbc_graph **out_graphs);

/* Frees one graph handle (its device memory is released with the last
 * handle of its build). BBC_E_INVAL if g is not a live graph of ctx. */
bbc_status bbc_graph_free(bbc_ctx *ctx, bbc_graph *g);

typedef struct {
    uint32_t n_u, n_v;
    uint64_t n_edges;
    int32_t anchor_side;      /* 0 = U, 1 = V */
    uint64_t device_bytes;    /* CSR footprint on the device */
} bbc_graph_info;
bbc_status bbc_get_graph_info(bbc_ctx *ctx, const bbc_graph *g, bbc_graph_info *out);

/* Number of balanced (p,q)-bicliques of g (Problem statement, Section 3):
 * |L| = p vertices of U, |R| = q of V. Algorithm 2 enumerates the vertices
 * of the graph's anchor side (U with BBC_ANCHOR_U, V with BBC_ANCHOR_V, else
 * the side the build chose) and takes C(n, .) on the other: supported are 3,
 * 4 or 5 vertices on the anchor side and 3..7 on the other, e.g. (3, 3) on
 * any graph, (3..5, q) anchored on U, (p, 3..5) anchored on V.
 * out_count: host int64. Errors: BBC_E_UNSUPPORTED (other (p, q) for the
 * graph's anchor side), BBC_E_OVERFLOW (the count, or a single C(n, q) term,
 * does not fit 64 bits), BBC_E_NOMEM, BBC_E_HIP. */
bbc_status bbc_count_global(bbc_ctx *ctx, const bbc_graph *g, int p, int q, int64_t *out_count);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * count as bbc_count_global, with every count buffer carved from a static
 * device array of 256 MiB that the library holds on each device it runs on
 * (looked up when a context is created there). The call allocates no device
 * or pinned host memory; the graph and out_count are the caller's.
 * Limits: a count that needs more than 256 MiB of workspace (roughly graphs
 * beyond a few hundred thousand edges, or fewer with many dense anchors)
 * returns BBC_E_NOMEM before any kernel runs on a buffer it lacks. Calls in
 * one process are serialized; the array keeps the last call's contents, and
 * everything a count needs zeroed is cleared by the call. Errors as for
 * bbc_count_global. */
bbc_status bbc_count_global_noalloc(bbc_ctx *ctx, const bbc_graph *g, int p, int q,
                                    int64_t *out_count);

/* The same count as bbc_count_global for 3 vertices on the graph's anchor
 * side and q = 3..7 on the other, by Algorithm 1 (BBWC, wedge-centric): for
 * every anchor, the signed 3-wedges through pairs of lower-priority partners
 * are bucketed by (partner pair, wedge type) and each bucket of size n adds
 * C(n, q). A second, independent path (it shares only the CSR with
 * bbc_count_global), for cross-checks on small and medium graphs.
 * out_count: host int64. Errors: BBC_E_UNSUPPORTED (other (p, q), or an
 * anchor with more than 393,216 wedge pairs: the path's per-anchor table),
 * BBC_E_OVERFLOW, BBC_E_NOMEM, BBC_E_HIP. */
bbc_status bbc_count_bbwc(bbc_ctx *ctx, const bbc_graph *g, int p, int q, int64_t *out_count);

/* The k vertices of the requested side (0 = U, 1 = V) that lie in the most
 * balanced (3,3)-bicliques, by the per-vertex counts above: out_ids[i],
 * out_counts[i] for i < *out_n = min(k, side size), counts descending, ties
 * to the smaller id. Host arrays of k entries (caller-owned). Errors as for
 * bbc_count_per_vertex. */
bbc_status bbc_top_vertices(bbc_ctx *ctx, const bbc_graph *g, int side, uint32_t k,
                            uint32_t *out_ids, int64_t *out_counts, uint32_t *out_n);

/* Edge queries for dynamic graphs (Section 6 names dynamic signed bipartite
 * graphs as the next direction). For query i, out[i] = number of balanced
 * (3,3)-bicliques that contain the edge (eu[i], ev[i]) (ids of U and V) in g
 * with that edge present with sign es[i] (+1 / -1): added if g lacks it,
 * re-signed if g has it with the other sign. This is the change of the
 * global count when the edge is inserted with sign es[i]; deleting an edge
 * of sign s changes the count by minus the query with s, and flipping it by
 * the query with -s minus the query with s. Every other edge is as in g.
 * All arrays are host memory of n_queries entries (out caller-owned); the
 * queries run in batches on the context's stream. Errors:
 * BBC_E_RANGE (an id outside the graph), BBC_E_SIGN (a sign other than
 * +1 / -1), BBC_E_OVERFLOW, BBC_E_NOMEM, BBC_E_HIP; out is then unspecified. */
bbc_status bbc_count_through_edges(bbc_ctx *ctx, const bbc_graph *g, uint64_t n_queries,
                                   const uint32_t *eu, const uint32_t *ev, const int8_t *es,
                                   int64_t *out);

/* Per-vertex counts: out_per_vertex[x] (caller-owned, n_u or n_v int64
 * entries; host memory, or device memory of the context's device, which the
 * call detects and then fills on the GPU without a host copy) = number of
 * balanced (3,3)-bicliques that contain
 * vertex x of the requested side (0 = U, 1 = V); their sum is 3 * count.
 * out_count (optional) receives the global count. Only (p, q) = (3, 3).
 * Either side works whichever side the graph is anchored on: the triples stay
 * on the anchor side, and a vertex of the other side gets C(n - 1, 2) from
 * every counted pair whose common class of size n holds it. */
bbc_status bbc_count_per_vertex(bbc_ctx *ctx, const bbc_graph *g, int p, int q, int side,
                                int64_t *out_per_vertex, int64_t *out_count);

/* Count many graphs in one persistent launch (replayed from a captured HIP
 * graph when the same set of graphs is counted again). out_counts: host
 * int64[n_graphs]. */
bbc_status bbc_count_batch(bbc_ctx *ctx, const bbc_graph *const *graphs, uint32_t n_graphs,
                           int64_t *out_counts);

/* Serving: queue a count request and return at once. A scheduler thread
 * admits queued requests while their device footprint fits under the
 * context's memory cap, batches every admitted request into the next launch
 * and overlaps launches on several streams (continuous batching).
 *   bbc_submit: a graph already built (it must stay alive until the result
 *     has been polled).
 *   bbc_submit_coo: a COO edge list (host pointers, copied before return);
 *     the scheduler builds and frees its CSR.
 * A result is independent of the other requests in flight. */
bbc_status bbc_submit(bbc_ctx *ctx, const bbc_graph *g, bbc_ticket *out);
bbc_status bbc_submit_coo(bbc_ctx *ctx, uint32_t n_u, uint32_t n_v, uint64_t n_edges,
                          const uint32_t *eu, const uint32_t *ev, const void *sign,
                          uint32_t flags, bbc_ticket *out);
/* BBC_OK with the count (the ticket is then retired), BBC_E_NOT_READY, the
 * request's own error (ticket retired), or BBC_E_UNKNOWN_TICKET. */
bbc_status bbc_poll(bbc_ctx *ctx, bbc_ticket t, int64_t *out_count);
/* Blocks until the request is done; same results as bbc_poll otherwise. */
bbc_status bbc_wait(bbc_ctx *ctx, bbc_ticket t, int64_t *out_count);

/* Statistics of the last count on this context (for measurement). The
 * kernel times are filled only while timing is enabled (bbc_set_timing):
 * they come from HIP events recorded on the context's stream around each
 * phase of the last synchronous build and count. */
typedef struct {
    uint64_t active_anchors;    /* anchor records written (anchors with >= 2 candidate classes) */
    uint64_t virtual_candidates;/* (partner, sign class) pairs with >= 3 shared neighbours */
    uint64_t pair_units;        /* triplet-kernel work units */
    uint64_t candidate_pairs;   /* pairs of candidate classes examined */
    uint64_t mask_words;        /* 32-bit mask words reserved by the pair-table kernel */
    uint64_t wedges;            /* 2-hop wedges scanned (oriented, pruned) */
    uint64_t pair_words;        /* sum over examined pairs of the mask width in words */
    float ms_build;             /* last bbc_build_csr: ingest .. adjacency kernels */
    float ms_pair;              /* pair-table kernels (all tiers) */
    float ms_plan;              /* unit planning */
    float ms_triplet;           /* triplet kernel */
    uint32_t attempts;          /* launches of the count sequence (1 unless buffers grew) */
    uint32_t deferred_b;        /* anchors handed from the 8192-slot to the 16384-slot LDS tier */
    uint32_t deferred_c;        /* anchors handed to the bounded global-memory tier */
    uint32_t deferred_d;        /* anchors handed to the full-size global-memory tier */
    uint32_t deferred_a;        /* anchors handed from the per-wave tier to the workgroup tiers
                                   (degree above 32, or more partners than a wave's table) */
    uint32_t deferred_r;        /* anchors handed to the rank-window tier (heavy anchors whose
                                   partners all rank within 2^17 above them) */
} bbc_count_stats;
bbc_status bbc_get_last_stats(bbc_ctx *ctx, bbc_count_stats *out);
/* Device memory of the context (for operators of the serving loop). The
 * allocator keeps freed blocks for reuse: reserved = live + cached; cached
 * blocks are released when an allocation would pass the cap. Served batches
 * are admitted while their reservation (builds plus one count workspace)
 * fits under the cap next to the live memory of the caller's own graphs and
 * workspaces and the reservations of the batches in flight. */
typedef struct {
    uint64_t cap_bytes;                 /* the context's cap (0 = none) */
    uint64_t reserved_bytes;            /* device memory the context holds */
    uint64_t peak_reserved_bytes;       /* its largest value so far */
    uint64_t live_bytes;                /* held by graphs and workspaces in use */
    uint64_t serve_admitted_bytes;      /* reservations of the served batches in flight */
    uint64_t serve_peak_admitted_bytes; /* their largest sum so far */
    uint64_t serve_queued;              /* requests waiting for admission */
    uint64_t serve_peak_queued;         /* the longest the queue has been */
} bbc_memory_stats;
bbc_status bbc_get_memory_stats(bbc_ctx *ctx, bbc_memory_stats *out);

/* Enable (1) or disable (0) per-phase event timing on this context. */
bbc_status bbc_set_timing(bbc_ctx *ctx, int enable);

/* Test hooks: conditions forced from the host so that tests can reach paths
 * real inputs reach only at sizes too large to test, without changing any
 * kernel. They apply to every later count of the context (serving workers
 * included) until reset with value 0.
 *   BBC_HOOK_NO_WINDOW_TIER: value != 0 keeps heavy anchors in the hash-table
 *     tiers of the pair kernels (the rank-window tier is skipped), so both
 *     routes can be compared on the same graph. Counts are unchanged.
 *   BBC_HOOK_PRELOAD_COUNT: every graph's 64-bit accumulator starts at
 *     (uint64_t)value instead of 0, so a count whose true value plus the
 *     preload passes 2^63 - 1 returns BBC_E_OVERFLOW (the carry path).
 *   BBC_HOOK_LAUNCH_SHAPE: every count (batched ones too, instead of the
 *     tuned shape) uses the launch shape given by value: bits 0-31 the unit
 *     column base (a power of two, 256 to 16384; a unit of w-word masks has
 *     about base / w columns), bits 32-39 triplet workgroups per compute
 *     unit (1 to 16), bits 40-47 tier-A pair workgroups per compute unit
 *     (1 to 8). Counts are unchanged; other values return BBC_E_INVAL.
 * Errors: BBC_E_INVAL (null context, unknown hook or invalid value). */
#define BBC_HOOK_NO_WINDOW_TIER 1
#define BBC_HOOK_PRELOAD_COUNT  2
#define BBC_HOOK_LAUNCH_SHAPE   3
bbc_status bbc_set_test_hook(bbc_ctx *ctx, int hook, int64_t value);

const char *bbc_status_string(bbc_status s);
/* Detail of the last error on this context (empty string if none). */
const char *bbc_last_error(bbc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* BBC_H */
