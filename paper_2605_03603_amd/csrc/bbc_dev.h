// bbc_dev.h -- internal declarations of libbbc (device layout, launchers).
// Not part of the public ABI (include/bbc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbc {

constexpr int kWave = 64;

// ----------------------------------------------------------------- layout
//
// A "graph set" holds one graph or a batch of disjoint graphs in one CSR.
// Every graph picks an anchor side S (the side whose triples are enumerated)
// and an opposite side O. Vertices of S are renumbered by priority
// (Definition 4.1: degree, then id), so that inside a graph a larger global
// rank means a higher priority; all graphs' S vertices are concatenated
// (graph g owns global ranks [s_base, s_base + n_s)) and so are O vertices.
//
//   s_off[NS+1], s_adj[M]: neighbours of S vertex r (in input order);
//                          entry = (global O index << 1) | (sign < 0)
//   o_off[NO+1], o_adj[M]: neighbours of O vertex v, sorted by rank;
//                          entry = (global rank << 1) | (sign < 0)
//   s_suf[M]               for S position t (edge (r, v)): x = first position
//                          in o_adj of the neighbours of v ranked above r (they
//                          end at o_off[v+1]); y = their number, 0 when below 2
//                          (v then closes no triple anchored at r), with the
//                          edge's sign bit (negative) in bit 31
//   s_graph[NS]            graph of each global rank
//   s_vert[NS]             the vertex's id inside its graph (input numbering)
//   o_vert (implicit)      O index - o_base is the id inside the graph
struct GraphDesc {
    uint32_t n_u, n_v;
    uint32_t side;         // 0: S = U, 1: S = V
    uint32_t n_s, n_o;
    uint32_t s_base, o_base;
    uint32_t u_base, v_base;   // slots of the input numbering (build only)
    uint32_t pad;
    uint64_t e_base, m;
};

struct CsrView {
    uint32_t G, NS, NO;
    uint64_t M;
    const uint64_t *s_off;
    const uint32_t *s_adj;
    const uint64_t *o_off;
    const uint32_t *o_adj;
    const uint2 *s_suf;
    const uint32_t *s_graph;
    const uint32_t *s_vert;
    const GraphDesc *desc;
};

// ------------------------------------------------------ build error flags
enum : uint32_t {
    kErrRange = 1u << 0,
    kErrSign = 1u << 1,
    kErrDup = 1u << 2,
};

// ------------------------------------------------------- count workspace
//
// Output of the pair-table kernel for one anchor with k >= 2 candidate
// classes (a "virtual candidate" is a partner w together with one sign
// class; its mask has bit p set when the p-th neighbour of the anchor is a
// common neighbour in that class).
struct AnchorRec {
    uint32_t rank;      // global rank of the anchor
    uint32_t k;         // virtual candidates
    uint32_t w32;       // 32-bit words per mask = ceil(deg / 32)
    uint32_t graph;
    uint64_t mask_off;  // first mask word
    uint64_t cand_off;  // first candidate id (global rank of its partner)
};

// A triplet work unit: rows [64*rb, 64*rb+64) x columns [c0, c1) of the
// lower triangle of one anchor's candidate-pair matrix.
struct Unit {
    uint32_t anchor;    // index into AnchorRec[]
    uint32_t rb;
    uint32_t c0, c1;
};

constexpr int kXcd = 8;   // MI355X: 8 XCDs; workgroup i runs on XCD i % 8

struct alignas(64) Cursor {
    uint32_t v;
    uint32_t pad[15];
};

struct Counters {           // device-side cursors and flags, zeroed per count
    unsigned long long mask_cursor;
    unsigned long long cand_cursor;
    unsigned long long wedges;
    unsigned long long pairs_examined;
    unsigned long long pair_words;
    uint32_t n_anchor;      // anchor records reserved (including unused slots)
    uint32_t over_cap;      // 1, 2: a workspace capacity was exceeded; 4: unsupported anchor;
                            // 8: lookup failure; 16: C(n, q) overflow; 32: more than 2^32 - 1 units
    uint32_t n_list[5];     // anchors handed to the workgroup tiers A, B, C, D and to the
                            // rank-window tier
    uint32_t n_units;       // written by the plan kernel: all units
    uint32_t n_cls_end[2];  // units of class 0 (masks <= 4 words) come first, then
                            // class 1 (up to 16 words), then class 2 (wider)
    unsigned long long need_masks, need_cands, need_recs, need_units;   // exact demand
    Cursor q_pair[6][kXcd]; // work-queue cursors of the pair tiers, one per XCD slice
    Cursor q_tri[2][kXcd];  // queues of the two triplet kernels
};

struct Workspace {
    Counters *ctr;
    AnchorRec *anchors;  uint64_t cap_anchors;
    Unit *units;         uint64_t cap_units;
    uint32_t *masks;     uint64_t cap_mask_words;
    uint32_t *cands;     uint64_t cap_cands;
    uint32_t *defer[5];  uint64_t cap_defer;     // anchors for tiers A, B, C, D, rank window
    uint32_t *gtab;      uint64_t gtab_words_per_block; uint32_t gtab_blocks;  // tier C tables
    uint32_t *dtab;      uint64_t dtab_words_per_block; uint32_t dtab_blocks;  // tier D tables
    uint32_t *bscr;      uint64_t bscr_words_per_block;   // per-block position lists of tier B
                                                           // and of the rank-window tier
    uint32_t *ucnt;      // [3 cap_anchors] units per anchor record, one slice per unit class
    uint64_t *uoff;      // [3 cap_anchors + 1] exclusive prefix of ucnt
    unsigned long long *count;   // [G] totals
    uint32_t *carry;             // [G] carries out of 64 bits
    unsigned long long *pv;      // [NS] per-vertex (by global rank) or null
    unsigned long long *pv_slot; // [cap_cands] per candidate slot, anchor-side per-vertex counts
    unsigned long long *pv_o;    // [NO] per-vertex of the opposite side or null
};

// --------------------------------------------------------------- helpers
__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t w = __shfl_up(v, o, kWave);
        if (lane >= (uint32_t)o) v += w;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_max64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

__host__ __device__ __forceinline__ uint64_t choose2(uint64_t n) { return n < 2 ? 0 : n * (n - 1) / 2; }
__host__ __device__ __forceinline__ uint64_t choose3(uint64_t n)
{
    return n < 3 ? 0 : n * (n - 1) / 2 * (n - 2) / 3;
}

}  // namespace bbc

// ------------------------------------------------------------ launchers
// (defined in the .hip files, called by the runtime)
namespace bbc {

// exclusive scan: out[i] = sum in[0..i), out[n] = total (out has n+1 slots)
hipError_t scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, void *tmp,
                           size_t tmp_bytes, hipStream_t s);
size_t scan_tmp_bytes(uint64_t n);

// stable LSD radix sort of (key, value) by the low `bits` bits of key.
// Result ends in k0/v0 (the buffers are ping-ponged).
hipError_t radix_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint64_t n,
                      int bits, void *tmp, size_t tmp_bytes, hipStream_t s);
size_t radix_tmp_bytes(uint64_t n);

}  // namespace bbc
