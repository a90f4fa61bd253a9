// bbc_edge.h -- balanced (3,3)-bicliques through edges (internal).
#pragma once

#include "bbc_dev.h"

namespace bbc {

// One query: a = input id of the endpoint on the anchor side S, b = global O
// index of the other endpoint, neg = 1 when the edge is taken as negative.
struct EdgeQuery {
    uint32_t a_id, b_idx, neg, pad;
};

// Device scratch of a batch of up to Q queries, sized for the largest degree
// D of the graph set; query i owns slice i of every per-query array.
struct EdgeScratch {
    uint32_t *inv;                  // [n_s] S rank of each input id of the graph
    uint32_t *ctl;                  // [Q x 8]: S rank of a, position of b, d_a, words per mask, partners
    unsigned long long *result;     // [Q]
    uint32_t *hkey, *hval;          // [Q x 2^lg] N(a) by opposite index: position << 1 | negative
    uint32_t lg;
    uint32_t *part;                 // [Q x part_stride] partner rank | (class differs) << 31
    uint32_t part_stride;           // D + 1
    uint32_t *masks;                // [Q x mask_stride]
    uint64_t mask_stride;           // (D + 1) x (D / 32 + 1)
};

// S ranks by input id for the graph whose S ranks are [s_base, s_base + n_s).
hipError_t edge_inverse(const CsrView &g, uint32_t s_base, uint32_t n_s, const EdgeScratch &x,
                        hipStream_t s);

// Number of balanced (3,3)-bicliques through each of the n <= Q queried edges
// (q: device array), every edge taken as present with its queried sign; the
// counts land in x.result[0 .. n). edge_inverse must have run for the graph.
hipError_t edge_through(const CsrView &g, const EdgeQuery *q, uint32_t n, const EdgeScratch &x,
                        hipStream_t s);

}  // namespace bbc
