// bbc_edge.h -- balanced (3,3)-bicliques through one edge (internal).
#pragma once

#include "bbc_dev.h"

namespace bbc {

// Device scratch of one edge query, sized for the largest degree D of the
// graph set (every array is reused by the next query).
struct EdgeScratch {
    uint32_t *ctl;                  // [8]: S rank of a, position of b, d_a, words per mask, partners
    unsigned long long *result;     // [1]
    uint32_t *hkey, *hval;          // [2^lg] N(a) by opposite index: position << 1 | negative
    uint32_t lg;
    uint32_t *part;                 // [D + 1] partner rank | (class differs) << 31
    uint32_t *masks;                // [(D + 1) x (D / 32 + 1)]
};

// Number of balanced (3,3)-bicliques through the edge (a, b) of graph g's
// set, with the edge taken as present with sign (-1)^neg_q: a is the
// endpoint on the anchor side S (input id a_id of a graph whose S ranks are
// [s_base, s_base + n_s)), b the endpoint on the other side (global O index
// b_idx). Enqueued on s; the count lands in x.result.
hipError_t edge_through(const CsrView &g, uint32_t s_base, uint32_t n_s, uint32_t a_id,
                        uint32_t b_idx, uint32_t neg_q, const EdgeScratch &x, uint32_t grid,
                        hipStream_t s);

}  // namespace bbc
