// bbc_bbwc.h -- Algorithm 1 (wedge-centric counting) as a second GPU path (internal).
#pragma once

#include "bbc_dev.h"

namespace bbc {

struct BbwcArgs {
    CsrView g;
    uint32_t a0, a1;               // S ranks of the graph
    uint32_t q;                    // vertices on the other side (3..7)
    uint32_t lg;                   // log2 of the slots per workgroup table
    unsigned long long *keys;      // [grid << lg] (w1 rank << 32) | w2 rank, or empty
    uint32_t *cnt;                 // [grid << lg][4] wedges per type
    uint32_t *used;                // [grid << lg] used slots of the current anchor
    uint32_t *cursor;              // [1] next anchor
    uint32_t *flags;               // [1] 1: an anchor has more wedge pairs than 3/4 of a table, 2: overflow
    unsigned long long *total;     // [1]
};

// Balanced (3, q)-bicliques with the triples on the anchor side S by
// Algorithm 1 (one workgroup per anchor at a time, grid workgroups).
hipError_t bbwc_count(const BbwcArgs &A, uint32_t grid, hipStream_t s);

}  // namespace bbc
