// bbc_build.h -- arguments of the device CSR builder (internal).
#pragma once

#include "bbc_dev.h"

namespace bbc {

enum : uint32_t {
    kSigns2Bit = 1u << 1,   // same bit values as BBC_SIGNS_2BIT_PACKED / BBC_SIGNS_01
    kSigns01 = 1u << 2,
};

struct BuildArgs {
    // input (device)
    const uint32_t *eu, *ev;
    const void *sign;
    uint32_t flags;
    uint64_t M;
    uint32_t G;
    const uint64_t *edge_off;      // [G+1]
    const GraphDesc *desc;         // [G]
    const uint32_t *u_base_arr;    // [G] U slot bases (for slot -> graph lookup)
    const uint32_t *v_base_arr;
    const uint32_t *s_base_arr;    // [G] (after the side choice)
    const uint32_t *o_base_arr;
    uint32_t NU, NV, NS, NO;
    // ingest outputs
    uint32_t *eg;                  // [M] (graph << 1) | negative
    uint32_t *deg_u, *deg_v;       // [NU], [NV]
    uint32_t *deg_x;               // [kXcd][NU + NV] zeroed per-XCD degree copies, or null
                                   // (then the increments go to deg_u, deg_v directly)
    uint32_t *err;
    unsigned long long *first_bad;
    unsigned long long *stat_c2_u, *stat_c2_v, *stat_d2_u, *stat_d2_v;   // [G]
    uint32_t *max_deg_u, *max_deg_v;
    // ranking
    uint32_t max_deg_s;            // max degree over S slots (key radix)
    int rank_bits, s_bits, o_bits;
    uint64_t *key0, *key1;
    uint32_t *val0, *val1;
    uint32_t *deg_o;               // [NO]
    uint32_t *deg_rank;            // [NS]
    uint32_t *rank_of;             // [NS] slot -> global rank
    // CSR outputs
    uint64_t *s_off, *o_off;
    uint32_t *s_adj, *o_adj, *s_graph, *s_vert;
    uint2 *s_suf;
    uint32_t *o_ent;               // [M] scratch: O-side entry per S position
    void *tmp;
    size_t tmp_bytes;
};

hipError_t build_ingest(const BuildArgs &a, hipStream_t s);
hipError_t build_rank(const BuildArgs &a, hipStream_t s);
hipError_t build_adjacency(const BuildArgs &a, hipStream_t s);
hipError_t fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t s);
hipError_t fill_u64(void *p, uint64_t v, uint64_t n, hipStream_t s);

}  // namespace bbc
