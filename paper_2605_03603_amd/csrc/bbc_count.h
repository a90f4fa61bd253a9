// bbc_count.h -- arguments of the counting kernels (internal).
#pragma once

#include "bbc_dev.h"

namespace bbc {

struct PairArgs {
    CsrView g;
    Workspace ws;
    uint32_t a0, a1;        // anchor range (global ranks) scanned by the per-wave tier
    int tier;               // 0: per-wave LDS tables; 1, 2: per-workgroup LDS tables;
                            // 3: bounded global tables; 4: full-size global tables;
                            // 5: rank-window LDS tables
    uint32_t chunk_base;    // triplet unit width in columns for 1-word masks (<= 2048)
    uint32_t gH;            // tier-2 table slots (power of two)
    int glog2h;
    uint32_t dH;            // tier-3 table slots
    int dlog2h;
    uint32_t gmaxd, gkmax;  // degree and candidate limits of tiers 2, 3 and 4
    uint32_t flags;         // kPairNoWindow: heavy anchors stay in the hash tiers
    uint32_t mask_chunk, cand_chunk;        // output reserved per workgroup at a time
    uint32_t wv_mask_chunk, wv_cand_chunk;  // and per wave of the per-wave tier
};

constexpr uint32_t kPairNoWindow = 1u;

struct TriArgs {
    CsrView g;
    Workspace ws;
    uint32_t q;             // mode 3: size of the vertex subsets of the opposite side
};

struct LaunchShape {
    uint32_t grid_w, grid_a, grid_b, grid_c, grid_d, grid_t;
};

hipError_t count_pairs(const PairArgs &P, const LaunchShape &sh, hipStream_t s);
// cut the anchors' pair matrices into triplet work units for p (3, 4 or 5)
// vertices on the anchor side (4: the pair triangles after every candidate,
// 5: after every pair of candidates)
hipError_t count_plan(const Workspace &ws, uint32_t chunk_base, void *tmp, size_t tmp_bytes,
                      uint32_t p, hipStream_t s);
// mode 0: totals only; 1: also per vertex of the anchor side; 2: per vertex of
// the opposite side; 3: totals with q (T.q, 4..7) vertices on the opposite side;
// 4, 5: totals with 4 or 5 vertices on the anchor side and q (T.q, 3..7) on the other
hipError_t count_triplets(const TriArgs &T, int mode, uint32_t grid, hipStream_t s);
// per-vertex counts into a device array: out[id[i]] = pv[i] for i < n (id
// null: out[i] = pv[i]); *bad |= 1 if a value does not fit int64
hipError_t per_vertex_to_device(const unsigned long long *pv, const uint32_t *id, uint32_t n,
                                int64_t *out, uint32_t *bad, hipStream_t s);
// workgroups (and waves) of the per-wave tier that fit on one compute unit
uint32_t wave_tier_blocks_per_cu();
uint32_t wave_tier_waves_per_cu();
uint32_t tier_c_max_degree();
// widest partner window (ranks above the anchor) of the rank-window tier
uint32_t window_tier_max_window();
uint32_t tier_c_max_k();
uint32_t max_unit_chunk();

}  // namespace bbc
