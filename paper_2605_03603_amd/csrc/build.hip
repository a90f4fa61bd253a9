// build.hip -- device CSR builder: COO validation, degrees, vertex priority,
// and both adjacency orientations with the edge sign folded into bit 0.
//
// Vertex priority follows Definition 4.1 of the paper (higher degree first,
// ties broken by the larger id); sorting is the paper's O(m) counting-sort
// step (proof of Theorem 1) done as a stable LSD radix sort on the GPU.
#include "bbc_build.h"

namespace bbc {

namespace {

constexpr int kT = 256;
constexpr uint32_t kSideBlocks = 256;   // workgroups of k_side_stats (one update each per graph)

__device__ __forceinline__ uint32_t find_graph(const uint64_t *__restrict__ off, uint32_t G,
                                               uint64_t x)
{
    // largest g with off[g] <= x (off has G+1 entries, off[0] = 0)
    uint32_t lo = 0, hi = G;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t find_graph32(const uint32_t *__restrict__ base, uint32_t G,
                                                 uint32_t x)
{
    uint32_t lo = 0, hi = G;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Degrees are counted with atomics. A hub takes one increment per edge, from
// every part of the edge list; with per-XCD copies of the counters (the
// workgroups of one XCD share a copy) each counter is updated from one XCD
// only, which keeps the increments of a hub in that XCD's L2.
__global__ void __launch_bounds__(kT) k_ingest(BuildArgs a)
{
    uint32_t *du = a.deg_u, *dv = a.deg_v;
    if (a.deg_x) {
        du = a.deg_x + (uint64_t)(blockIdx.x % kXcd) * ((uint64_t)a.NU + a.NV);
        dv = du + a.NU;
    }
    for (uint64_t e = (uint64_t)blockIdx.x * kT + threadIdx.x; e < a.M;
         e += (uint64_t)gridDim.x * kT) {
        uint32_t g = a.G == 1 ? 0 : find_graph(a.edge_off, a.G, e);
        const GraphDesc &d = a.desc[g];
        uint32_t u = a.eu[e], v = a.ev[e];
        int neg = 0;
        bool ok_sign;
        if (a.flags & kSigns2Bit) {
            uint32_t code = (((const uint8_t *)a.sign)[e >> 2] >> (2 * (e & 3))) & 3u;
            ok_sign = code == 1u || code == 3u;
            neg = code == 3u;
        } else {
            int s = ((const int8_t *)a.sign)[e];
            if (a.flags & kSigns01) { ok_sign = s == 0 || s == 1; neg = s == 0; }
            else { ok_sign = s == 1 || s == -1; neg = s < 0; }
        }
        bool ok_range = u < d.n_u && v < d.n_v;
        if (!ok_range) { atomicOr(a.err, kErrRange); atomicMin(a.first_bad, (unsigned long long)e); }
        if (!ok_sign) { atomicOr(a.err, kErrSign); atomicMin(a.first_bad, (unsigned long long)e); }
        a.eg[e] = (g << 1) | (uint32_t)neg;
        if (ok_range) {
            atomicAdd(&du[d.u_base + u], 1u);
            atomicAdd(&dv[d.v_base + v], 1u);
        }
    }
}

// deg_u, deg_v = the sums of the per-XCD copies
__global__ void __launch_bounds__(kT) k_deg_sum(BuildArgs a)
{
    const uint64_t n = (uint64_t)a.NU + a.NV;
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kT) {
        uint32_t t = 0;
#pragma unroll
        for (int x = 0; x < kXcd; x++) t += a.deg_x[x * n + i];
        if (i < a.NU) a.deg_u[i] = t;
        else a.deg_v[i - a.NU] = t;
    }
}

// Per-graph degree statistics of one side (side 0: U slots, 1: V slots):
// sum of C(d, 2), sum of d^2 and the largest degree. Each workgroup takes a
// contiguous range of slots, and each thread adds up its slots until the
// graph changes, so that a set of a few large graphs updates each graph's
// sums once per workgroup (updates of one address serialise).
__global__ void __launch_bounds__(kT) k_side_stats(BuildArgs a, int side, uint32_t n_slots)
{
    constexpr uint32_t kNone = 0xffffffffu;
    constexpr int NW = kT / kWave;
    __shared__ uint32_t s_g[NW], s_max[NW];
    __shared__ unsigned long long s_c2[NW], s_d2[NW];
    const uint32_t *deg = side ? a.deg_v : a.deg_u;
    const uint32_t *base = side ? a.v_base_arr : a.u_base_arr;
    unsigned long long *c2p = side ? a.stat_c2_v : a.stat_c2_u;
    unsigned long long *d2p = side ? a.stat_d2_v : a.stat_d2_u;
    const uint32_t per = (uint32_t)(((uint64_t)n_slots + gridDim.x - 1) / gridDim.x);
    const uint32_t lo = (uint32_t)min((uint64_t)blockIdx.x * per, (uint64_t)n_slots);
    const uint32_t hi = (uint32_t)min((uint64_t)lo + per, (uint64_t)n_slots);
    uint32_t g_cur = kNone, mx = 0;
    uint64_t c2 = 0, d2 = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kT) {
        const uint32_t g = a.G == 1 ? 0 : find_graph32(base, a.G, i);
        const uint32_t dg = deg[i];
        mx = max(mx, dg);
        if (g != g_cur) {
            if (c2) atomicAdd(c2p + g_cur, (unsigned long long)c2);
            if (d2) atomicAdd(d2p + g_cur, (unsigned long long)d2);
            g_cur = g; c2 = 0; d2 = 0;
        }
        c2 += choose2(dg);
        d2 += (uint64_t)dg * dg;
    }
    // what is left: one update per workgroup where all threads end in one graph
    const uint32_t key = (c2 | d2) ? g_cur : kNone;
    uint32_t kmin = key, kmax = key == kNone ? 0u : key;
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor(kmin, o, kWave));
        kmax = max(kmax, (uint32_t)__shfl_xor(kmax, o, kWave));
        mx = max(mx, (uint32_t)__shfl_xor(mx, o, kWave));
    }
    const uint32_t w = threadIdx.x / kWave;
    if (kmin != kNone && kmin != kmax) {   // several graphs in this wave
        if (key != kNone) {
            atomicAdd(c2p + key, (unsigned long long)c2);
            atomicAdd(d2p + key, (unsigned long long)d2);
        }
        kmin = kNone;
        c2 = d2 = 0;
    }
    c2 = wave_sum<uint64_t>(c2);
    d2 = wave_sum<uint64_t>(d2);
    if (__lane_id() == 0) { s_g[w] = kmin; s_max[w] = mx; s_c2[w] = c2; s_d2[w] = d2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t g = kNone, m = 0;
        uint64_t t2 = 0, q2 = 0;
        for (int x = 0; x < NW; x++) {
            m = max(m, s_max[x]);
            if (s_g[x] == kNone) continue;
            if (s_g[x] != g) {
                if (g != kNone) {
                    atomicAdd(c2p + g, (unsigned long long)t2);
                    atomicAdd(d2p + g, (unsigned long long)q2);
                }
                g = s_g[x]; t2 = 0; q2 = 0;
            }
            t2 += s_c2[x];
            q2 += s_d2[x];
        }
        if (g != kNone) {
            atomicAdd(c2p + g, (unsigned long long)t2);
            atomicAdd(d2p + g, (unsigned long long)q2);
        }
        if (m) atomicMax(side ? a.max_deg_v : a.max_deg_u, m);
    }
}

// One thread per global S slot / O slot: degree in the chosen orientation
// and the rank-sort key (graph, degree) with the vertex id as value.
__global__ void __launch_bounds__(kT) k_gather(BuildArgs a)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < (uint64_t)a.NS + a.NO;
         i += (uint64_t)gridDim.x * kT) {
        if (i < a.NS) {
            uint32_t g = a.G == 1 ? 0 : find_graph32(a.s_base_arr, a.G, (uint32_t)i);
            const GraphDesc &d = a.desc[g];
            uint32_t x = (uint32_t)i - d.s_base;
            uint32_t dg = d.side ? a.deg_v[d.v_base + x] : a.deg_u[d.u_base + x];
            a.key0[i] = (uint64_t)g * (a.max_deg_s + 1ull) + dg;
            a.val0[i] = x;
        } else {
            uint32_t j = (uint32_t)(i - a.NS);
            uint32_t g = a.G == 1 ? 0 : find_graph32(a.o_base_arr, a.G, j);
            const GraphDesc &d = a.desc[g];
            uint32_t x = j - d.o_base;
            a.deg_o[j] = d.side ? a.deg_u[d.u_base + x] : a.deg_v[d.v_base + x];
        }
    }
}

// After the stable sort by (graph, degree) position p is the global rank.
__global__ void __launch_bounds__(kT) k_rank_scatter(BuildArgs a)
{
    for (uint64_t p = (uint64_t)blockIdx.x * kT + threadIdx.x; p < a.NS;
         p += (uint64_t)gridDim.x * kT) {
        uint64_t key = a.key0[p];
        uint32_t g = (uint32_t)(key / (a.max_deg_s + 1ull));
        uint32_t dg = (uint32_t)(key % (a.max_deg_s + 1ull));
        uint32_t x = a.val0[p];
        a.rank_of[a.desc[g].s_base + x] = (uint32_t)p;
        a.s_vert[p] = x;
        a.s_graph[p] = g;
        a.deg_rank[p] = dg;
    }
}

__global__ void __launch_bounds__(kT) k_edge_keys(BuildArgs a)
{
    for (uint64_t e = (uint64_t)blockIdx.x * kT + threadIdx.x; e < a.M;
         e += (uint64_t)gridDim.x * kT) {
        uint32_t ge = a.eg[e];
        uint32_t g = ge >> 1, neg = ge & 1;
        const GraphDesc &d = a.desc[g];
        uint32_t u = a.eu[e], v = a.ev[e];
        uint32_t s_loc = d.side ? v : u, o_loc = d.side ? u : v;
        a.key0[e] = a.rank_of[d.s_base + s_loc];
        a.val0[e] = ((d.o_base + o_loc) << 1) | neg;
    }
}

// Sorted by rank (stably: a list keeps the input order): emit s_adj and
// prepare the (O index -> S position) keys whose stable sort yields the
// O-side lists in rank order. o_ent[t] is the O-side entry of S position t.
__global__ void __launch_bounds__(kT) k_s_finish(BuildArgs a)
{
    for (uint64_t t = (uint64_t)blockIdx.x * kT + threadIdx.x; t < a.M;
         t += (uint64_t)gridDim.x * kT) {
        const uint32_t r = (uint32_t)a.key0[t];
        const uint32_t val = a.val0[t];
        a.s_adj[t] = val;
        a.key1[t] = val >> 1;
        a.val1[t] = (uint32_t)t;
        a.o_ent[t] = (r << 1) | (val & 1);
    }
}

// Sorted by O index (stably, so each O list is in rank order): emit o_adj
// and, for every S position, where the part of the O list ranked above the
// S vertex starts and how long it is.
__global__ void __launch_bounds__(kT) k_o_finish(BuildArgs a)
{
    // every thread of the grid runs the same number of rounds, so that whole
    // waves take part in the shuffles below
    const uint64_t stride = (uint64_t)gridDim.x * kT;
    for (uint64_t t0 = (uint64_t)blockIdx.x * kT; t0 < a.M; t0 += stride) {
        const uint64_t t = t0 + threadIdx.x;
        const bool in = t < a.M;
        const uint32_t ts = in ? a.val1[t] : 0u;
        const uint32_t ent = in ? a.o_ent[ts] : 0u;
        const uint32_t v = in ? (uint32_t)a.key1[t] : 0u;
        // the previous position's entry and O vertex: from the lane below, or
        // loaded by the first lane of the wave
        uint32_t ent_p = __shfl_up(ent, 1, kWave), v_p = __shfl_up(v, 1, kWave);
        if (__lane_id() == 0 && in && t > 0) {
            ent_p = a.o_ent[a.val1[t - 1]];
            v_p = (uint32_t)a.key1[t - 1];
        }
        if (!in) continue;
        a.o_adj[t] = ent;
        // a repeated (u, v) pair: equal neighbours in one O list are adjacent
        if (t > 0 && v_p == v && (ent_p >> 1) == (ent >> 1))
            atomicOr(a.err, kErrDup);
        uint32_t len = (uint32_t)(a.o_off[v + 1] - t - 1);
        if (len < 2) len = 0;
        a.s_suf[ts] = make_uint2((uint32_t)t + 1, len | ((ent & 1u) << 31));
    }
}

__global__ void __launch_bounds__(kT) k_fill_u32(uint32_t *p, uint32_t v, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kT)
        p[i] = v;
}

__global__ void __launch_bounds__(kT) k_fill_u64(unsigned long long *p, unsigned long long v,
                                                 uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kT)
        p[i] = v;
}

inline uint32_t grid_for(uint64_t n, uint32_t cap = 8192)
{
    uint64_t b = (n + kT - 1) / kT;
    if (b < 1) b = 1;
    return (uint32_t)(b < cap ? b : cap);
}

}  // namespace

hipError_t fill_u32(uint32_t *p, uint32_t v, uint64_t n, hipStream_t s)
{
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kT), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t fill_u64(void *p, uint64_t v, uint64_t n, hipStream_t s)
{
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(kT), 0, s, (unsigned long long *)p,
                       (unsigned long long)v, n);
    return hipGetLastError();
}

hipError_t build_ingest(const BuildArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_ingest, dim3(grid_for(a.M)), dim3(kT), 0, s, a);
    if (a.deg_x)
        hipLaunchKernelGGL(k_deg_sum, dim3(grid_for((uint64_t)a.NU + a.NV)), dim3(kT), 0, s, a);
    hipLaunchKernelGGL(k_side_stats, dim3(grid_for(a.NU, kSideBlocks)), dim3(kT), 0, s, a, 0, a.NU);
    hipLaunchKernelGGL(k_side_stats, dim3(grid_for(a.NV, kSideBlocks)), dim3(kT), 0, s, a, 1, a.NV);
    return hipGetLastError();
}

hipError_t build_rank(const BuildArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, dim3(grid_for((uint64_t)a.NS + a.NO)), dim3(kT), 0, s, a);
    hipError_t e = radix_sort(a.key0, a.val0, a.key1, a.val1, a.NS, a.rank_bits, a.tmp,
                              a.tmp_bytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rank_scatter, dim3(grid_for(a.NS)), dim3(kT), 0, s, a);
    e = scan_u32_to_u64(a.deg_rank, a.s_off, a.NS, a.tmp, a.tmp_bytes, s);
    if (e != hipSuccess) return e;
    e = scan_u32_to_u64(a.deg_o, a.o_off, a.NO, a.tmp, a.tmp_bytes, s);
    return e;
}

hipError_t build_adjacency(const BuildArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_edge_keys, dim3(grid_for(a.M)), dim3(kT), 0, s, a);
    hipError_t e = radix_sort(a.key0, a.val0, a.key1, a.val1, a.M, a.s_bits, a.tmp, a.tmp_bytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_s_finish, dim3(grid_for(a.M)), dim3(kT), 0, s, a);
    // key0/val0 are free again and serve as the ping-pong buffers
    e = radix_sort(a.key1, a.val1, a.key0, a.val0, a.M, a.o_bits, a.tmp, a.tmp_bytes, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_o_finish, dim3(grid_for(a.M)), dim3(kT), 0, s, a);
    return hipGetLastError();
}

}  // namespace bbc
