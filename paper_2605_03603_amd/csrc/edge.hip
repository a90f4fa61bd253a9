// edge.hip -- balanced (3,3)-bicliques through one edge: the change of the
// count when the edge is inserted, deleted or re-signed (Section 6 names
// dynamic signed bipartite graphs as the next direction).
//
// Let a be the endpoint on the anchor side S and b the other one. A balanced
// (3,3)-biclique (L, R) through (a, b) has L = {a, w, w'} with w, w' in N(b)
// and R = {b, r, r'}. By Lemma 1 and its converse, R lies in one sign class
// of the common neighbours of L, the class of b. For a partner w in N(b),
// let sigma_w = s(a, b) s(w, b) and M_w = { v in N(a) with edge (w, v) and
// s(a, v) s(w, v) = sigma_w } (b included): these are the members of b's
// class seen from the wedge type of w (Section 4, wedge types). For two
// partners, M_w n M_w' is exactly b's class in the common neighbourhood of
// {a, w, w'}, of size n, and b lies in C(n - 1, 2) of its 3-subsets. So
//
//   through(a, b) = sum over pairs w < w' in N(b) \ {a} of C(|M_w n M_w'| - 1, 2),
//
// with s(a, b) the queried sign and every other edge as in the graph.

#include "bbc_build.h"
#include "bbc_edge.h"

namespace bbc {

namespace {

constexpr uint32_t kNone = 0xffffffffu;
constexpr int kSetupThreads = 1024;
constexpr int kT = 256;

__device__ __forceinline__ uint32_t edge_hash(uint32_t x, uint32_t lg)
{
    return (x * 0x9E3779B1u) >> (32 - lg);
}

// the S rank of a: the one rank of the graph whose input id is a_id
__global__ void __launch_bounds__(kT) k_edge_locate(CsrView g, uint32_t s_base, uint32_t n_s,
                                                    uint32_t a_id, EdgeScratch x)
{
    for (uint32_t r = blockIdx.x * kT + threadIdx.x; r < n_s; r += gridDim.x * kT)
        if (g.s_vert[s_base + r] == a_id) x.ctl[0] = s_base + r;
}

// N(a) into the hash table (b left out: its position stands for the queried
// sign), the partners N(b) \ {a} with their class bit, cleared masks
__global__ void __launch_bounds__(kSetupThreads) k_edge_setup(CsrView g, uint32_t b_idx,
                                                              uint32_t neg_q, EdgeScratch x)
{
    __shared__ uint32_t sh_pb, sh_np;
    const uint32_t tid = threadIdx.x;
    const uint32_t r = x.ctl[0];
    const uint64_t s0 = g.s_off[r];
    const uint32_t da = (uint32_t)(g.s_off[r + 1] - s0);
    const uint32_t H = 1u << x.lg;
    for (uint32_t h = tid; h < H; h += kSetupThreads) x.hkey[h] = kNone;
    if (tid == 0) { sh_pb = da; sh_np = 0; }
    __syncthreads();
    // position of b in N(a), or da when the edge is new
    for (uint32_t t = tid; t < da; t += kSetupThreads)
        if ((g.s_adj[s0 + t] >> 1) == b_idx) atomicMin(&sh_pb, t);
    for (uint32_t t = tid; t < da; t += kSetupThreads) {
        const uint32_t e = g.s_adj[s0 + t];
        const uint32_t key = e >> 1;
        if (key == b_idx) continue;
        uint32_t h = edge_hash(key, x.lg);
        for (;;) {
            const uint32_t old = atomicCAS(&x.hkey[h], kNone, key);
            if (old == kNone) { x.hval[h] = (t << 1) | (e & 1u); break; }
            h = (h + 1) & (H - 1);
        }
    }
    const uint64_t b0 = g.o_off[b_idx];
    const uint32_t db = (uint32_t)(g.o_off[b_idx + 1] - b0);
    for (uint32_t t = tid; t < db; t += kSetupThreads) {
        const uint32_t e = g.o_adj[b0 + t];
        const uint32_t w = e >> 1;
        if (w == r) continue;
        const uint32_t i = atomicAdd(&sh_np, 1u);
        x.part[i] = w | (((e & 1u) ^ neg_q) << 31);
    }
    __syncthreads();
    const uint32_t W = da / 32 + 1;   // positions 0 .. da
    for (uint64_t i = tid; i < (uint64_t)sh_np * W; i += kSetupThreads) x.masks[i] = 0;
    if (tid == 0) {
        x.ctl[1] = sh_pb;
        x.ctl[2] = da;
        x.ctl[3] = W;
        x.ctl[4] = sh_np;
    }
}

// one wave per partner w: bit p of M_w for every neighbour of w at position
// p of N(a) whose wedge type is w's class at b
__global__ void __launch_bounds__(kT) k_edge_masks(CsrView g, uint32_t b_idx, EdgeScratch x)
{
    const uint32_t np = x.ctl[4], W = x.ctl[3], pb = x.ctl[1];
    const uint32_t lane = __lane_id();
    const uint32_t H = 1u << x.lg;
    const uint32_t nw = gridDim.x * (kT / kWave);
    for (uint32_t i = blockIdx.x * (kT / kWave) + threadIdx.x / kWave; i < np; i += nw) {
        const uint32_t pw = x.part[i];
        const uint32_t w = pw & 0x7fffffffu, cls = pw >> 31;
        uint32_t *M = x.masks + (uint64_t)i * W;
        if (lane == 0) atomicOr(&M[pb >> 5], 1u << (pb & 31));
        const uint64_t s0 = g.s_off[w];
        const uint32_t dw = (uint32_t)(g.s_off[w + 1] - s0);
        for (uint32_t t = lane; t < dw; t += kWave) {
            const uint32_t e = g.s_adj[s0 + t];
            const uint32_t key = e >> 1;
            if (key == b_idx) continue;
            uint32_t h = edge_hash(key, x.lg);
            for (;;) {
                const uint32_t k = x.hkey[h];
                if (k == kNone) break;
                if (k == key) {
                    const uint32_t v = x.hval[h];
                    const uint32_t p = v >> 1;
                    if (((v ^ e) & 1u) == cls) atomicOr(&M[p >> 5], 1u << (p & 31));
                    break;
                }
                h = (h + 1) & (H - 1);
            }
        }
    }
}

// one wave per partner i: C(|M_i n M_j| - 1, 2) over the partners j > i
__global__ void __launch_bounds__(kT) k_edge_pairs(EdgeScratch x)
{
    const uint32_t np = x.ctl[4], W = x.ctl[3];
    const uint32_t lane = __lane_id();
    const uint32_t nw = gridDim.x * (kT / kWave);
    uint64_t acc = 0;
    for (uint32_t i = blockIdx.x * (kT / kWave) + threadIdx.x / kWave; i < np; i += nw) {
        const uint32_t *Mi = x.masks + (uint64_t)i * W;
        for (uint32_t j = i + 1 + lane; j < np; j += kWave) {
            const uint32_t *Mj = x.masks + (uint64_t)j * W;
            uint32_t n = 0;
            for (uint32_t w = 0; w < W; w++) n += __popc(Mi[w] & Mj[w]);
            if (n >= 3) acc += (uint64_t)(n - 1) * (n - 2) / 2;
        }
    }
    acc = wave_sum<uint64_t>(acc);
    if (lane == 0 && acc) atomicAdd(x.result, (unsigned long long)acc);
}

}  // namespace

hipError_t edge_through(const CsrView &g, uint32_t s_base, uint32_t n_s, uint32_t a_id,
                        uint32_t b_idx, uint32_t neg_q, const EdgeScratch &x, uint32_t grid,
                        hipStream_t s)
{
    hipError_t e = fill_u32(x.ctl, 0, 8, s);
    if (e == hipSuccess) e = fill_u64(x.result, 0, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_locate, dim3(grid), dim3(kT), 0, s, g, s_base, n_s, a_id, x);
    hipLaunchKernelGGL(k_edge_setup, dim3(1), dim3(kSetupThreads), 0, s, g, b_idx, neg_q, x);
    hipLaunchKernelGGL(k_edge_masks, dim3(grid), dim3(kT), 0, s, g, b_idx, x);
    hipLaunchKernelGGL(k_edge_pairs, dim3(grid), dim3(kT), 0, s, x);
    return hipGetLastError();
}

}  // namespace bbc
