// edge.hip -- balanced (3,3)-bicliques through an edge: the change of the
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
constexpr uint32_t kBlocksPerQuery = 4;   // workgroups of the mask and pair kernels per query

__device__ __forceinline__ uint32_t edge_hash(uint32_t x, uint32_t lg)
{
    return (x * 0x9E3779B1u) >> (32 - lg);
}

// S rank of every input id of the graph
__global__ void __launch_bounds__(kT) k_edge_inverse(CsrView g, uint32_t s_base, uint32_t n_s,
                                                     EdgeScratch x)
{
    for (uint32_t r = blockIdx.x * kT + threadIdx.x; r < n_s; r += gridDim.x * kT)
        x.inv[g.s_vert[s_base + r]] = s_base + r;
}

// one workgroup per query: N(a) into the query's hash table (b left out: its
// position stands for the queried sign), the partners N(b) \ {a} with their
// class bit, cleared masks
__global__ void __launch_bounds__(kSetupThreads) k_edge_setup(CsrView g, const EdgeQuery *qs,
                                                              EdgeScratch x)
{
    __shared__ uint32_t sh_pb, sh_np;
    const uint32_t tid = threadIdx.x, qi = blockIdx.x;
    const EdgeQuery q = qs[qi];
    uint32_t *ctl = x.ctl + 8 * qi;
    const uint32_t H = 1u << x.lg;
    uint32_t *hkey = x.hkey + (uint64_t)qi * H, *hval = x.hval + (uint64_t)qi * H;
    uint32_t *part = x.part + (uint64_t)qi * x.part_stride;
    uint32_t *masks = x.masks + (uint64_t)qi * x.mask_stride;
    const uint32_t r = x.inv[q.a_id];
    const uint64_t s0 = g.s_off[r];
    const uint32_t da = (uint32_t)(g.s_off[r + 1] - s0);
    for (uint32_t h = tid; h < H; h += kSetupThreads) hkey[h] = kNone;
    if (tid == 0) { sh_pb = da; sh_np = 0; }
    __syncthreads();
    // position of b in N(a), or da when the edge is new
    for (uint32_t t = tid; t < da; t += kSetupThreads)
        if ((g.s_adj[s0 + t] >> 1) == q.b_idx) atomicMin(&sh_pb, t);
    for (uint32_t t = tid; t < da; t += kSetupThreads) {
        const uint32_t e = g.s_adj[s0 + t];
        const uint32_t key = e >> 1;
        if (key == q.b_idx) continue;
        uint32_t h = edge_hash(key, x.lg);
        for (;;) {
            const uint32_t old = atomicCAS(&hkey[h], kNone, key);
            if (old == kNone) { hval[h] = (t << 1) | (e & 1u); break; }
            h = (h + 1) & (H - 1);
        }
    }
    const uint64_t b0 = g.o_off[q.b_idx];
    const uint32_t db = (uint32_t)(g.o_off[q.b_idx + 1] - b0);
    for (uint32_t t = tid; t < db; t += kSetupThreads) {
        const uint32_t e = g.o_adj[b0 + t];
        const uint32_t w = e >> 1;
        if (w == r) continue;
        const uint32_t i = atomicAdd(&sh_np, 1u);
        part[i] = w | (((e & 1u) ^ q.neg) << 31);
    }
    __syncthreads();
    const uint32_t W = da / 32 + 1;   // positions 0 .. da
    for (uint64_t i = tid; i < (uint64_t)sh_np * W; i += kSetupThreads) masks[i] = 0;
    if (tid == 0) {
        ctl[0] = r;
        ctl[1] = sh_pb;
        ctl[2] = da;
        ctl[3] = W;
        ctl[4] = sh_np;
    }
}

// kBlocksPerQuery workgroups per query, one wave per partner w: bit p of M_w
// for every neighbour of w at position p of N(a) whose wedge type is w's
// class at b
__global__ void __launch_bounds__(kT) k_edge_masks(CsrView g, const EdgeQuery *qs, EdgeScratch x)
{
    const uint32_t qi = blockIdx.x / kBlocksPerQuery, sub = blockIdx.x % kBlocksPerQuery;
    const uint32_t *ctl = x.ctl + 8 * qi;
    const uint32_t np = ctl[4], W = ctl[3], pb = ctl[1];
    const uint32_t b_idx = qs[qi].b_idx;
    const uint32_t lane = __lane_id();
    const uint32_t H = 1u << x.lg;
    const uint32_t *hkey = x.hkey + (uint64_t)qi * H, *hval = x.hval + (uint64_t)qi * H;
    const uint32_t *part = x.part + (uint64_t)qi * x.part_stride;
    uint32_t *masks = x.masks + (uint64_t)qi * x.mask_stride;
    const uint32_t nw = kBlocksPerQuery * (kT / kWave);
    for (uint32_t i = sub * (kT / kWave) + threadIdx.x / kWave; i < np; i += nw) {
        const uint32_t pw = part[i];
        const uint32_t w = pw & 0x7fffffffu, cls = pw >> 31;
        uint32_t *M = masks + (uint64_t)i * W;
        if (lane == 0) atomicOr(&M[pb >> 5], 1u << (pb & 31));
        const uint64_t s0 = g.s_off[w];
        const uint32_t dw = (uint32_t)(g.s_off[w + 1] - s0);
        for (uint32_t t = lane; t < dw; t += kWave) {
            const uint32_t e = g.s_adj[s0 + t];
            const uint32_t key = e >> 1;
            if (key == b_idx) continue;
            uint32_t h = edge_hash(key, x.lg);
            for (;;) {
                const uint32_t k = hkey[h];
                if (k == kNone) break;
                if (k == key) {
                    const uint32_t v = hval[h];
                    const uint32_t p = v >> 1;
                    if (((v ^ e) & 1u) == cls) atomicOr(&M[p >> 5], 1u << (p & 31));
                    break;
                }
                h = (h + 1) & (H - 1);
            }
        }
    }
}

// kBlocksPerQuery workgroups per query, one wave per partner i:
// C(|M_i n M_j| - 1, 2) over the partners j > i
__global__ void __launch_bounds__(kT) k_edge_pairs(EdgeScratch x)
{
    const uint32_t qi = blockIdx.x / kBlocksPerQuery, sub = blockIdx.x % kBlocksPerQuery;
    const uint32_t *ctl = x.ctl + 8 * qi;
    const uint32_t np = ctl[4], W = ctl[3];
    const uint32_t *masks = x.masks + (uint64_t)qi * x.mask_stride;
    const uint32_t lane = __lane_id();
    const uint32_t nw = kBlocksPerQuery * (kT / kWave);
    uint64_t acc = 0;
    for (uint32_t i = sub * (kT / kWave) + threadIdx.x / kWave; i < np; i += nw) {
        const uint32_t *Mi = masks + (uint64_t)i * W;
        for (uint32_t j = i + 1 + lane; j < np; j += kWave) {
            const uint32_t *Mj = masks + (uint64_t)j * W;
            uint32_t n = 0;
            for (uint32_t w = 0; w < W; w++) n += __popc(Mi[w] & Mj[w]);
            if (n >= 3) acc += (uint64_t)(n - 1) * (n - 2) / 2;
        }
    }
    acc = wave_sum<uint64_t>(acc);
    if (lane == 0 && acc) atomicAdd(&x.result[qi], (unsigned long long)acc);
}

}  // namespace

hipError_t edge_inverse(const CsrView &g, uint32_t s_base, uint32_t n_s, const EdgeScratch &x,
                        hipStream_t s)
{
    const uint32_t grid = std::max(1u, std::min((n_s + kT - 1) / kT, 4096u));
    hipLaunchKernelGGL(k_edge_inverse, dim3(grid), dim3(kT), 0, s, g, s_base, n_s, x);
    return hipGetLastError();
}

hipError_t edge_through(const CsrView &g, const EdgeQuery *q, uint32_t n, const EdgeScratch &x,
                        hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipError_t e = fill_u64(x.result, 0, n, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_edge_setup, dim3(n), dim3(kSetupThreads), 0, s, g, q, x);
    hipLaunchKernelGGL(k_edge_masks, dim3(n * kBlocksPerQuery), dim3(kT), 0, s, g, q, x);
    hipLaunchKernelGGL(k_edge_pairs, dim3(n * kBlocksPerQuery), dim3(kT), 0, s, x);
    return hipGetLastError();
}

}  // namespace bbc
