// bbwc.hip -- Algorithm 1 (BBWC, wedge-centric counting) for p = 3 on the
// anchor side, as a second, independent GPU path.
//
// For an anchor u and every v in N(u), each pair w1 > w2 (by priority,
// Definition 4.1) of neighbours of v ranked below u forms a signed 3-wedge
// <u, w1, w2, v>; Lemma 1 puts all wedges of a balanced biclique in one of
// the 4 wedge types, so the wedges are counted in buckets keyed by (w1, w2)
// and type, and every bucket of size n adds C(n, q). Unlike Algorithm 2 this
// enumerates wedge pairs, not candidate pairs, and orients to lower-priority
// partners; the two paths share only the CSR.

#include "bbc_build.h"
#include "bbc_bbwc.h"

namespace bbc {

namespace {

constexpr int kT = 256;
constexpr unsigned long long kEmptyKey = ~0ull;

__device__ __forceinline__ uint32_t bbwc_hash(unsigned long long key, uint32_t lg)
{
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - lg));
}

// C(n, q) for q <= 7 in 128 bits (each step C(n, i) (n - i) / (i + 1) is
// exact); ovf is set when the result needs more than 64 bits
__device__ __forceinline__ unsigned long long bbwc_choose(uint64_t n, uint32_t q, bool &ovf)
{
    if (n < q) return 0;
    unsigned __int128 c = 1;
    for (uint32_t i = 0; i < q; i++) c = c * (n - i) / (i + 1);
    if (c >> 64) ovf = true;
    return (unsigned long long)c;
}

// One workgroup at a time per anchor: insert the anchor's wedge pairs into
// the workgroup's table (key, 4 type counters), then sum C(n, q) over the
// used slots and clear them.
__global__ void __launch_bounds__(kT) k_bbwc(BbwcArgs A)
{
    __shared__ uint32_t sh_anchor, sh_used;
    __shared__ unsigned long long sh_pairs;
    const uint32_t tid = threadIdx.x, lane = __lane_id();
    const CsrView &g = A.g;
    const uint32_t cap = 1u << A.lg;
    unsigned long long *keys = A.keys + (uint64_t)blockIdx.x * cap;
    uint32_t *cnt = A.cnt + (uint64_t)blockIdx.x * cap * 4;
    uint32_t *used = A.used + (uint64_t)blockIdx.x * cap;
    unsigned long long total = 0;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            sh_anchor = atomicAdd(A.cursor, 1u);
            sh_used = 0;
            sh_pairs = 0;
        }
        __syncthreads();
        const uint32_t r = sh_anchor;
        if (r >= A.a1 - A.a0) break;
        const uint32_t u = A.a0 + r;
        const uint64_t s0 = g.s_off[u];
        const uint32_t du = (uint32_t)(g.s_off[u + 1] - s0);
        // wedge pairs of the anchor: sum over v of C(prefix below u, 2); the
        // prefix of v's list (sorted by rank) ends at u's own entry
        for (uint32_t t = tid; t < du; t += kT) {
            const uint32_t v = g.s_adj[s0 + t] >> 1;
            const uint64_t o0 = g.o_off[v];
            uint64_t lo = o0, hi = g.o_off[v + 1];
            while (lo < hi) {
                const uint64_t mid = (lo + hi) / 2;
                if ((g.o_adj[mid] >> 1) < u) lo = mid + 1; else hi = mid;
            }
            const uint64_t L = lo - o0;
            atomicAdd(&sh_pairs, (unsigned long long)(L * (L - (L > 0)) / 2));
        }
        __syncthreads();
        if (sh_pairs > (unsigned long long)(cap - cap / 4)) {
            if (tid == 0) atomicOr(A.flags, 1u);   // anchor too large for the table
            continue;
        }
        // insert: thread t takes wedge pairs of position t's prefix
        for (uint32_t t = 0; t < du; t++) {
            const uint32_t e = g.s_adj[s0 + t];
            const uint32_t v = e >> 1, su = e & 1u;
            const uint64_t o0 = g.o_off[v];
            uint64_t lo = o0, hi = g.o_off[v + 1];
            while (lo < hi) {
                const uint64_t mid = (lo + hi) / 2;
                if ((g.o_adj[mid] >> 1) < u) lo = mid + 1; else hi = mid;
            }
            const uint32_t L = (uint32_t)(lo - o0);
            const uint64_t np = (uint64_t)L * (L - (L > 0)) / 2;
            for (uint64_t k = tid; k < np; k += kT) {
                // pair index k -> (i > j) with i in [1, L): k = i (i - 1) / 2 + j
                uint32_t i = (uint32_t)((sqrt(8.0 * (double)k + 1.0) + 1.0) / 2.0);
                while ((uint64_t)i * (i - 1) / 2 > k) i--;
                while ((uint64_t)(i + 1) * i / 2 <= k) i++;
                const uint32_t j = (uint32_t)(k - (uint64_t)i * (i - 1) / 2);
                const uint32_t e1 = g.o_adj[o0 + i], e2 = g.o_adj[o0 + j];   // rank(e1) > rank(e2)
                const unsigned long long key = ((unsigned long long)(e1 >> 1) << 32) | (e2 >> 1);
                const uint32_t type = (((e1 & 1u) ^ su) << 1) | ((e2 & 1u) ^ su);
                uint32_t h = bbwc_hash(key, A.lg);
                for (;;) {
                    const unsigned long long old = atomicCAS(&keys[h], kEmptyKey, key);
                    if (old == kEmptyKey) {
                        used[atomicAdd(&sh_used, 1u)] = h;
                        atomicAdd(&cnt[4 * h + type], 1u);
                        break;
                    }
                    if (old == key) { atomicAdd(&cnt[4 * h + type], 1u); break; }
                    h = (h + 1) & (cap - 1);
                }
            }
        }
        __syncthreads();
        bool ovf = false;
        for (uint32_t t = tid; t < sh_used; t += kT) {
            const uint32_t h = used[t];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const unsigned long long add = bbwc_choose(cnt[4 * h + c], A.q, ovf);
                if (total + add < total) ovf = true;
                total += add;
                cnt[4 * h + c] = 0;
            }
            keys[h] = kEmptyKey;
        }
        if (ovf) atomicOr(A.flags, 2u);
    }
    // per lane, then per wave (a carry out of 64 bits is an overflow)
    bool carry = false;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_xor(total, o, kWave);
        carry |= total + other < total;
        total += other;
    }
    if (carry) atomicOr(A.flags, 2u);
    if (lane == 0 && total) {
        const unsigned long long old = atomicAdd(A.total, total);
        if (old + total < old) atomicOr(A.flags, 2u);
    }
}

}  // namespace

hipError_t bbwc_count(const BbwcArgs &A, uint32_t grid, hipStream_t s)
{
    hipError_t e = fill_u64(A.keys, ~0ull, (uint64_t)grid << A.lg, s);
    if (e == hipSuccess) e = fill_u32(A.cnt, 0, ((uint64_t)grid << A.lg) * 4, s);
    if (e == hipSuccess) e = fill_u32(A.cursor, 0, 1, s);
    if (e == hipSuccess) e = fill_u32(A.flags, 0, 1, s);
    if (e == hipSuccess) e = fill_u64(A.total, 0, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bbwc, dim3(grid), dim3(kT), 0, s, A);
    return hipGetLastError();
}

}  // namespace bbc
