// prims.hip -- device-wide exclusive scan and stable LSD radix sort for gfx950.
//
// Both are written for 64-wide wavefronts: tiles of 256 threads (4 waves)
// x 8 items, wave-level scans with cross-lane shuffles, and (in the sort)
// stable in-tile ranking from 8 ballots per item.
#include "bbc_dev.h"

namespace bbc {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v)
{
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T x = __shfl_up(v, o, kWave);
        if (lane >= o) v += x;
    }
    return v;
}

// Exclusive scan of one value per thread over a 256-thread block; returns
// the prefix and writes the block total to *total.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *total)
{
    __shared__ T wsum[kThreads / kWave];
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    T inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    T base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kThreads / kWave; i++) {
        T s = wsum[i];
        if (i < w) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kThreads) k_tile_sums(const TI *__restrict__ in, uint64_t n,
                                                        TO *__restrict__ sums)
{
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    TO s = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
        if (i < n) s += (TO)in[i];
    }
    TO tot;
    block_excl_scan<TO>(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// In-place exclusive scan of the per-tile sums with one block (any length).
template <typename TO>
__global__ void __launch_bounds__(kThreads) k_scan_sums(TO *__restrict__ sums, uint64_t nt)
{
    TO carry = 0;
    for (uint64_t b = 0; b < nt; b += kThreads) {
        uint64_t i = b + threadIdx.x;
        TO v = i < nt ? sums[i] : 0;
        TO tot;
        TO ex = block_excl_scan<TO>(v, &tot);
        if (i < nt) sums[i] = carry + ex;
        carry += tot;
    }
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(kThreads) k_scan_tiles(const TI *__restrict__ in,
                                                         TO *__restrict__ out, uint64_t n,
                                                         const TO *__restrict__ sums)
{
    const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
    TI v[kItems];
    TO s = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        v[j] = base + j < n ? in[base + j] : 0;
        s += (TO)v[j];
    }
    TO tot;
    TO run = sums[blockIdx.x] + block_excl_scan<TO>(s, &tot);
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        if (base + j < n) out[base + j] = run;
        run += (TO)v[j];
    }
    // the thread whose range ends at or covers position n writes the total
    if (base <= n && n <= base + kItems) out[n] = run;
}

template <typename TI, typename TO>
hipError_t scan_impl(const TI *in, TO *out, uint64_t n, void *tmp, size_t tmp_bytes,
                     hipStream_t s)
{
    uint64_t nt = (n + kTile - 1) / kTile;
    if (nt == 0) {
        return hipMemsetAsync(out, 0, sizeof(TO), s);
    }
    if (tmp_bytes < nt * sizeof(TO)) return hipErrorInvalidValue;
    TO *sums = (TO *)tmp;
    hipLaunchKernelGGL((k_tile_sums<TI, TO>), dim3(nt), dim3(kThreads), 0, s, in, n, sums);
    hipLaunchKernelGGL((k_scan_sums<TO>), dim3(1), dim3(kThreads), 0, s, sums, nt);
    hipLaunchKernelGGL((k_scan_tiles<TI, TO>), dim3(nt), dim3(kThreads), 0, s, in, out, n, sums);
    return hipGetLastError();
}

// ------------------------------------------------------------ radix sort
constexpr int kRadix = 256;

__global__ void __launch_bounds__(kThreads) k_radix_hist(const uint64_t *__restrict__ keys,
                                                         uint64_t n, int shift, uint64_t nt,
                                                         uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nt + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: items of a tile keep their order within each digit. Items
// are taken 256 at a time (one per thread, thread order = input order);
// inside a wave, lanes with equal digits are found with 8 ballots; waves of
// the block are ordered through per-wave digit counts in LDS.
__global__ void __launch_bounds__(kThreads) k_radix_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, uint64_t n, int shift, uint64_t nt,
    const uint32_t *__restrict__ offs)
{
    __shared__ uint32_t run[kRadix];
    __shared__ uint32_t wcnt[kThreads / kWave][kRadix];
    const int t = threadIdx.x, w = t / kWave;
    run[t] = offs[(uint64_t)t * nt + blockIdx.x];
#pragma unroll
    for (int i = 0; i < kThreads / kWave; i++) wcnt[i][t] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    const uint64_t lt = lanemask_lt();
    for (int j = 0; j < kItems; j++) {
        uint64_t i = base + (uint64_t)j * kThreads + t;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0;
        uint32_t val = valid ? vin[i] : 0;
        uint32_t d = (uint32_t)(key >> shift) & (kRadix - 1);
        uint64_t m = ballot64(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            bool bit = (d >> b) & 1;
            uint64_t bb = ballot64(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t rank = __popcll(m & lt);
        if (valid && rank == 0) wcnt[w][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int x = 0; x < w; x++) pos += wcnt[x][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int x = 0; x < kThreads / kWave; x++) {
            add += wcnt[x][t];
            wcnt[x][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

}  // namespace

size_t scan_tmp_bytes(uint64_t n) { return ((n + kTile - 1) / kTile + 1) * sizeof(uint64_t); }

hipError_t scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t n, void *tmp,
                           size_t tmp_bytes, hipStream_t s)
{
    return scan_impl<uint32_t, uint64_t>(in, out, n, tmp, tmp_bytes, s);
}

size_t radix_tmp_bytes(uint64_t n)
{
    uint64_t nt = (n + kTile - 1) / kTile;
    uint64_t nh = nt * kRadix;
    return 256 + nh * sizeof(uint32_t) * 2 + sizeof(uint32_t) + scan_tmp_bytes(nh) * 2;
}

hipError_t radix_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint64_t n,
                      int bits, void *tmp, size_t tmp_bytes, hipStream_t s)
{
    if (n <= 1 || bits <= 0) return hipSuccess;
    if (n >= (1ull << 32)) return hipErrorInvalidValue;
    if (tmp_bytes < radix_tmp_bytes(n)) return hipErrorInvalidValue;
    uint64_t nt = (n + kTile - 1) / kTile;
    uint64_t nh = nt * kRadix;
    uint32_t *hist = (uint32_t *)tmp;
    uint32_t *offs = hist + nh;
    void *stmp = (void *)(((uintptr_t)(offs + nh + 1) + 255) & ~(uintptr_t)255);
    size_t stmp_bytes = tmp_bytes - ((char *)stmp - (char *)tmp);
    int passes = (bits + 7) / 8;
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(nt), dim3(kThreads), 0, s, ka, n, shift, nt, hist);
        hipError_t e = scan_impl<uint32_t, uint32_t>(hist, offs, nh, stmp, stmp_bytes, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(nt), dim3(kThreads), 0, s, ka, va, kb, vb, n,
                           shift, nt, offs);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    if (ka != k0) {
        hipError_t e = hipMemcpyAsync(k0, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(v0, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace bbc
