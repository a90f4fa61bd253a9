// runtime.cpp -- host runtime and C ABI of libbbc.
//
// Owns device memory (a caching allocator under the context's cap), graph
// sets, count workspaces, the batched path (persistent kernels replayed from
// a captured HIP graph, launch shape chosen by a small autotuner), and the
// serving loop (continuous batching over several streams).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "bbc.h"
#include "bbc_build.h"
#include "bbc_count.h"
#include "bbc_edge.h"
#include "bbc_bbwc.h"

using namespace bbc;

namespace {

struct HipError {
    hipError_t e;
    const char *what;
};

#define HIP_OK(expr)                                                 \
    do {                                                             \
        hipError_t e_ = (expr);                                      \
        if (e_ != hipSuccess) throw HipError{e_, #expr};             \
    } while (0)

struct StatusError {
    bbc_status s;
    std::string msg;
};

[[noreturn]] void fail(bbc_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    throw StatusError{s, buf};
}

int bit_width(uint64_t x)
{
    int b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------- allocator
// Allocations are tagged by the thread that makes them: the serving workers
// tag theirs 1, everything else is 0. The serving admission charges live
// tag-0 memory (graphs and workspaces of the caller's own calls) against the
// cap and reserves the rest per admitted batch.
thread_local int tl_alloc_tag = 0;

class Allocator {
  public:
    Allocator(uint64_t cap) : cap_(cap) {}
    // Arena mode: every allocation is carved from [base, base + size) by a
    // bump pointer and nothing is freed until arena_reset(); no device memory
    // is ever allocated or freed.
    Allocator(void *base, uint64_t size) : cap_(size), arena_((char *)base) {}
    ~Allocator() { release_all(); }

    void *alloc(uint64_t bytes)
    {
        if (bytes == 0) bytes = 256;
        bytes = round_up(bytes, 256);
        const int tag = tl_alloc_tag;
        std::lock_guard<std::mutex> lk(mu_);
        if (arena_) {
            if (used_ + bytes > cap_)
                fail(BBC_E_NOMEM, "the count needs more than the %llu-byte static scratch of the "
                                  "no-allocation entry point (%llu bytes more)",
                     (unsigned long long)cap_, (unsigned long long)(used_ + bytes - cap_));
            void *p = arena_ + used_;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return p;
        }
        auto it = free_.lower_bound(bytes);
        if (it != free_.end() && it->first <= bytes * 2 + (4u << 20)) {
            void *p = it->second;
            live_[p] = Live{it->first, tag};
            live_tag_[tag] += it->first;
            free_.erase(it);
            return p;
        }
        uint64_t sz = bytes < (1u << 20) ? bytes : round_up(bytes, 2u << 20);
        if (cap_ && used_ + sz > cap_) {
            trim_locked();
            if (used_ + sz > cap_)
                fail(BBC_E_NOMEM, "device memory cap %llu bytes reached (need %llu more, %llu in use)",
                     (unsigned long long)cap_, (unsigned long long)sz, (unsigned long long)used_);
        }
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim_locked();
            e = hipMalloc(&p, sz);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                fail(BBC_E_NOMEM, "hipMalloc of %llu bytes failed", (unsigned long long)sz);
            }
        }
        used_ += sz;
        peak_ = std::max(peak_, used_);
        live_[p] = Live{sz, tag};
        live_tag_[tag] += sz;
        return p;
    }

    void free(void *p)
    {
        if (!p || arena_) return;
        std::lock_guard<std::mutex> lk(mu_);
        auto it = live_.find(p);
        if (it == live_.end()) return;
        free_.emplace(it->second.bytes, p);
        live_tag_[it->second.tag] -= it->second.bytes;
        live_.erase(it);
    }

    uint64_t used()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return used_;
    }
    uint64_t cap() const { return cap_; }
    uint64_t peak()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return peak_;
    }
    uint64_t live(int tag)
    {
        std::lock_guard<std::mutex> lk(mu_);
        return live_tag_[tag & 1];
    }

    void release_all()
    {
        std::lock_guard<std::mutex> lk(mu_);
        trim_locked();
    }

    void arena_reset()
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (arena_) used_ = 0;
    }

  private:
    struct Live { uint64_t bytes; int tag; };
    void trim_locked()
    {
        for (auto &kv : free_) {
            (void)hipFree(kv.second);
            used_ -= kv.first;
        }
        free_.clear();
    }
    std::mutex mu_;
    uint64_t cap_, used_ = 0, peak_ = 0;
    char *arena_ = nullptr;
    uint64_t live_tag_[2] = {0, 0};
    std::multimap<uint64_t, void *> free_;
    std::unordered_map<void *, Live> live_;
};

// A device buffer that returns its memory to the allocator.
struct DBuf {
    Allocator *al = nullptr;
    void *p = nullptr;
    uint64_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { reset(); }
    void reset()
    {
        if (p && al) {
            // A buffer released while an exception unwinds the stack may still
            // be read or written by copies and kernels enqueued before the
            // failure (the builder allocates between enqueues): wait for the
            // device before the allocator can hand the memory to another
            // stream or free it.
            if (std::uncaught_exceptions() > 0) (void)hipDeviceSynchronize();
            al->free(p);
        }
        p = nullptr;
        bytes = 0;
    }
    void ensure(Allocator *a, uint64_t n)
    {
        if (p && bytes >= n) return;
        reset();
        al = a;
        p = a->alloc(n);
        bytes = n;
    }
    template <typename T>
    T *as() const { return (T *)p; }
};

// Pinned host staging area (or, with use_external, memory the caller owns:
// then nothing is allocated and a request beyond its size fails).
struct HBuf {
    void *p = nullptr;
    uint64_t bytes = 0;
    bool external = false;
    void use_external(void *q, uint64_t n)
    {
        p = q;
        bytes = n;
        external = true;
    }
    ~HBuf()
    {
        if (!p || external) return;
        // as for DBuf: an in-flight copy may still read this staging memory
        if (std::uncaught_exceptions() > 0) (void)hipDeviceSynchronize();
        (void)hipHostFree(p);
    }
    void ensure(uint64_t n)
    {
        if (p && bytes >= n) return;
        if (external)
            fail(BBC_E_NOMEM, "host staging of %llu bytes exceeds the %llu-byte static buffer",
                 (unsigned long long)n, (unsigned long long)bytes);
        if (p) (void)hipHostFree(p);
        p = nullptr;
        HIP_OK(hipHostMalloc(&p, n, hipHostMallocDefault));
        bytes = n;
    }
    template <typename T>
    T *as() const { return (T *)p; }
};

}  // namespace

// ------------------------------------------------------------- graph set
struct GraphSet {
    Allocator *al;
    uint32_t G = 0, NS = 0, NO = 0;
    uint64_t M = 0;
    std::vector<GraphDesc> desc;
    DBuf d_desc, s_off, o_off, s_adj, o_adj, s_graph, s_vert;
    DBuf s_suf;
    // sizing hints learnt by earlier counts
    uint64_t hint_masks = 0, hint_cands = 0, hint_units = 0;
    // oriented wedges through the opposite sides, sum over graphs of
    // sum_o C(d_o, 2) (the first workspace guess of a single graph)
    uint64_t wedges_o = 0;
    uint32_t max_deg = 0;   // largest vertex degree of the set, either side
    // anchor-side tuning of a single large graph: shape key and side used
    uint64_t tune_key = 0;
    uint32_t tune_side = 0;
    uint64_t device_bytes() const
    {
        return d_desc.bytes + s_off.bytes + o_off.bytes + s_adj.bytes + o_adj.bytes +
               s_suf.bytes + s_graph.bytes + s_vert.bytes;
    }
    CsrView view() const
    {
        CsrView v;
        memset(&v, 0, sizeof(v));
        v.G = G; v.NS = NS; v.NO = NO; v.M = M;
        v.s_off = s_off.as<uint64_t>(); v.s_adj = s_adj.as<uint32_t>();
        v.o_off = o_off.as<uint64_t>(); v.o_adj = o_adj.as<uint32_t>();
        v.s_suf = s_suf.as<uint2>();
        v.s_graph = s_graph.as<uint32_t>(); v.s_vert = s_vert.as<uint32_t>();
        v.desc = d_desc.as<GraphDesc>();
        return v;
    }
};

struct bbc_graph {
    std::shared_ptr<GraphSet> set;
    uint32_t idx;
};

namespace {

// Count workspace (one per stream that counts).
struct Work {
    DBuf ctr, anchors, units, masks, cands, defer0, defer1, defer2, defer3, defer4, gtab, dtab, bscr, count,
        carry, pv, pv_o, pv_slot;
    DBuf ucnt, uoff, ptmp;
    HBuf host;          // counters + counts + carries read back
    HBuf bhost;         // small staging of the CSR builder
    HBuf coo;           // pinned COO staging of the serving loop
    uint64_t cap_anchors = 0, cap_units = 0, cap_masks = 0, cap_cands = 0, cap_defer = 0;
    uint32_t gtab_blocks = 0, dtab_blocks = 0, bscr_blocks = 0;
    uint64_t gtab_words = 0, dtab_words = 0, bscr_words = 0, ptmp_bytes = 0;
    uint32_t gH = 0, dH = 0;
    int glog2 = 0, dlog2 = 0;
    uint32_t gmaxd = 0, gkmax = 0;
    Allocator *arena = nullptr;   // no-allocation counts: every buffer from this arena
    uint32_t mask_chunk = 1u << 16, cand_chunk = 1u << 13;   // output chunks of the last count
    uint32_t wv_mask_chunk = 4096, wv_cand_chunk = 4096;
    // captured replay of a batched count
    hipGraphExec_t exec = nullptr;
    std::vector<unsigned char> exec_args;   // bytes of the LaunchArgs it was captured with
    ~Work()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
    uint64_t device_bytes() const
    {
        uint64_t b = 0;
        for (const DBuf *x : {&ctr, &anchors, &units, &masks, &cands, &defer0, &defer1, &defer2,
                              &defer3, &defer4, &gtab, &dtab, &bscr, &count, &carry, &pv, &pv_o,
                              &pv_slot, &ucnt, &uoff, &ptmp})
            b += x->bytes;
        return b;
    }
    // Return every device buffer to the allocator (the pinned host buffers
    // stay); the next count sizes the workspace again.
    void release_device()
    {
        for (DBuf *b : {&ctr, &anchors, &units, &masks, &cands, &defer0, &defer1, &defer2, &defer3,
                        &defer4, &gtab, &dtab, &bscr, &count, &carry, &pv, &pv_o, &pv_slot, &ucnt,
                        &uoff, &ptmp})
            b->reset();
        cap_anchors = cap_units = cap_masks = cap_cands = cap_defer = 0;
        gtab_blocks = dtab_blocks = bscr_blocks = 0;
        gtab_words = dtab_words = bscr_words = ptmp_bytes = 0;
        gH = dH = 0;
        glog2 = dlog2 = 0;
        gmaxd = gkmax = 0;
        if (exec) { (void)hipGraphExecDestroy(exec); exec = nullptr; }
        exec_args.clear();
    }
};

// Launch shape. The defaults, measured on the Chung-Lu graphs of 2M x 500k
// vertices and 40M edges and of 100k x 50k vertices and 2M edges: a unit
// column base of 4096 against 2048 is 2.3% faster on the larger and neutral
// on the smaller; 4 triplet workgroups per compute unit against 6 are 2%
// faster on the smaller and neutral on the larger.
struct Shape {
    uint32_t chunk_base = 4096;
    uint32_t grid_a_per_cu = 2;
    uint32_t grid_t_per_cu = 4;
};

}  // namespace

struct Request {
    bbc_ticket id;
    std::shared_ptr<GraphSet> set;   // prebuilt graph (set + index) or null
    uint32_t idx = 0;
    // COO request
    uint32_t n_u = 0, n_v = 0, flags = 0;
    std::vector<uint32_t> eu, ev;
    std::vector<uint8_t> sign;
    uint64_t m = 0;
    uint32_t max_deg = 0;     // largest vertex degree (COO requests: counted at submission)
    uint64_t w2_max = 0;      // oriented wedges of the costlier anchor side
    uint32_t n_s_max = 0;     // larger side
    int nomem_retries = 0;    // requeued after running out of memory behind other batches
    bool done = false;
    bbc_status status = BBC_OK;
    int64_t result = 0;
};

struct bbc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int num_cus = 256;
    std::unique_ptr<Allocator> al;
    std::string last_error;
    std::mutex err_mu;
    Work work;
    bbc_count_stats stats{};
    bool timing = false;
    // test hooks (bbc_set_test_hook): host-forced conditions
    bool hook_no_window = false;
    uint64_t hook_preload = 0;
    bool hook_shape_set = false;
    Shape hook_shape;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    std::map<uint64_t, Shape> tuned;   // autotuner cache by size class
    struct SideTime { float ms[2] = {0, 0}; bool tried[2] = {false, false}; };
    std::map<uint64_t, SideTime> side_tune;   // anchor side by graph shape
    // workspace sizes a count of a graph shape needed (size class and side):
    // a later graph of the same shape starts from them instead of from the
    // edge-count guess, which saves a rerun on graphs with heavy anchors
    struct WsHint { uint64_t masks = 0, cands = 0, units = 0; };
    std::map<uint64_t, WsHint> ws_hint;
    std::mutex tune_mu;
    hipEvent_t tev[2] = {nullptr, nullptr};
    // serving
    std::mutex q_mu;
    std::condition_variable q_cv, done_cv;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<bbc_ticket, std::shared_ptr<Request>> requests;
    uint64_t next_ticket = 1;
    uint64_t admitted_bytes = 0;    // reservations of the batches in flight
    int serve_large = 0;            // workers holding a large request
    int serve_small_gpu = 0;        // batches of small requests building or counting
    std::condition_variable small_cv;
    uint64_t peak_admitted = 0;
    uint64_t peak_queued = 0;
    // graph handles the caller holds (released by bbc_graph_free or on destroy)
    std::mutex g_mu;
    std::unordered_set<bbc_graph *> graphs;
    bool stopping = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> serve_streams;
};

namespace {

void set_error(bbc_ctx *ctx, const std::string &m)
{
    if (!ctx) return;
    std::lock_guard<std::mutex> lk(ctx->err_mu);
    ctx->last_error = m;
}

template <typename F>
bbc_status guard(bbc_ctx *ctx, F &&f)
{
    try {
        f();
        set_error(ctx, "");
        return BBC_OK;
    } catch (const StatusError &e) {
        set_error(ctx, e.msg);
        return e.s;
    } catch (const HipError &e) {
        set_error(ctx, std::string(e.what) + ": " + hipGetErrorString(e.e));
        (void)hipGetLastError();
        return BBC_E_HIP;
    } catch (const std::bad_alloc &) {
        set_error(ctx, "host allocation failed");
        return BBC_E_NOMEM;
    }
}

// -------------------------------------------------------------- building
struct CooIn {
    uint32_t G;
    const uint32_t *n_u, *n_v;
    const uint64_t *edge_off;    // host [G+1]
    const uint32_t *eu, *ev;
    const void *sign;
    uint32_t flags;
};

uint64_t sign_bytes(uint64_t m, uint32_t flags)
{
    return (flags & BBC_SIGNS_2BIT_PACKED) ? (m + 3) / 4 : m;
}

void check_flags(uint32_t flags)
{
    const uint32_t known = BBC_IN_DEVICE_PTRS | BBC_SIGNS_2BIT_PACKED | BBC_SIGNS_01 |
                           BBC_ANCHOR_U | BBC_ANCHOR_V | BBC_ANCHOR_SMALLER;
    if (flags & ~known) fail(BBC_E_INVAL, "unknown flag bits 0x%x", flags & ~known);
    if ((flags & BBC_SIGNS_2BIT_PACKED) && (flags & BBC_SIGNS_01))
        fail(BBC_E_INVAL, "BBC_SIGNS_2BIT_PACKED and BBC_SIGNS_01 are exclusive");
    int a = !!(flags & BBC_ANCHOR_U) + !!(flags & BBC_ANCHOR_V) + !!(flags & BBC_ANCHOR_SMALLER);
    if (a > 1) fail(BBC_E_INVAL, "at most one BBC_ANCHOR_* flag");
}

// Anchor side of one graph. Work of the pair table anchored on S is about the
// number of 2-hop wedges through O, sum_o C(d_o, 2); work of the triplet
// phase grows with the mask width, about the edge-weighted mean degree of S.
// The ratio of the two sides' wedge counts (larger / smaller) goes to
// *wedge_ratio.
uint32_t choose_side(uint32_t flags, uint32_t n_u, uint32_t n_v, uint64_t m, uint64_t c2_u,
                     uint64_t c2_v, uint64_t d2_u, uint64_t d2_v, double *wedge_ratio = nullptr)
{
    if (wedge_ratio) {
        const double lo = (double)std::min(c2_u, c2_v), hi = (double)std::max(c2_u, c2_v);
        *wedge_ratio = lo > 0 ? hi / lo : 1e30;
    }
    if (flags & BBC_ANCHOR_U) return 0;
    if (flags & BBC_ANCHOR_V) return 1;
    if (flags & BBC_ANCHOR_SMALLER) return n_v < n_u ? 1 : 0;
    if (m == 0) return 0;
    double wu = (double)d2_u / (double)m, wv = (double)d2_v / (double)m;
    double cost_u = (double)c2_v * (1.0 + wu / 32.0);   // anchored on U: wedges centred in V
    double cost_v = (double)c2_u * (1.0 + wv / 32.0);
    return cost_v < cost_u ? 1 : 0;
}

constexpr uint64_t kSideTuneMinEdges = 1u << 18;
// Only shapes whose two sides' wedge counts (the pair-phase work) are within
// this factor are timed on both sides; beyond it the estimate's side is kept
// (a 2M x 500k power-law graph with 2.3x the wedges on one side counts 16x
// slower there: timing it once would cost more than the estimate can lose).
constexpr double kSideTuneMaxRatio = 2.0;
// vertex slots (|U| + |V| over the set) up to which the ingest counts degrees
// in per-XCD copies (8 words per slot)
constexpr uint64_t kDegCopyMaxSlots = 1u << 22;

// Graphs with the same size classes and degree-statistic ratio share a key.
uint64_t side_key(uint32_t n_u, uint32_t n_v, uint64_t m, uint64_t c2_u, uint64_t c2_v,
                  uint64_t d2_u, uint64_t d2_v)
{
    auto lb = [](double x) { return x > 1 ? (int)std::lround(4.0 * std::log2(x)) : 0; };
    const int r1 = lb(1.0 + (double)c2_u / (1.0 + (double)c2_v) * 64.0);
    const int r2 = lb(1.0 + (double)d2_u / (1.0 + (double)d2_v) * 64.0);
    return ((uint64_t)bit_width(n_u) << 56) | ((uint64_t)bit_width(n_v) << 48) |
           ((uint64_t)bit_width(m) << 40) | ((uint64_t)(r1 & 0xfff) << 20) | (uint64_t)(r2 & 0xfff) | 1;
}

std::shared_ptr<GraphSet> build_set(bbc_ctx *ctx, const CooIn &in, hipStream_t s, HBuf &hb)
{
    Allocator *al = ctx->al.get();
    const uint32_t G = in.G;
    if (G == 0) fail(BBC_E_INVAL, "no graphs");
    check_flags(in.flags);
    const uint64_t M = in.edge_off[G];
    uint64_t NU = 0, NV = 0;
    for (uint32_t g = 0; g < G; g++) {
        if (in.edge_off[g + 1] < in.edge_off[g]) fail(BBC_E_INVAL, "edge offsets decrease at graph %u", g);
        NU += in.n_u[g];
        NV += in.n_v[g];
    }
    if (in.edge_off[0] != 0) fail(BBC_E_INVAL, "edge_offsets[0] must be 0");
    if (M > 0 && (!in.eu || !in.ev || !in.sign)) fail(BBC_E_INVAL, "null edge array");
    if (M >= (1ull << 32) - 1) fail(BBC_E_UNSUPPORTED, "more than 2^32-2 edges in one build");
    if (NU >= (1ull << 31) || NV >= (1ull << 31)) fail(BBC_E_UNSUPPORTED, "more than 2^31-1 vertices per side");

    auto set = std::make_shared<GraphSet>();
    set->al = al;
    set->G = G;
    set->M = M;
    set->desc.resize(G);

    // inputs on the device
    DBuf d_eu, d_ev, d_sign;
    const uint32_t *eu = in.eu, *ev = in.ev;
    const void *sign = in.sign;
    const uint64_t sb = sign_bytes(M, in.flags);
    if (!(in.flags & BBC_IN_DEVICE_PTRS) && M > 0) {
        d_eu.ensure(al, M * 4); d_ev.ensure(al, M * 4); d_sign.ensure(al, sb);
        HIP_OK(hipMemcpyAsync(d_eu.p, in.eu, M * 4, hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(d_ev.p, in.ev, M * 4, hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(d_sign.p, in.sign, sb, hipMemcpyHostToDevice, s));
        eu = d_eu.as<uint32_t>(); ev = d_ev.as<uint32_t>(); sign = d_sign.p;
    }

    // per-graph descriptors: U/V slot bases
    std::vector<uint32_t> ub(G), vb(G);
    {
        uint64_t u = 0, v = 0;
        for (uint32_t g = 0; g < G; g++) {
            GraphDesc &d = set->desc[g];
            memset(&d, 0, sizeof(d));
            d.n_u = in.n_u[g]; d.n_v = in.n_v[g];
            d.u_base = (uint32_t)u; d.v_base = (uint32_t)v;
            d.e_base = in.edge_off[g]; d.m = in.edge_off[g + 1] - in.edge_off[g];
            ub[g] = (uint32_t)u; vb[g] = (uint32_t)v;
            u += d.n_u; v += d.n_v;
        }
    }
    // small per-graph arrays in one device block
    const uint64_t small_bytes = (G + 1) * 8 + G * sizeof(GraphDesc) + 4 * G * 4 + 4 * G * 8 + 64;
    DBuf d_small;
    d_small.ensure(al, small_bytes);
    char *sp = d_small.as<char>();
    uint64_t *d_eoff = (uint64_t *)sp; sp += (G + 1) * 8;
    GraphDesc *d_desc_tmp = (GraphDesc *)sp; sp += G * sizeof(GraphDesc);
    uint32_t *d_ub = (uint32_t *)sp; sp += G * 4;
    uint32_t *d_vb = (uint32_t *)sp; sp += G * 4;
    uint32_t *d_sbase = (uint32_t *)sp; sp += G * 4;
    uint32_t *d_obase = (uint32_t *)sp; sp += G * 4;
    unsigned long long *d_stats = (unsigned long long *)sp; sp += 4 * G * 8;
    uint32_t *d_flags = (uint32_t *)sp;   // err, max_deg_u, max_deg_v, pad, first_bad (u64)

    hb.ensure((G + 1) * 8 + G * sizeof(GraphDesc) + 4 * G * 4 + 4 * G * 8 + 64);
    {
        char *hp = hb.as<char>();
        memcpy(hp, in.edge_off, (G + 1) * 8);
        memcpy(hp + (G + 1) * 8, set->desc.data(), G * sizeof(GraphDesc));
        memcpy(hp + (G + 1) * 8 + G * sizeof(GraphDesc), ub.data(), G * 4);
        memcpy(hp + (G + 1) * 8 + G * sizeof(GraphDesc) + G * 4, vb.data(), G * 4);
        HIP_OK(hipMemcpyAsync(d_small.p, hp, (G + 1) * 8 + G * sizeof(GraphDesc) + 2 * G * 4,
                              hipMemcpyHostToDevice, s));
    }
    DBuf eg, deg_u, deg_v, deg_x;
    eg.ensure(al, std::max<uint64_t>(M, 1) * 4);
    deg_u.ensure(al, std::max<uint64_t>(NU, 1) * 4);
    deg_v.ensure(al, std::max<uint64_t>(NV, 1) * 4);
    // per-XCD degree copies (k_ingest) while they stay small
    const bool xcd_copies = NU + NV <= kDegCopyMaxSlots;
    if (xcd_copies) {
        deg_x.ensure(al, (uint64_t)kXcd * (NU + NV) * 4);
        HIP_OK(fill_u32(deg_x.as<uint32_t>(), 0, (uint64_t)kXcd * (NU + NV), s));
    } else {
        HIP_OK(fill_u32(deg_u.as<uint32_t>(), 0, NU, s));
        HIP_OK(fill_u32(deg_v.as<uint32_t>(), 0, NV, s));
    }
    HIP_OK(fill_u64(d_stats, 0, 4ull * G, s));
    HIP_OK(fill_u32(d_flags, 0, 4, s));
    HIP_OK(fill_u64(d_flags + 4, ~0ull, 1, s));

    BuildArgs a;
    memset(&a, 0, sizeof(a));
    a.eu = eu; a.ev = ev; a.sign = sign; a.flags = in.flags; a.M = M; a.G = G;
    a.edge_off = d_eoff; a.desc = d_desc_tmp; a.u_base_arr = d_ub; a.v_base_arr = d_vb;
    a.NU = (uint32_t)NU; a.NV = (uint32_t)NV;
    a.eg = eg.as<uint32_t>(); a.deg_u = deg_u.as<uint32_t>(); a.deg_v = deg_v.as<uint32_t>();
    a.deg_x = xcd_copies ? deg_x.as<uint32_t>() : nullptr;
    a.err = d_flags; a.max_deg_u = d_flags + 1; a.max_deg_v = d_flags + 2;
    a.first_bad = (unsigned long long *)(d_flags + 4);
    a.stat_c2_u = d_stats; a.stat_c2_v = d_stats + G; a.stat_d2_u = d_stats + 2 * G;
    a.stat_d2_v = d_stats + 3 * G;
    const bool timed = ctx->timing && s == ctx->stream;
    if (timed) HIP_OK(hipEventRecord(ctx->ev[4], s));
    HIP_OK(build_ingest(a, s));

    // read back validation flags and degree statistics
    char *hp = hb.as<char>();
    unsigned long long *h_stats = (unsigned long long *)hp;
    uint32_t *h_flags = (uint32_t *)(hp + 4 * G * 8);
    HIP_OK(hipMemcpyAsync(h_stats, d_stats, 4 * G * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(h_flags, d_flags, 24, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const uint32_t err = h_flags[0];
    const uint64_t first_bad = *(uint64_t *)(h_flags + 4);
    if (err & kErrRange) fail(BBC_E_RANGE, "edge %llu has an endpoint out of range", (unsigned long long)first_bad);
    if (err & kErrSign) fail(BBC_E_SIGN, "edge %llu has an invalid sign", (unsigned long long)first_bad);
    const uint32_t maxdu = h_flags[1], maxdv = h_flags[2];
    set->max_deg = std::max(maxdu, maxdv);

    // side choice and S/O numbering
    uint64_t ns = 0, no = 0;
    std::vector<uint32_t> sbase(G), obase(G);
    bool any_u = false, any_v = false;
    const bool auto_side = !(in.flags & (BBC_ANCHOR_U | BBC_ANCHOR_V | BBC_ANCHOR_SMALLER));
    for (uint32_t g = 0; g < G; g++) {
        GraphDesc &d = set->desc[g];
        double ratio = 1.0;
        d.side = choose_side(in.flags, d.n_u, d.n_v, d.m, h_stats[g], h_stats[G + g],
                             h_stats[2 * G + g], h_stats[3 * G + g], &ratio);
        if (G == 1 && auto_side && d.m >= kSideTuneMinEdges && ratio <= kSideTuneMaxRatio) {
            // a recurring large shape: time each side once, then keep the faster
            const uint64_t key = side_key(d.n_u, d.n_v, d.m, h_stats[0], h_stats[1],
                                          h_stats[2], h_stats[3]);
            std::lock_guard<std::mutex> lk(ctx->tune_mu);
            auto &st = ctx->side_tune[key];
            if (st.tried[0] && st.tried[1]) d.side = st.ms[1] < st.ms[0] ? 1 : 0;
            else if (st.tried[d.side]) d.side ^= 1;
            set->tune_key = key;
            set->tune_side = d.side;
        }
        d.n_s = d.side ? d.n_v : d.n_u;
        d.n_o = d.side ? d.n_u : d.n_v;
        set->wedges_o += d.side ? h_stats[g] : h_stats[G + g];
        d.s_base = (uint32_t)ns; d.o_base = (uint32_t)no;
        sbase[g] = d.s_base; obase[g] = d.o_base;
        ns += d.n_s; no += d.n_o;
        (d.side ? any_v : any_u) = true;
    }
    set->NS = (uint32_t)ns;
    set->NO = (uint32_t)no;
    {
        char *p2 = hp;
        memcpy(p2, set->desc.data(), G * sizeof(GraphDesc));
        memcpy(p2 + G * sizeof(GraphDesc), sbase.data(), G * 4);
        memcpy(p2 + G * sizeof(GraphDesc) + G * 4, obase.data(), G * 4);
        HIP_OK(hipMemcpyAsync(d_desc_tmp, p2, G * sizeof(GraphDesc), hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(d_sbase, p2 + G * sizeof(GraphDesc), G * 4, hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(d_obase, p2 + G * sizeof(GraphDesc) + G * 4, G * 4,
                              hipMemcpyHostToDevice, s));
    }
    const uint32_t max_deg_s = std::max(any_u ? maxdu : 0u, any_v ? maxdv : 0u);
    const uint64_t NS = ns, NO = no;
    const uint64_t nkv = std::max<uint64_t>(std::max(NS, M), 1);
    DBuf key0, key1, val0, val1, deg_o, deg_rank, rank_of, tmp;
    key0.ensure(al, nkv * 8); key1.ensure(al, nkv * 8);
    val0.ensure(al, nkv * 4); val1.ensure(al, nkv * 4);
    deg_o.ensure(al, std::max<uint64_t>(NO, 1) * 4);
    deg_rank.ensure(al, std::max<uint64_t>(NS, 1) * 4);
    rank_of.ensure(al, std::max<uint64_t>(NS, 1) * 4);
    const size_t tmp_bytes = std::max(radix_tmp_bytes(nkv), scan_tmp_bytes(nkv + 1)) + 1024;
    tmp.ensure(al, tmp_bytes);

    set->d_desc.ensure(al, G * sizeof(GraphDesc));
    set->s_off.ensure(al, (NS + 1) * 8);
    set->o_off.ensure(al, (NO + 1) * 8);
    set->s_adj.ensure(al, std::max<uint64_t>(M, 1) * 4);
    set->o_adj.ensure(al, std::max<uint64_t>(M, 1) * 4);
    set->s_suf.ensure(al, std::max<uint64_t>(M, 1) * 8);
    DBuf o_ent;
    o_ent.ensure(al, std::max<uint64_t>(M, 1) * 4);
    set->s_graph.ensure(al, std::max<uint64_t>(NS, 1) * 4);
    set->s_vert.ensure(al, std::max<uint64_t>(NS, 1) * 4);
    HIP_OK(hipMemcpyAsync(set->d_desc.p, d_desc_tmp, G * sizeof(GraphDesc),
                          hipMemcpyDeviceToDevice, s));

    a.desc = d_desc_tmp; a.s_base_arr = d_sbase; a.o_base_arr = d_obase;
    a.NS = (uint32_t)NS; a.NO = (uint32_t)NO;
    a.max_deg_s = max_deg_s;
    a.rank_bits = bit_width((uint64_t)G * (max_deg_s + 1ull) - 1);
    // S lists are sorted by rank only (order within a list does not matter);
    // the stable sort by O index that follows puts every O list in rank order
    a.s_bits = NS > 1 ? bit_width(NS - 1) : 0;
    a.o_bits = NO > 1 ? bit_width(NO - 1) : 0;
    a.key0 = key0.as<uint64_t>(); a.key1 = key1.as<uint64_t>();
    a.val0 = val0.as<uint32_t>(); a.val1 = val1.as<uint32_t>();
    a.deg_o = deg_o.as<uint32_t>(); a.deg_rank = deg_rank.as<uint32_t>();
    a.rank_of = rank_of.as<uint32_t>();
    a.s_off = set->s_off.as<uint64_t>(); a.o_off = set->o_off.as<uint64_t>();
    a.s_adj = set->s_adj.as<uint32_t>(); a.o_adj = set->o_adj.as<uint32_t>();
    a.s_suf = set->s_suf.as<uint2>(); a.o_ent = o_ent.as<uint32_t>();
    a.s_graph = set->s_graph.as<uint32_t>(); a.s_vert = set->s_vert.as<uint32_t>();
    a.tmp = tmp.p; a.tmp_bytes = tmp_bytes;
    HIP_OK(build_rank(a, s));
    HIP_OK(build_adjacency(a, s));
    if (timed) HIP_OK(hipEventRecord(ctx->ev[5], s));
    HIP_OK(hipMemcpyAsync(h_flags, d_flags, 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (timed) HIP_OK(hipEventElapsedTime(&ctx->stats.ms_build, ctx->ev[4], ctx->ev[5]));
    if (h_flags[0] & kErrDup) fail(BBC_E_DUP_EDGE, "an edge (u, v) appears more than once");
    return set;
}

// -------------------------------------------------------------- counting
struct CountReq {
    const GraphSet *set;
    uint32_t g0, g1;        // graph range
    int mode;               // 0 totals, 1 per vertex of S, 2 per vertex of O, 3 totals for q > 3
    uint32_t q;             // mode 3: vertices taken on the opposite side
    // anchors of global rank [alo, ahi) only (alo < ahi; else the whole range
    // of graphs g0 .. g1 - 1): every count of the method is a sum over its
    // anchors, so the counts of a partition of the anchors add up to the
    // graph's count
    uint32_t alo = 0, ahi = 0;
    bool preload = true;    // the accumulator preload of the test hook applies
};

uint64_t hint_key(const GraphSet &set)
{
    const uint64_t side = set.G == 1 ? set.desc[0].side : 2;
    return ((uint64_t)bit_width(set.NS) << 40) | ((uint64_t)bit_width(set.NO) << 32) |
           ((uint64_t)bit_width(set.M) << 24) | ((uint64_t)std::min(set.G, 0xffffu) << 2) | side;
}

// The first workspace guess of a single graph from its oriented wedges W2
// (ensure_work): mask words, candidates and units.
uint64_t work_bytes_from_wedges(uint64_t w2)
{
    return 4 * (w2 / 20 * 9 + w2 / 10) + sizeof(Unit) * (w2 / 40);
}

void ensure_work(bbc_ctx *ctx, Work &w, GraphSet &set)
{
    Allocator *al = w.arena ? w.arena : ctx->al.get();
    uint64_t M = std::max<uint64_t>(set.M, 1);
    uint64_t hint_masks, hint_cands, hint_units;
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        auto it = ctx->ws_hint.find(hint_key(set));
        if (it != ctx->ws_hint.end()) {
            set.hint_masks = std::max(set.hint_masks, it->second.masks);
            set.hint_cands = std::max(set.hint_cands, it->second.cands);
            set.hint_units = std::max(set.hint_units, it->second.units);
        }
        hint_masks = set.hint_masks; hint_cands = set.hint_cands; hint_units = set.hint_units;
    }
    // records are reserved 16 at a time per wave of the per-wave tier and per
    // workgroup of the others
    const uint64_t agents = (uint64_t)ctx->num_cus * (wave_tier_waves_per_cu() + 8) + 64;
    uint64_t want_anchors = std::max<uint64_t>(set.NS, 1) + 16ull * agents;
    // first guesses; an overflowing count records its exact demand and reruns once
    uint64_t want_masks = std::max<uint64_t>({hint_masks, 2 * M, 1ull << 22});
    uint64_t want_cands = std::max<uint64_t>({hint_cands, M / 2, 1ull << 20});
    uint64_t want_units = std::max<uint64_t>({hint_units, M / 16, 1ull << 16});
    if (set.G == 1 && hint_masks == 0 && set.wedges_o > 0) {
        // no count of this shape yet: the Chung-Lu workloads need 0.23 W2
        // (100k x 50k) to 0.42 W2 (2M x 500k, wider masks) mask words, under
        // 0.07 W2 candidates and under W2 / 60 units (W2 = the oriented
        // wedges); with some margin these are taken if they fit a quarter of
        // the free device memory and a third of the room left under the
        // context's cap
        const uint64_t W2 = set.wedges_o;
        const uint64_t gm = W2 / 20 * 9, gc = W2 / 10, gu = W2 / 40;
        const uint64_t bytes = work_bytes_from_wedges(W2);
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            fr = 0;
        }
        uint64_t room = fr / 4;
        if (al->cap()) room = std::min<uint64_t>(room, al->cap() > al->used() ? (al->cap() - al->used()) / 3 : 0);
        if (bytes <= room) {
            want_masks = std::max(want_masks, gm);
            want_cands = std::max(want_cands, gc);
            want_units = std::max(want_units, gu);
        }
    }
    // A capacity is cleared before its buffers are (re)allocated and set only
    // once all of them are: DBuf::ensure releases the old buffer first, so an
    // allocation that fails (BBC_E_NOMEM under the context's cap) must not
    // leave a capacity that a later count on this workspace would trust with
    // a null buffer.
    if (w.cap_anchors < want_anchors) {
        w.cap_anchors = 0;
        w.anchors.ensure(al, want_anchors * sizeof(AnchorRec));
        w.ucnt.ensure(al, 3 * want_anchors * 4);
        w.uoff.ensure(al, (3 * want_anchors + 1) * 8);
        w.ptmp_bytes = scan_tmp_bytes(3 * want_anchors + 1) + 256;
        w.ptmp.ensure(al, w.ptmp_bytes);
        w.cap_anchors = want_anchors;
    }
    // 64 words of slack past the capacity: scalar column loads of the last
    // mask may be issued for a full 16-word group
    if (w.cap_masks < want_masks) {
        w.cap_masks = 0;
        w.masks.ensure(al, (want_masks + 64) * 4);
        w.cap_masks = want_masks;
    }
    if (w.cap_cands < want_cands) {
        w.cap_cands = 0;
        w.cands.ensure(al, want_cands * 4);
        w.cap_cands = want_cands;
    }
    if (w.cap_units < want_units) {
        w.cap_units = 0;
        w.units.ensure(al, want_units * sizeof(Unit));
        w.cap_units = want_units;
    }
    if (w.cap_defer < set.NS + 1ull) {
        w.cap_defer = 0;
        w.defer0.ensure(al, (set.NS + 1ull) * 4); w.defer1.ensure(al, (set.NS + 1ull) * 4);
        w.defer2.ensure(al, (set.NS + 1ull) * 4); w.defer3.ensure(al, (set.NS + 1ull) * 4);
        w.defer4.ensure(al, (set.NS + 1ull) * 4);
        w.cap_defer = set.NS + 1ull;
    }
    w.ctr.ensure(al, sizeof(Counters));
    w.count.ensure(al, std::max<uint32_t>(set.G, 1) * 8);
    w.carry.ensure(al, std::max<uint32_t>(set.G, 1) * 4);
    w.host.ensure(sizeof(Counters) + 12ull * std::max<uint32_t>(set.G, 1) + 64);
    const uint32_t maxd = tier_c_max_degree(), kmax = tier_c_max_k();
    // tier B and the rank-window tier: per-block position lists in global
    // memory, sized for the set's largest degree
    const uint64_t bwords = 2ull * (std::min(set.max_deg, maxd) + 1ull);
    if (!w.bscr.p || w.bscr_blocks < (uint32_t)ctx->num_cus || w.bscr_words < bwords) {
        w.bscr_blocks = 0;
        w.bscr.ensure(al, bwords * 4 * ctx->num_cus);
        w.bscr_words = bwords;
        w.bscr_blocks = ctx->num_cus;
    }
    // tiers C and D: hash tables in global memory. C: up to 2^20 slots on
    // one block per CU; D: sized for the largest anchor side of any graph
    // (every partner fits), on a few blocks. At least 2^18 slots: the compact
    // table of up to 65535 candidate classes takes half of the region. Only
    // anchors whose partner window is wider than the rank-window tier's, or
    // anchors no tier supports, reach them: while every graph's anchor side
    // is narrower than that window they get one block each.
    uint32_t max_ns = 0;
    for (auto &d : set.desc) max_ns = std::max(max_ns, d.n_s);
    const bool wide = max_ns > window_tier_max_window() + 1u;
    uint32_t HD = 1u << 18;
    int lgd = 18;
    while (HD < 2ull * max_ns + 64 && lgd < 25) { HD <<= 1; lgd++; }
    const uint32_t HC = std::min(HD, 1u << 20);
    const int lgc = std::min(lgd, 20);
    const uint64_t cwords = (2ull * HC + 2ull * maxd + kmax + 64 + 3) & ~3ull;
    const uint32_t cblocks = wide ? (uint32_t)std::max<uint64_t>(
                                        1, std::min<uint64_t>(ctx->num_cus, (2ull << 30) / (cwords * 4)))
                                  : 1u;
    if (!w.gtab.p || w.gH < HC || w.gtab_blocks < cblocks) {
        // per-block regions start 16-byte aligned (the table is read 4 slots at a time)
        w.gtab_blocks = 0;
        w.gtab.ensure(al, cwords * 4 * cblocks);
        w.gH = HC; w.glog2 = lgc; w.gmaxd = maxd; w.gkmax = kmax;
        w.gtab_words = cwords; w.gtab_blocks = cblocks;
    }
    const uint64_t dwords = (2ull * HD + 2ull * maxd + kmax + 64 + 3) & ~3ull;
    const uint32_t dblocks = wide ? (uint32_t)std::max<uint64_t>(
                                        1, std::min<uint64_t>(16, (1ull << 30) / (dwords * 4)))
                                  : 1u;
    if (!w.dtab.p || w.dH < HD || w.dtab_blocks < dblocks) {
        w.dtab_blocks = 0;
        w.dtab.ensure(al, dwords * 4 * dblocks);
        w.dH = HD; w.dlog2 = lgd;
        w.dtab_words = dwords; w.dtab_blocks = dblocks;
    }
}

// Device bytes a count of a set of m edges and n_s anchor-side vertices
// (either side: the larger of the two is taken) may hold in its workspace on
// the first attempt: the first guesses of ensure_work, with the global-memory
// tiers at one block and tier B's lists for degrees up to max_deg.
uint64_t work_bytes_estimate(uint64_t m, uint64_t n_s, uint32_t max_deg, int num_cus)
{
    const uint64_t M = std::max<uint64_t>(m, 1);
    const uint64_t agents = (uint64_t)num_cus * (wave_tier_waves_per_cu() + 8) + 64;
    const uint64_t anchors = n_s + 16 * agents;
    uint64_t b = 0;
    b += anchors * (sizeof(AnchorRec) + 12 + 24) + scan_tmp_bytes(3 * anchors + 1);
    b += (std::max<uint64_t>(2 * M, 1ull << 22) + 64) * 4;                 // masks
    b += std::max<uint64_t>(M / 2, 1ull << 20) * 4;                        // candidates
    b += std::max<uint64_t>(M / 16, 1ull << 16) * sizeof(Unit);            // units
    b += 5 * (n_s + 1) * 4;                                                // tier lists
    b += 2ull * (std::min(max_deg, tier_c_max_degree()) + 1) * 4 * num_cus;  // tier B lists
    const uint64_t tier_words = 2ull * (1u << 18) + 3ull * 65536 + 64;
    b += 2 * tier_words * 4;                                               // tiers C, D
    return b + (4u << 20);
}

Workspace ws_view(Work &w, bool pv, bool pvo)
{
    Workspace ws;
    memset(&ws, 0, sizeof(ws));
    ws.ctr = w.ctr.as<Counters>();
    ws.anchors = w.anchors.as<AnchorRec>(); ws.cap_anchors = w.cap_anchors;
    ws.units = w.units.as<Unit>(); ws.cap_units = w.cap_units;
    ws.masks = w.masks.as<uint32_t>(); ws.cap_mask_words = w.cap_masks;
    ws.cands = w.cands.as<uint32_t>(); ws.cap_cands = w.cap_cands;
    ws.defer[0] = w.defer0.as<uint32_t>(); ws.defer[1] = w.defer1.as<uint32_t>();
    ws.defer[2] = w.defer2.as<uint32_t>(); ws.defer[3] = w.defer3.as<uint32_t>();
    ws.defer[4] = w.defer4.as<uint32_t>();
    ws.cap_defer = w.cap_defer;
    ws.gtab = w.gtab.as<uint32_t>(); ws.gtab_words_per_block = w.gtab_words;
    ws.gtab_blocks = w.gtab_blocks;
    ws.dtab = w.dtab.as<uint32_t>(); ws.dtab_words_per_block = w.dtab_words;
    ws.dtab_blocks = w.dtab_blocks;
    ws.bscr = w.bscr.as<uint32_t>(); ws.bscr_words_per_block = w.bscr_words;
    ws.ucnt = w.ucnt.as<uint32_t>(); ws.uoff = w.uoff.as<uint64_t>();
    ws.count = w.count.as<unsigned long long>();
    ws.carry = w.carry.as<uint32_t>();
    ws.pv = pv ? w.pv.as<unsigned long long>() : nullptr;
    ws.pv_slot = pv ? w.pv_slot.as<unsigned long long>() : nullptr;
    ws.pv_o = pvo ? w.pv_o.as<unsigned long long>() : nullptr;
    return ws;
}

// Enqueue one full count (zeroing, pair tiers, triplets) on stream s.
// Nothing here reads back, so the sequence can be captured.
// Every value the count sequence passes to a kernel. A captured replay is
// valid only while this is byte-for-byte the same.
struct LaunchArgs {
    PairArgs P;
    LaunchShape ls;
    TriArgs T;
    int mode;
    uint32_t G, NS, NO;
    void *ptmp;
    uint64_t ptmp_bytes;
    uint64_t preload;       // starting value of every graph's accumulator (0 but in tests)
};

// Output chunks of the pair kernels: each workgroup (each wave of the
// per-wave tier) reserves mask words and candidates a chunk at a time and
// abandons a chunk's tail when the next anchor does not fit, so the demand of
// a count is at least one chunk per agent that took an anchor. Chunks scale
// with the edges of the counted graphs (about 2 mask words per edge over all
// agents), between a floor that keeps reservations rare and the sizes that
// the largest graphs use.
struct Chunks { uint32_t mask, cand, wv_mask, wv_cand; };

uint32_t pow2_clamp(uint64_t x, uint32_t lo, uint32_t hi)
{
    uint32_t c = lo;
    while (c < hi && 2ull * c <= x) c <<= 1;
    return c;
}

Chunks chunk_sizes(const bbc_ctx *ctx, const GraphSet &set, uint32_t g0, uint32_t g1)
{
    uint64_t m = 0;
    for (uint32_t g = g0; g < g1; g++) m += set.desc[g].m;
    const uint64_t wg_agents = (uint64_t)ctx->num_cus * 4;
    const uint64_t waves = (uint64_t)ctx->num_cus * wave_tier_waves_per_cu();
    Chunks c;
    c.mask = pow2_clamp(2 * m / wg_agents, 2048, 1u << 16);
    c.cand = pow2_clamp(m / 4 / wg_agents, 256, 1u << 13);
    c.wv_mask = pow2_clamp(2 * m / waves, 256, 4096);
    c.wv_cand = c.wv_mask;
    return c;
}

LaunchArgs make_args(bbc_ctx *ctx, Work &w, const CountReq &r, const Shape &shp)
{
    const GraphSet &set = *r.set;
    LaunchArgs L;
    memset(&L, 0, sizeof(L));
    const bool pv = r.mode == 1, pvo = r.mode == 2;
    Workspace ws = ws_view(w, pv, pvo);
    L.P.g = set.view();
    L.P.ws = ws;
    L.P.a0 = set.desc[r.g0].s_base;
    L.P.a1 = set.desc[r.g1 - 1].s_base + set.desc[r.g1 - 1].n_s;
    if (r.alo < r.ahi) { L.P.a0 = r.alo; L.P.a1 = r.ahi; }
    // per-vertex counts keep one LDS sum per unit column: their units stay narrower
    L.P.chunk_base = std::min(shp.chunk_base, r.mode == 1 ? max_unit_chunk() : 16384u);
    // The totals of one graph with 2^32 or more oriented wedges take units twice
    // as long unless the caller forced a shape: with anchors of thousands of
    // candidates, the longer units spread each row once for more columns
    // (the 40M-edge Chung-Lu graph, 1.5e10 wedges: triplets 508 -> 504 ms;
    // the 2M-edge one, 3.3e8 wedges, measured 6% slower in its triplet phase
    // and keeps the default).
    if (r.mode == 0 && !ctx->hook_shape_set && set.G == 1 && shp.chunk_base == Shape().chunk_base &&
        set.wedges_o >= (1ull << 32))
        L.P.chunk_base = 2 * shp.chunk_base;
    L.P.gH = w.gH; L.P.glog2h = w.glog2; L.P.gmaxd = w.gmaxd; L.P.gkmax = w.gkmax;
    L.P.dH = w.dH; L.P.dlog2h = w.dlog2;
    L.ls.grid_w = std::max(1u, ctx->num_cus * wave_tier_blocks_per_cu());
    L.ls.grid_a = std::max(1u, ctx->num_cus * shp.grid_a_per_cu);
    L.ls.grid_b = std::max(1u, (uint32_t)ctx->num_cus);
    L.ls.grid_c = w.gtab_blocks;
    L.ls.grid_d = w.dtab_blocks;
    L.ls.grid_t = std::max(1u, ctx->num_cus * shp.grid_t_per_cu);
    L.T.g = L.P.g;
    L.T.ws = ws;
    L.T.q = r.mode >= 3 ? r.q : 3u;
    L.mode = r.mode;
    L.G = set.G; L.NS = set.NS; L.NO = set.NO;
    L.ptmp = w.ptmp.p;
    L.ptmp_bytes = w.ptmp_bytes;
    L.P.flags = ctx->hook_no_window ? kPairNoWindow : 0u;
    const Chunks ch = chunk_sizes(ctx, set, r.g0, r.g1);
    L.P.mask_chunk = ch.mask; L.P.cand_chunk = ch.cand;
    L.P.wv_mask_chunk = ch.wv_mask; L.P.wv_cand_chunk = ch.wv_cand;
    w.mask_chunk = ch.mask; w.cand_chunk = ch.cand;
    w.wv_mask_chunk = ch.wv_mask; w.wv_cand_chunk = ch.wv_cand;
    L.preload = r.preload ? ctx->hook_preload : 0;
    return L;
}

void enqueue_args(bbc_ctx *ctx, const LaunchArgs &L, hipStream_t s, bool timed)
{
    const Workspace &ws = L.P.ws;
    HIP_OK(fill_u32((uint32_t *)ws.ctr, 0, sizeof(Counters) / 4, s));
    HIP_OK(fill_u64(ws.count, L.preload, L.G, s));
    HIP_OK(fill_u32(ws.carry, 0, L.G, s));
    if (L.mode == 1) HIP_OK(fill_u64(ws.pv, 0, L.NS, s));
    if (L.mode == 2) HIP_OK(fill_u64(ws.pv_o, 0, L.NO, s));
    if (timed) HIP_OK(hipEventRecord(ctx->ev[0], s));
    HIP_OK(count_pairs(L.P, L.ls, s));
    if (timed) HIP_OK(hipEventRecord(ctx->ev[1], s));
    HIP_OK(count_plan(ws, L.P.chunk_base, L.ptmp, L.ptmp_bytes, L.mode >= 4 ? (uint32_t)L.mode : 3u, s));
    if (timed) HIP_OK(hipEventRecord(ctx->ev[2], s));
    HIP_OK(count_triplets(L.T, L.mode, L.ls.grid_t, s));
    if (timed) HIP_OK(hipEventRecord(ctx->ev[3], s));
}

// Enqueue one full count (zeroing, pair tiers, planning, triplets) on
// stream s. Nothing here reads back, so the sequence can be captured.
void enqueue_count(bbc_ctx *ctx, Work &w, const CountReq &r, const Shape &shp, hipStream_t s,
                   bool timed = false)
{
    enqueue_args(ctx, make_args(ctx, w, r, shp), s, timed);
}

void enqueue_readback(Work &w, const GraphSet &set, hipStream_t s)
{
    char *hp = w.host.as<char>();
    HIP_OK(hipMemcpyAsync(hp, w.ctr.p, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(hp + sizeof(Counters), w.count.p, 8ull * set.G, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(hp + sizeof(Counters) + 8ull * set.G, w.carry.p, 4ull * set.G,
                          hipMemcpyDeviceToHost, s));
}

// After a readback: true if the count is complete, false if buffers must grow.
bool check_counters(bbc_ctx *ctx, Work &w, GraphSet &set)
{
    const Counters *c = w.host.as<Counters>();
    if (c->over_cap & 8u) fail(BBC_E_HIP, "internal error: pair table lookup failed");
    if (c->over_cap & 16u) fail(BBC_E_OVERFLOW, "a term C(n, q) of the count needs more than 64 bits");
    if (c->over_cap & 32u)
        fail(BBC_E_UNSUPPORTED, "the count needs more than 2^32 - 1 triplet work units (too many "
                                "candidate subsets for this graph)");
    if (c->over_cap & 4u)
        fail(BBC_E_UNSUPPORTED, "an anchor has degree above %u or more than %u candidate classes",
             tier_c_max_degree(), tier_c_max_k());
    // demand plus room for the reservation chunks of the per-wave tier (4096
    // words) and of the workgroup tiers. A set may be counted by several
    // threads at once (serving workers and the caller): its hints are updated
    // under the tuning lock.
    // The slack covers chunks that other workgroups may hold next time; it
    // is at most the demand itself, so that a small set's hint stays small.
    const uint64_t wv = (uint64_t)ctx->num_cus * wave_tier_waves_per_cu();
    const uint64_t slack_m =
        std::min<uint64_t>(4ull * ctx->num_cus * w.mask_chunk + wv * w.wv_mask_chunk,
                           std::max<uint64_t>(c->need_masks, 1u << 16));
    const uint64_t slack_c =
        std::min<uint64_t>(4ull * ctx->num_cus * w.cand_chunk + wv * w.wv_cand_chunk,
                           std::max<uint64_t>(c->need_cands, 1u << 13));
    const bool grow = (c->over_cap & 3u) != 0;
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        set.hint_masks = std::max<uint64_t>(set.hint_masks, c->need_masks + c->need_masks / 16 + slack_m);
        set.hint_cands = std::max<uint64_t>(set.hint_cands, c->need_cands + c->need_cands / 16 + slack_c);
        if (grow) {
            set.hint_units = std::max<uint64_t>(set.hint_units, c->need_units + c->need_units / 16 + 1024);
        } else {
            set.hint_units = std::max<uint64_t>(set.hint_units, (uint64_t)c->n_units + c->n_units / 8);
            if (!w.arena) {   // (a no-allocation count keeps its hints in the set only)
                auto &h = ctx->ws_hint[hint_key(set)];
                h.masks = std::max(h.masks, set.hint_masks);
                h.cands = std::max(h.cands, set.hint_cands);
                h.units = std::max(h.units, set.hint_units);
            }
        }
    }
    if (grow) return false;
    // the statistics describe the last count on the context's own workspace
    if (&w != &ctx->work) return true;
    ctx->stats.active_anchors = c->n_anchor;
    ctx->stats.virtual_candidates = c->cand_cursor;
    ctx->stats.pair_units = c->n_units;
    ctx->stats.candidate_pairs = c->pairs_examined;
    ctx->stats.mask_words = c->mask_cursor;
    ctx->stats.wedges = c->wedges;
    ctx->stats.pair_words = c->pair_words;
    ctx->stats.deferred_a = c->n_list[0];
    ctx->stats.deferred_b = c->n_list[1];
    ctx->stats.deferred_c = c->n_list[2];
    ctx->stats.deferred_d = c->n_list[3];
    ctx->stats.deferred_r = c->n_list[4];
    return true;
}

void results_from_host(Work &w, const GraphSet &set, uint32_t g0, uint32_t g1, int64_t *out)
{
    const char *hp = w.host.as<char>();
    const uint64_t *cnt = (const uint64_t *)(hp + sizeof(Counters));
    const uint32_t *car = (const uint32_t *)(hp + sizeof(Counters) + 8ull * set.G);
    for (uint32_t g = g0; g < g1; g++) {
        if (car[g] || cnt[g] > (uint64_t)INT64_MAX)
            fail(BBC_E_OVERFLOW, "graph %u: count does not fit in int64", g);
        out[g - g0] = (int64_t)cnt[g];
    }
}

// The fixed launch shape of single-graph counts (a test hook may force another)
Shape default_shape(const bbc_ctx *ctx) { return ctx->hook_shape_set ? ctx->hook_shape : Shape(); }

// One synchronous count of a graph range; grows buffers and retries as needed.
void count_sync(bbc_ctx *ctx, Work &w, GraphSet &set, uint32_t g0, uint32_t g1, int mode,
                const Shape &shp, hipStream_t s, int64_t *out, uint32_t q = 3, uint32_t alo = 0,
                uint32_t ahi = 0, bool preload = true)
{
    CountReq r{&set, g0, g1, mode, q, alo, ahi, preload};
    const bool timed = ctx->timing && s == ctx->stream && &w == &ctx->work;
    const bool tune = set.tune_key && mode == 0 && s == ctx->stream && &w == &ctx->work;
    if (tune && !ctx->tev[0]) {
        HIP_OK(hipEventCreate(&ctx->tev[0]));
        HIP_OK(hipEventCreate(&ctx->tev[1]));
    }
    for (int attempt = 0; attempt < 8; attempt++) {
        if (w.arena) {
            // an arena cannot free: every attempt carves its buffers afresh
            w.release_device();
            w.arena->arena_reset();
        }
        ensure_work(ctx, w, set);
        if (mode == 1) {
            w.pv.ensure(ctx->al.get(), std::max<uint64_t>(set.NS, 1) * 8);
            w.pv_slot.ensure(ctx->al.get(), std::max<uint64_t>(w.cap_cands, 1) * 8);
        }
        if (mode == 2) w.pv_o.ensure(ctx->al.get(), std::max<uint64_t>(set.NO, 1) * 8);
        if (tune) HIP_OK(hipEventRecord(ctx->tev[0], s));
        enqueue_count(ctx, w, r, shp, s, timed);
        if (tune) HIP_OK(hipEventRecord(ctx->tev[1], s));
        enqueue_readback(w, set, s);
        HIP_OK(hipStreamSynchronize(s));
        if (check_counters(ctx, w, set)) {
            if (tune) {
                float ms = 0;
                HIP_OK(hipEventElapsedTime(&ms, ctx->tev[0], ctx->tev[1]));
                std::lock_guard<std::mutex> lk(ctx->tune_mu);
                auto &st = ctx->side_tune[set.tune_key];
                const uint32_t sd = set.tune_side;
                st.ms[sd] = st.tried[sd] ? std::min(st.ms[sd], ms) : ms;
                st.tried[sd] = true;
            }
            if (&w == &ctx->work) ctx->stats.attempts = attempt + 1;
            if (timed) {
                HIP_OK(hipEventElapsedTime(&ctx->stats.ms_pair, ctx->ev[0], ctx->ev[1]));
                HIP_OK(hipEventElapsedTime(&ctx->stats.ms_plan, ctx->ev[1], ctx->ev[2]));
                HIP_OK(hipEventElapsedTime(&ctx->stats.ms_triplet, ctx->ev[2], ctx->ev[3]));
            }
            results_from_host(w, set, g0, g1, out);
            return;
        }
    }
    fail(BBC_E_NOMEM, "count workspace kept overflowing");
}

uint64_t size_class(const GraphSet &set)
{
    return ((uint64_t)bit_width(set.NS) << 16) | ((uint64_t)bit_width(set.M) << 8) |
           (uint64_t)std::min(set.G, 255u);
}

// Autotuner: time a few launch shapes on this graph set and keep the best
// per size class.
Shape tune_shape(bbc_ctx *ctx, Work &w, GraphSet &set, hipStream_t s)
{
    if (ctx->hook_shape_set) return ctx->hook_shape;
    const uint64_t key = size_class(set);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) return it->second;
    std::vector<Shape> cands;
    for (uint32_t cb : {512u, 2048u, 4096u})
        for (uint32_t gt : {4u, 8u}) {
            Shape sh;
            sh.chunk_base = cb;
            sh.grid_t_per_cu = gt;
            cands.push_back(sh);
        }
    std::vector<int64_t> tmp(set.G);
    count_sync(ctx, w, set, 0, set.G, 0, cands[0], s, tmp.data());   // sizes the workspace
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    Shape best = cands[0];
    float best_ms = 1e30f;
    for (const Shape &sh : cands) {
        CountReq r{&set, 0, set.G, 0};
        HIP_OK(hipEventRecord(e0, s));
        enqueue_count(ctx, w, r, sh, s);
        HIP_OK(hipEventRecord(e1, s));
        HIP_OK(hipEventSynchronize(e1));
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) { best_ms = ms; best = sh; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->tuned[key] = best;
    return best;
}

// Batched count of a whole graph set: the launch sequence is captured once
// into a HIP graph and replayed.
void count_set_batched(bbc_ctx *ctx, Work &w, GraphSet &set, hipStream_t s, int64_t *out)
{
    Shape shp = tune_shape(ctx, w, set, s);
    CountReq r{&set, 0, set.G, 0};
    for (int attempt = 0; attempt < 4; attempt++) {
        ensure_work(ctx, w, set);
        const LaunchArgs L = make_args(ctx, w, r, shp);
        const unsigned char *lb = (const unsigned char *)&L;
        const bool same = w.exec && w.exec_args.size() == sizeof(L) &&
                          memcmp(w.exec_args.data(), lb, sizeof(L)) == 0;
        if (!same) {
            if (w.exec) { (void)hipGraphExecDestroy(w.exec); w.exec = nullptr; }
            w.exec_args.clear();
            hipGraph_t graph = nullptr;
            HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                enqueue_args(ctx, L, s, false);
            } catch (...) {
                hipGraph_t junk = nullptr;
                (void)hipStreamEndCapture(s, &junk);
                if (junk) (void)hipGraphDestroy(junk);
                throw;
            }
            HIP_OK(hipStreamEndCapture(s, &graph));
            hipError_t e = hipGraphInstantiate(&w.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIP_OK(e);
            w.exec_args.assign(lb, lb + sizeof(L));
        }
        HIP_OK(hipGraphLaunch(w.exec, s));
        enqueue_readback(w, set, s);
        HIP_OK(hipStreamSynchronize(s));
        if (check_counters(ctx, w, set)) {
            results_from_host(w, set, 0, set.G, out);
            return;
        }
    }
    fail(BBC_E_NOMEM, "batched count workspace kept overflowing");
}

// ---------------------------------------------------------------- serving
constexpr int kServeStreams = 4;
constexpr size_t kServeBatchMax = 4096;
constexpr uint64_t kServeBatchEdges = 8ull << 20;    // bounds one batch (and the wait of its small requests)
// A request of kServeLargeEdges edges or more is a batch of its own, at most
// kServeLargeWorkers workers hold one at a time (small requests behind it may
// go first), and its count runs in anchor ranges of about kServeChunkEdges
// edges, one synchronous count each, so that the other workers' batches get
// the GPU between them instead of waiting for the whole count.
constexpr uint64_t kServeLargeEdges = 1ull << 20;
constexpr int kServeLargeWorkers = 2;
constexpr uint64_t kServeChunkEdges = 512ull << 10;
constexpr uint32_t kServeMaxChunks = 16;
// Before its build and each of its ranges, a large request waits for the
// batches of small requests on the GPU to finish, up to this long in all per
// request: those batches then run without sharing the GPU with a large count.
constexpr int kServeYieldUs = 2000;

// memcpy split over up to 4 threads for large copies
void copy_par(void *dst, const void *src, uint64_t bytes)
{
    constexpr uint64_t kMin = 4ull << 20;
    const uint32_t nt = bytes >= kMin ? 4u : 1u;
    if (nt == 1) { memcpy(dst, src, bytes); return; }
    auto part = [&](uint32_t t) {
        const uint64_t b0 = bytes * t / nt, b1 = bytes * (t + 1) / nt;
        memcpy((char *)dst + b0, (const char *)src + b0, b1 - b0);
    };
    std::vector<std::thread> th;
    for (uint32_t t = 1; t < nt; t++) th.emplace_back(part, t);
    part(0);
    for (auto &x : th) x.join();
}

// Device bytes the build of a COO request of m edges and n vertices may hold
// at its peak: the uploaded COO, the sort buffers and the CSR it produces
// (the workspace of its count is reserved separately).
uint64_t build_bytes_estimate(uint64_t m, uint64_t n)
{
    const uint64_t M = std::max<uint64_t>(m, 1), nkv = std::max<uint64_t>(M, n);
    return 40 * M + 24 * nkv + 128 * n + radix_tmp_bytes(nkv) + (2u << 20);
}

// What a batch of requests reserves under the context's cap: the builds of
// its COO requests and one count workspace sized for all of them together.
struct Reservation {
    uint64_t build = 0, m = 0, n_s = 0, w2 = 0, n = 0;
    uint32_t max_deg = 0;
    void add(const Request &r)
    {
        if (!r.set) build += build_bytes_estimate(r.m, (uint64_t)r.n_u + r.n_v);
        m = r.set ? std::max(m, r.m) : m + r.m;
        n_s = r.set ? std::max<uint64_t>(n_s, r.n_s_max) : n_s + r.n_s_max;
        max_deg = std::max(max_deg, r.max_deg);
        w2 = std::max(w2, r.w2_max);
        n++;
    }
    uint64_t bytes(int num_cus) const
    {
        uint64_t b = build + work_bytes_estimate(m, n_s, max_deg, num_cus);
        // a graph counted alone starts from its wedge count (ensure_work)
        if (n == 1) b += work_bytes_from_wedges(w2);
        // allocations of 1 MB and more are rounded up to 2 MB
        return b + b / 4 + (8u << 20);
    }
};

// Device bytes a serving worker may keep between batches: a sixteenth of the
// cap (four workers keep at most a quarter of it), 1 GiB without a cap.
uint64_t serve_keep_bytes(const bbc_ctx *ctx)
{
    const uint64_t cap = ctx->al->cap();
    return cap ? cap / 16 : (1ull << 30);
}

// Marks a batch of small requests as building or counting on the GPU for
// its lifetime (large requests wait for such batches at their range
// boundaries).
struct SmallOnGpu {
    bbc_ctx *ctx;
    explicit SmallOnGpu(bbc_ctx *c) : ctx(c)
    {
        std::lock_guard<std::mutex> lk(ctx->q_mu);
        ctx->serve_small_gpu++;
    }
    ~SmallOnGpu()
    {
        {
            std::lock_guard<std::mutex> lk(ctx->q_mu);
            ctx->serve_small_gpu--;
        }
        ctx->small_cv.notify_all();
    }
};

void serve_worker(bbc_ctx *ctx, int slot)
{
    hipStream_t s = ctx->serve_streams[slot];
    Work w;
    tl_alloc_tag = 1;
    (void)hipSetDevice(ctx->device);
    auto finish = [&](const std::shared_ptr<Request> &r, bbc_status st, int64_t v) {
        std::lock_guard<std::mutex> lk(ctx->q_mu);
        r->status = st;
        r->result = v;
        r->done = true;
        r->eu.clear(); r->eu.shrink_to_fit();
        r->ev.clear(); r->ev.shrink_to_fit();
        r->sign.clear(); r->sign.shrink_to_fit();
    };
    int64_t yield_left_us = 0;   // what the large request in hand may still wait
    auto yield_to_small = [&] {
        if (yield_left_us <= 0) return;
        const auto t0 = std::chrono::steady_clock::now();
        std::unique_lock<std::mutex> lk(ctx->q_mu);
        ctx->small_cv.wait_for(lk, std::chrono::microseconds(yield_left_us),
                               [&] { return ctx->serve_small_gpu == 0 || ctx->stopping; });
        yield_left_us -= std::chrono::duration_cast<std::chrono::microseconds>(
                             std::chrono::steady_clock::now() - t0).count();
    };
    // the count of graph gi of a set (m edges) as the sum of the counts of
    // anchor ranges of equal size; the test hook's preload goes to the first
    auto count_chunked = [&](GraphSet &set, uint32_t gi, uint64_t m, int64_t *out) {
        const GraphDesc &d = set.desc[gi];
        const uint32_t n = (uint32_t)std::min<uint64_t>(
            kServeMaxChunks, std::max<uint64_t>(1, std::min<uint64_t>(m / kServeChunkEdges, d.n_s)));
        uint64_t tot = 0;
        for (uint32_t c = 0; c < n; c++) {
            const uint32_t lo = d.s_base + (uint32_t)((uint64_t)d.n_s * c / n);
            const uint32_t hi = d.s_base + (uint32_t)((uint64_t)d.n_s * (c + 1) / n);
            int64_t v = 0;
            if (lo < hi) {
                yield_to_small();
                count_sync(ctx, w, set, gi, gi + 1, 0, default_shape(ctx), s, &v, 3, lo, hi, c == 0);
            }
            tot += (uint64_t)v;
            if (tot > (uint64_t)INT64_MAX) fail(BBC_E_OVERFLOW, "count does not fit in int64");
        }
        *out = (int64_t)tot;
    };
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        uint64_t batch_bytes = 0;
        bool large = false;
        std::vector<std::shared_ptr<Request>> too_big;
        {
            std::unique_lock<std::mutex> lk(ctx->q_mu);
            ctx->q_cv.wait(lk, [&] { return ctx->stopping || !ctx->queue.empty(); });
            if (ctx->stopping && ctx->queue.empty()) return;
            // admission in arrival order while the batch's reservation fits
            // under the cap next to the memory the caller holds (tag 0) and
            // the reservations of the batches in flight
            // every worker may keep a workspace of up to keep bytes between
            // batches: that allowance is set aside from the cap
            const uint64_t cap = ctx->al->cap() ? ctx->al->cap() - kServeStreams * serve_keep_bytes(ctx)
                                                : 0;
            const uint64_t held = cap ? ctx->al->live(0) : 0;
            Reservation res;
            uint64_t batch_edges = 0;
            for (size_t qi = 0; qi < ctx->queue.size() && batch.size() < kServeBatchMax;) {
                const std::shared_ptr<Request> r = ctx->queue[qi];
                Reservation alone;
                alone.add(*r);
                if (cap && held + alone.bytes(ctx->num_cus) > cap) {
                    // can never fit while the caller holds what it holds
                    too_big.push_back(r);
                    ctx->queue.erase(ctx->queue.begin() + qi);
                    continue;
                }
                if (r->m >= kServeLargeEdges) {
                    // a batch of its own; with kServeLargeWorkers large
                    // requests in flight, the small ones behind it go first
                    if (!batch.empty() || ctx->serve_large >= kServeLargeWorkers) {
                        qi++;
                        continue;
                    }
                    const uint64_t want = alone.bytes(ctx->num_cus);
                    if (cap && held + ctx->admitted_bytes + want > cap) break;
                    batch_bytes = want;
                    batch.push_back(r);
                    ctx->queue.erase(ctx->queue.begin() + qi);
                    large = true;
                    break;
                }
                Reservation next = res;
                next.add(*r);
                const uint64_t want = next.bytes(ctx->num_cus);
                if (cap && held + ctx->admitted_bytes + want > cap) break;
                if (!batch.empty() && batch_edges + r->m > kServeBatchEdges) break;
                batch_edges += r->m;
                res = next;
                batch_bytes = want;
                batch.push_back(r);
                ctx->queue.erase(ctx->queue.begin() + qi);
            }
            if (large) ctx->serve_large++;
            yield_left_us = large ? kServeYieldUs : 0;
            ctx->admitted_bytes += batch_bytes;
            ctx->peak_admitted = std::max(ctx->peak_admitted, ctx->admitted_bytes);
            if (batch.empty() && too_big.empty()) {
                // wait until another worker releases its reservation
                ctx->q_cv.wait_for(lk, std::chrono::milliseconds(1));
                continue;
            }
        }
        for (auto &r : too_big) {
            set_error(ctx, "a served request needs more device memory than the cap leaves");
            finish(r, BBC_E_NOMEM, 0);
        }
        if (!too_big.empty()) ctx->done_cv.notify_all();
        if (batch.empty()) continue;
        // COO requests of the batch are built together; prebuilt graphs are
        // counted through their own sets
        std::vector<std::shared_ptr<Request>> coo, pre, requeue;
        for (auto &r : batch) (r->set ? pre : coo).push_back(r);
        // out of memory while other batches hold reservations: the requests
        // go back to the front of the queue (at most a few times each)
        auto others_in_flight = [&] {
            std::lock_guard<std::mutex> lk(ctx->q_mu);
            return ctx->admitted_bytes > batch_bytes;
        };
        // results are published after the batch has released its memory and
        // its reservation, so a caller that has every result sees the memory
        // free again
        struct Outcome { std::shared_ptr<Request> r; bbc_status st; int64_t v; };
        std::vector<Outcome> outcomes;
        auto settle = [&](const std::shared_ptr<Request> &r, bbc_status st, int64_t v) {
            if (st == BBC_E_NOMEM && r->nomem_retries < 8 && others_in_flight()) {
                r->nomem_retries++;
                requeue.push_back(r);
            } else {
                outcomes.push_back({r, st, v});
            }
        };
        if (!coo.empty()) {
            // group by sign encoding / anchor flags
            std::map<uint32_t, std::vector<std::shared_ptr<Request>>> by_flags;
            for (auto &r : coo) by_flags[r->flags].push_back(r);
            for (auto &kv : by_flags) {
                auto &rs = kv.second;
                const uint32_t flags = kv.first;
                std::vector<uint32_t> nu(rs.size()), nv(rs.size());
                std::vector<uint64_t> off(rs.size() + 1, 0);
                for (size_t i = 0; i < rs.size(); i++) {
                    nu[i] = rs[i]->n_u; nv[i] = rs[i]->n_v;
                    off[i + 1] = off[i] + rs[i]->m;
                }
                const uint64_t M = off.back();
                const uint64_t sbytes = sign_bytes(M, flags);
                // concatenate into pinned memory: the uploads are then true DMA copies
                w.coo.ensure(8 * std::max<uint64_t>(M, 1) + sbytes + 64);
                uint32_t *eu = w.coo.as<uint32_t>();
                uint32_t *ev = eu + M;
                uint8_t *sg = (uint8_t *)(ev + M);
                memset(sg, 0, sbytes);
                bool packed = flags & BBC_SIGNS_2BIT_PACKED;
                for (size_t i = 0; i < rs.size(); i++) {
                    copy_par(eu + off[i], rs[i]->eu.data(), rs[i]->m * 4);
                    copy_par(ev + off[i], rs[i]->ev.data(), rs[i]->m * 4);
                    if (!packed) {
                        copy_par(sg + off[i], rs[i]->sign.data(), rs[i]->m);
                    } else {
                        for (uint64_t e = 0; e < rs[i]->m; e++) {
                            uint32_t code = (rs[i]->sign[e >> 2] >> (2 * (e & 3))) & 3u;
                            uint64_t t = off[i] + e;
                            sg[t >> 2] |= (uint8_t)(code << (2 * (t & 3)));
                        }
                    }
                }
                CooIn in{(uint32_t)rs.size(), nu.data(), nv.data(), off.data(), eu, ev,
                         sg, flags & ~BBC_IN_DEVICE_PTRS};
                std::vector<int64_t> res(rs.size());
                bbc_status st = guard(nullptr, [&] {
                    if (large) {
                        yield_to_small();
                        auto set = build_set(ctx, in, s, w.bhost);
                        count_chunked(*set, 0, rs[0]->m, res.data());
                    } else {
                        SmallOnGpu on(ctx);
                        auto set = build_set(ctx, in, s, w.bhost);
                        count_sync(ctx, w, *set, 0, set->G, 0, default_shape(ctx), s, res.data());
                    }
                });
                if (st == BBC_E_NOMEM && others_in_flight()) {
                    for (auto &r : rs) settle(r, st, 0);
                } else if (st != BBC_OK && rs.size() > 1) {
                    // isolate the failing request: count each alone
                    for (size_t i = 0; i < rs.size(); i++) {
                        uint64_t o2[2] = {0, rs[i]->m};
                        CooIn one{1, &nu[i], &nv[i], o2, rs[i]->eu.data(), rs[i]->ev.data(),
                                  rs[i]->sign.data(), flags & ~BBC_IN_DEVICE_PTRS};
                        int64_t v = 0;
                        bbc_status st1 = guard(nullptr, [&] {
                            auto set = build_set(ctx, one, s, w.bhost);
                            count_sync(ctx, w, *set, 0, 1, 0, default_shape(ctx), s, &v);
                        });
                        settle(rs[i], st1, v);
                    }
                } else {
                    for (size_t i = 0; i < rs.size(); i++) settle(rs[i], st, res[i]);
                }
            }
        }
        for (auto &r : pre) {
            int64_t v = 0;
            bbc_status st = guard(nullptr, [&] {
                if (large) {
                    count_chunked(*r->set, r->idx, r->m, &v);
                } else {
                    SmallOnGpu on(ctx);
                    count_sync(ctx, w, *r->set, r->idx, r->idx + 1, 0, default_shape(ctx), s, &v);
                }
            });
            settle(r, st, v);
        }
        // a workspace larger than the kept allowance goes back to the
        // allocator; a smaller one stays for the next batch (reallocating it
        // for every batch costs more than the counts of small graphs)
        if (w.device_bytes() > serve_keep_bytes(ctx)) w.release_device();
        {
            std::lock_guard<std::mutex> lk(ctx->q_mu);
            ctx->admitted_bytes -= batch_bytes;
            if (large) ctx->serve_large--;
            for (auto it = requeue.rbegin(); it != requeue.rend(); ++it) ctx->queue.push_front(*it);
        }
        for (auto &o : outcomes) finish(o.r, o.st, o.v);
        ctx->done_cv.notify_all();
        ctx->q_cv.notify_all();
    }
}

void start_serving(bbc_ctx *ctx)
{
    if (!ctx->workers.empty()) return;
    for (int i = 0; i < kServeStreams; i++) {
        hipStream_t s;
        HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        ctx->serve_streams.push_back(s);
    }
    for (int i = 0; i < kServeStreams; i++) ctx->workers.emplace_back(serve_worker, ctx, i);
}

bbc_ticket enqueue_request(bbc_ctx *ctx, std::shared_ptr<Request> r)
{
    std::lock_guard<std::mutex> lk(ctx->q_mu);
    if (ctx->workers.empty()) start_serving(ctx);
    r->id = ctx->next_ticket++;
    ctx->requests[r->id] = r;
    ctx->queue.push_back(r);
    ctx->peak_queued = std::max<uint64_t>(ctx->peak_queued, ctx->queue.size());
    ctx->q_cv.notify_one();
    return r->id;
}

}  // namespace

namespace {

// ------------------------------------------------- no-allocation counts
// The workspace of bbc_count_global_noalloc: a static device array (each
// device the library runs on holds its own copy until the process ends). Its
// device address is looked up once per device when a context is created on
// it; host code passes that address, never the array's name.
constexpr uint64_t kNoallocScratchBytes = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_noalloc_mu;
char g_noalloc_host[1u << 20];     // counters, counts and carries read back

// Look the array up on the current device (called with `device` current).
hipError_t init_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char *bbc_status_string(bbc_status s)
{
    switch (s) {
        case BBC_OK: return "ok";
        case BBC_E_INVAL: return "invalid argument";
        case BBC_E_RANGE: return "edge endpoint out of range";
        case BBC_E_SIGN: return "invalid edge sign";
        case BBC_E_DUP_EDGE: return "duplicate edge";
        case BBC_E_NOMEM: return "out of device memory or over the memory cap";
        case BBC_E_OVERFLOW: return "count does not fit in int64";
        case BBC_E_UNSUPPORTED: return "unsupported (p, q) or input";
        case BBC_E_NOT_READY: return "request not finished";
        case BBC_E_UNKNOWN_TICKET: return "unknown ticket";
        case BBC_E_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *bbc_last_error(bbc_ctx *ctx)
{
    if (!ctx) return "null context";
    return ctx->last_error.c_str();
}

bbc_status bbc_ctx_create(int device, void *hip_stream, uint64_t mem_cap_bytes, bbc_ctx **out)
{
    if (!out) return BBC_E_INVAL;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) { (void)hipGetLastError(); return BBC_E_HIP; }
    if (device < 0 || device >= n) return BBC_E_INVAL;
    std::unique_ptr<bbc_ctx> ctx(new (std::nothrow) bbc_ctx());
    if (!ctx) return BBC_E_NOMEM;
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) { (void)hipGetLastError(); return BBC_E_HIP; }
    if (init_scratch(device) != hipSuccess) { (void)hipGetLastError(); return BBC_E_HIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
    ctx->al.reset(new Allocator(mem_cap_bytes));
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            return BBC_E_HIP;
        }
        ctx->own_stream = true;
    }
    *out = ctx.release();
    return BBC_OK;
}

void bbc_ctx_destroy(bbc_ctx *ctx)
{
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->q_mu);
        ctx->stopping = true;
    }
    ctx->q_cv.notify_all();
    for (auto &t : ctx->workers) t.join();
    for (auto s : ctx->serve_streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    (void)hipStreamSynchronize(ctx->stream);
    ctx->requests.clear();
    ctx->queue.clear();
    // graphs the caller did not free: their device memory goes back before
    // the allocator is destroyed with the context
    for (bbc_graph *g : ctx->graphs) delete g;
    ctx->graphs.clear();
    if (ctx->work.exec) { (void)hipGraphExecDestroy(ctx->work.exec); ctx->work.exec = nullptr; }
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : ctx->tev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

bbc_status bbc_build_csr(bbc_ctx *ctx, uint32_t n_u, uint32_t n_v, uint64_t n_edges,
                         const uint32_t *eu, const uint32_t *ev, const void *sign, uint32_t flags,
                         bbc_graph **out)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!out) fail(BBC_E_INVAL, "null output pointer");
        (void)hipSetDevice(ctx->device);
        uint64_t off[2] = {0, n_edges};
        CooIn in{1, &n_u, &n_v, off, eu, ev, sign, flags};
        auto set = build_set(ctx, in, ctx->stream, ctx->work.bhost);
        bbc_graph *h = new bbc_graph{set, 0};
        std::lock_guard<std::mutex> lk(ctx->g_mu);
        ctx->graphs.insert(h);
        *out = h;
    });
}

bbc_status bbc_build_csr_batch(bbc_ctx *ctx, uint32_t n_graphs, const uint32_t *n_u,
                               const uint32_t *n_v, const uint64_t *edge_offsets,
                               const uint32_t *eu, const uint32_t *ev, const void *sign,
                               uint32_t flags, bbc_graph **out_graphs)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!out_graphs || !n_u || !n_v || !edge_offsets) fail(BBC_E_INVAL, "null argument");
        if (n_graphs == 0) fail(BBC_E_INVAL, "n_graphs is 0");
        (void)hipSetDevice(ctx->device);
        CooIn in{n_graphs, n_u, n_v, edge_offsets, eu, ev, sign, flags};
        auto set = build_set(ctx, in, ctx->stream, ctx->work.bhost);
        std::vector<bbc_graph *> hs(n_graphs, nullptr);
        for (uint32_t i = 0; i < n_graphs; i++) hs[i] = new bbc_graph{set, i};
        std::lock_guard<std::mutex> lk(ctx->g_mu);
        ctx->graphs.insert(hs.begin(), hs.end());
        std::copy(hs.begin(), hs.end(), out_graphs);
    });
}

bbc_status bbc_graph_free(bbc_ctx *ctx, bbc_graph *g)
{
    if (!ctx || !g) return BBC_E_INVAL;
    {
        std::lock_guard<std::mutex> lk(ctx->g_mu);
        if (!ctx->graphs.erase(g)) return BBC_E_INVAL;   // not a live graph of this context
    }
    delete g;
    return BBC_OK;
}

bbc_status bbc_get_graph_info(bbc_ctx *ctx, const bbc_graph *g, bbc_graph_info *out)
{
    if (!ctx || !g || !out) return BBC_E_INVAL;
    const GraphDesc &d = g->set->desc[g->idx];
    out->n_u = d.n_u;
    out->n_v = d.n_v;
    out->n_edges = d.m;
    out->anchor_side = (int32_t)d.side;
    out->device_bytes = g->set->G == 1 ? g->set->device_bytes()
                                       : (uint64_t)((double)g->set->device_bytes() * d.m /
                                                    std::max<uint64_t>(g->set->M, 1));
    return BBC_OK;
}

// Count mode of a global count of balanced (p, q)-bicliques on g: the
// vertices on the graph's anchor side form the enumerated subsets (3: pairs
// of candidates, 4: triples), those on the other side are chosen by C(n, q);
// (p, q) with the sides exchanged is the same count on the transposed graph.
// *nb receives the number taken on the other side.
// Device of p if it is device memory the HIP runtime knows, else -1 (host
// memory).
static int device_of_pointer(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return a.type == hipMemoryTypeDevice ? a.device : -1;
}

static int global_count_mode(const bbc_graph *g, int p, int q, int *nb)
{
    const uint32_t side = g->set->desc[g->idx].side;
    const int na = side == 0 ? p : q;
    *nb = side == 0 ? q : p;
    if (na == 3 && *nb == 3) return 0;
    if (na == 3 && *nb >= 4 && *nb <= 7) return 3;
    if ((na == 4 || na == 5) && *nb >= 3 && *nb <= 7) return na;
    fail(BBC_E_UNSUPPORTED,
         "(p, q) = (%d, %d) on a graph anchored on %s: supported are 3, 4 or 5 vertices on "
         "the anchor side (BBC_ANCHOR_U / BBC_ANCHOR_V) and 3..7 on the other",
         p, q, side ? "V" : "U");
}

bbc_status bbc_count_global(bbc_ctx *ctx, const bbc_graph *g, int p, int q, int64_t *out_count)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!g || !out_count) fail(BBC_E_INVAL, "null argument");
        int nb = 3;
        const int mode = global_count_mode(g, p, q, &nb);
        (void)hipSetDevice(ctx->device);
        int64_t v = 0;
        count_sync(ctx, ctx->work, *g->set, g->idx, g->idx + 1, mode, default_shape(ctx), ctx->stream,
                   &v, (uint32_t)nb);
        *out_count = v;
    });
}

bbc_status bbc_count_global_noalloc(bbc_ctx *ctx, const bbc_graph *g, int p, int q,
                                    int64_t *out_count)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!g || !out_count) fail(BBC_E_INVAL, "null argument");
        int nb = 3;
        const int mode = global_count_mode(g, p, q, &nb);
        (void)hipSetDevice(ctx->device);
        void *base = scratch_of(ctx->device);
        if (!base) fail(BBC_E_HIP, "no static scratch address for device %d", ctx->device);
        // one no-allocation count at a time in this process: the calls share
        // the device's scratch array and the host readback buffer
        std::lock_guard<std::mutex> lk(g_noalloc_mu);
        Allocator arena(base, kNoallocScratchBytes);
        Work w;
        w.arena = &arena;
        w.host.use_external(g_noalloc_host, sizeof(g_noalloc_host));
        int64_t v = 0;
        count_sync(ctx, w, *g->set, g->idx, g->idx + 1, mode, default_shape(ctx), ctx->stream, &v,
                   (uint32_t)nb);
        *out_count = v;
    });
}

bbc_status bbc_count_through_edges(bbc_ctx *ctx, const bbc_graph *g, uint64_t n_queries,
                                   const uint32_t *eu, const uint32_t *ev, const int8_t *es,
                                   int64_t *out)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!g) fail(BBC_E_INVAL, "null graph");
        if (n_queries == 0) return;
        if (!eu || !ev || !es || !out) fail(BBC_E_INVAL, "null argument");
        const GraphSet &set = *g->set;
        const GraphDesc &d = set.desc[g->idx];
        for (uint64_t i = 0; i < n_queries; i++) {
            if (eu[i] >= d.n_u || ev[i] >= d.n_v)
                fail(BBC_E_RANGE, "query %llu: edge (%u, %u) outside %u x %u", (unsigned long long)i,
                     eu[i], ev[i], d.n_u, d.n_v);
            if (es[i] != 1 && es[i] != -1)
                fail(BBC_E_SIGN, "query %llu: sign %d is not +1 or -1", (unsigned long long)i, (int)es[i]);
        }
        (void)hipSetDevice(ctx->device);
        Allocator *al = ctx->al.get();
        hipStream_t s = ctx->stream;
        // scratch for the largest degree D of the set, per query of a batch;
        // the batch holds as many queries as fit 512 MiB
        const uint64_t D = set.max_deg;
        uint32_t lg = 6;
        while ((1ull << lg) < 2 * (D + 1)) lg++;
        const uint64_t H = 1ull << lg;
        const uint64_t mask_stride = (D + 1) * (D / 32 + 1);
        const uint64_t per_query = 4 * (8 + 2 + 2 * H + (D + 1) + mask_stride) + 16;
        const uint64_t Q = std::max<uint64_t>(1, std::min<uint64_t>({n_queries, (512ull << 20) / per_query, 65536}));
        DBuf inv, ctl, res, hk, hv, part, masks, qbuf;
        inv.ensure(al, std::max<uint64_t>(d.n_s, 1) * 4);
        ctl.ensure(al, Q * 8 * 4);
        res.ensure(al, Q * 8);
        hk.ensure(al, Q * H * 4);
        hv.ensure(al, Q * H * 4);
        part.ensure(al, Q * (D + 1) * 4);
        masks.ensure(al, Q * mask_stride * 4);
        qbuf.ensure(al, Q * sizeof(EdgeQuery));
        EdgeScratch x;
        x.inv = inv.as<uint32_t>();
        x.ctl = ctl.as<uint32_t>();
        x.result = res.as<unsigned long long>();
        x.hkey = hk.as<uint32_t>();
        x.hval = hv.as<uint32_t>();
        x.lg = lg;
        x.part = part.as<uint32_t>();
        x.part_stride = (uint32_t)(D + 1);
        x.masks = masks.as<uint32_t>();
        x.mask_stride = mask_stride;
        const CsrView view = set.view();
        HIP_OK(edge_inverse(view, d.s_base, d.n_s, x, s));
        std::vector<EdgeQuery> hq(Q);
        std::vector<unsigned long long> hr(Q);
        for (uint64_t q0 = 0; q0 < n_queries; q0 += Q) {
            const uint32_t n = (uint32_t)std::min<uint64_t>(Q, n_queries - q0);
            for (uint32_t i = 0; i < n; i++) {
                // a on the anchor side S, b on the other
                const uint64_t j = q0 + i;
                hq[i].a_id = d.side ? ev[j] : eu[j];
                hq[i].b_idx = d.o_base + (d.side ? eu[j] : ev[j]);
                hq[i].neg = es[j] < 0 ? 1u : 0u;
                hq[i].pad = 0;
            }
            HIP_OK(hipMemcpyAsync(qbuf.p, hq.data(), n * sizeof(EdgeQuery), hipMemcpyHostToDevice, s));
            HIP_OK(edge_through(view, qbuf.as<EdgeQuery>(), n, x, s));
            HIP_OK(hipMemcpyAsync(hr.data(), x.result, n * 8ull, hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            for (uint32_t i = 0; i < n; i++) {
                if (hr[i] > (unsigned long long)INT64_MAX)
                    fail(BBC_E_OVERFLOW, "query %llu: count needs more than 63 bits", (unsigned long long)(q0 + i));
                out[q0 + i] = (int64_t)hr[i];
            }
        }
    });
}

bbc_status bbc_count_bbwc(bbc_ctx *ctx, const bbc_graph *g, int p, int q, int64_t *out_count)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!g || !out_count) fail(BBC_E_INVAL, "null argument");
        const GraphDesc &d = g->set->desc[g->idx];
        const int na = d.side == 0 ? p : q, nb = d.side == 0 ? q : p;
        if (na != 3 || nb < 3 || nb > 7)
            fail(BBC_E_UNSUPPORTED, "(p, q) = (%d, %d): the wedge-centric path takes 3 vertices on "
                                    "the anchor side (%s) and 3..7 on the other",
                 p, q, d.side ? "V" : "U");
        (void)hipSetDevice(ctx->device);
        Allocator *al = ctx->al.get();
        hipStream_t s = ctx->stream;
        const uint32_t lg = 19;
        const uint32_t grid = std::max(1u, (uint32_t)ctx->num_cus / 2);
        const uint64_t slots = (uint64_t)grid << lg;
        DBuf keys, cnt, used, small;
        keys.ensure(al, slots * 8);
        cnt.ensure(al, slots * 16);
        used.ensure(al, slots * 4);
        small.ensure(al, 64);
        BbwcArgs A;
        A.g = g->set->view();
        A.a0 = d.s_base;
        A.a1 = d.s_base + d.n_s;
        A.q = (uint32_t)nb;
        A.lg = lg;
        A.keys = keys.as<unsigned long long>();
        A.cnt = cnt.as<uint32_t>();
        A.used = used.as<uint32_t>();
        A.total = small.as<unsigned long long>();
        A.cursor = small.as<uint32_t>() + 2;
        A.flags = small.as<uint32_t>() + 3;
        HIP_OK(bbwc_count(A, grid, s));
        uint32_t h[4];
        HIP_OK(hipMemcpyAsync(h, small.p, 16, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        const uint32_t flags = h[3];
        if (flags & 1u)
            fail(BBC_E_UNSUPPORTED, "an anchor has more than %llu wedge pairs (the wedge-centric "
                                    "path's table)", (unsigned long long)((1u << lg) - (1u << lg) / 4));
        if (flags & 2u) fail(BBC_E_OVERFLOW, "the count does not fit 64 bits");
        const unsigned long long v = (unsigned long long)h[0] | ((unsigned long long)h[1] << 32);
        if (v > (unsigned long long)INT64_MAX) fail(BBC_E_OVERFLOW, "the count does not fit int64");
        *out_count = (int64_t)v;
    });
}

bbc_status bbc_count_per_vertex(bbc_ctx *ctx, const bbc_graph *g, int p, int q, int side,
                                int64_t *out_per_vertex, int64_t *out_count)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!g || !out_per_vertex) fail(BBC_E_INVAL, "null argument");
        if (p != 3 || q != 3) fail(BBC_E_UNSUPPORTED, "only (p, q) = (3, 3) is supported");
        if (side != 0 && side != 1) fail(BBC_E_INVAL, "side must be 0 (U) or 1 (V)");
        (void)hipSetDevice(ctx->device);
        GraphSet &set = *g->set;
        const GraphDesc &d = set.desc[g->idx];
        const int mode = (uint32_t)side == d.side ? 1 : 2;
        int64_t v = 0;
        count_sync(ctx, ctx->work, set, g->idx, g->idx + 1, mode, default_shape(ctx), ctx->stream, &v);
        Work &w = ctx->work;
        const int out_dev = device_of_pointer(out_per_vertex);
        if (out_dev >= 0 && out_dev != ctx->device)
            fail(BBC_E_INVAL, "out_per_vertex is memory of device %d, the context's is %d", out_dev,
                 ctx->device);
        if (out_dev >= 0) {
            // a device array of this device: remapped and checked on the GPU
            const uint32_t n = mode == 1 ? d.n_s : d.n_o;
            const unsigned long long *pv = mode == 1 ? w.pv.as<unsigned long long>() + d.s_base
                                                     : w.pv_o.as<unsigned long long>() + d.o_base;
            const uint32_t *id = mode == 1 ? set.s_vert.as<uint32_t>() + d.s_base : nullptr;
            uint32_t *bad = w.carry.as<uint32_t>();   // (the count's carries were read already)
            HIP_OK(fill_u32(bad, 0, 1, ctx->stream));
            HIP_OK(per_vertex_to_device(pv, id, n, out_per_vertex, bad, ctx->stream));
            uint32_t hb = 0;
            HIP_OK(hipMemcpyAsync(&hb, bad, 4, hipMemcpyDeviceToHost, ctx->stream));
            HIP_OK(hipStreamSynchronize(ctx->stream));
            if (hb) fail(BBC_E_OVERFLOW, "per-vertex count exceeds int64");
        } else if (mode == 1) {
            const uint32_t n = d.n_s;
            std::vector<uint64_t> pv(n);
            std::vector<uint32_t> vert(n);
            if (n) {
                HIP_OK(hipMemcpyAsync(pv.data(), w.pv.as<uint64_t>() + d.s_base, n * 8ull,
                                      hipMemcpyDeviceToHost, ctx->stream));
                HIP_OK(hipMemcpyAsync(vert.data(), set.s_vert.as<uint32_t>() + d.s_base, n * 4ull,
                                      hipMemcpyDeviceToHost, ctx->stream));
                HIP_OK(hipStreamSynchronize(ctx->stream));
            }
            std::vector<int64_t> res(n, 0);
            for (uint32_t i = 0; i < n; i++) {
                if (pv[i] > (uint64_t)INT64_MAX) fail(BBC_E_OVERFLOW, "per-vertex count exceeds int64");
                res[vert[i]] = (int64_t)pv[i];
            }
            std::copy(res.begin(), res.end(), out_per_vertex);
        } else {
            const uint32_t n = d.n_o;
            std::vector<uint64_t> pv(n);
            if (n) {
                HIP_OK(hipMemcpyAsync(pv.data(), w.pv_o.as<uint64_t>() + d.o_base, n * 8ull,
                                      hipMemcpyDeviceToHost, ctx->stream));
                HIP_OK(hipStreamSynchronize(ctx->stream));
            }
            for (uint32_t i = 0; i < n; i++) {
                if (pv[i] > (uint64_t)INT64_MAX) fail(BBC_E_OVERFLOW, "per-vertex count exceeds int64");
                out_per_vertex[i] = (int64_t)pv[i];
            }
        }
        if (out_count) *out_count = v;
    });
}

bbc_status bbc_top_vertices(bbc_ctx *ctx, const bbc_graph *g, int side, uint32_t k,
                            uint32_t *out_ids, int64_t *out_counts, uint32_t *out_n)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!g || !out_n || (k > 0 && (!out_ids || !out_counts))) fail(BBC_E_INVAL, "null argument");
        if (side != 0 && side != 1) fail(BBC_E_INVAL, "side must be 0 (U) or 1 (V)");
        const GraphDesc &d = g->set->desc[g->idx];
        const uint32_t n = side == 0 ? d.n_u : d.n_v;
        std::vector<int64_t> pv(std::max<uint32_t>(n, 1));
        const bbc_status st = bbc_count_per_vertex(ctx, g, 3, 3, side, pv.data(), nullptr);
        if (st != BBC_OK) fail(st, "%s", ctx->last_error.c_str());
        // the k largest counts, ties to the smaller id
        std::vector<uint32_t> ids(n);
        for (uint32_t i = 0; i < n; i++) ids[i] = i;
        const uint32_t kk = std::min(k, n);
        std::partial_sort(ids.begin(), ids.begin() + kk, ids.end(), [&](uint32_t a, uint32_t b) {
            return pv[a] != pv[b] ? pv[a] > pv[b] : a < b;
        });
        for (uint32_t i = 0; i < kk; i++) {
            out_ids[i] = ids[i];
            out_counts[i] = pv[ids[i]];
        }
        *out_n = kk;
    });
}

bbc_status bbc_count_batch(bbc_ctx *ctx, const bbc_graph *const *graphs, uint32_t n_graphs,
                           int64_t *out_counts)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if ((!graphs || !out_counts) && n_graphs) fail(BBC_E_INVAL, "null argument");
        for (uint32_t i = 0; i < n_graphs; i++)
            if (!graphs[i]) fail(BBC_E_INVAL, "null graph %u", i);
        (void)hipSetDevice(ctx->device);
        std::vector<int64_t> res(n_graphs, 0);
        uint32_t i = 0;
        while (i < n_graphs) {
            GraphSet *set = graphs[i]->set.get();
            // the whole set in its own order: one batched replay
            if (graphs[i]->idx == 0 && i + set->G <= n_graphs) {
                bool whole = true;
                for (uint32_t j = 0; j < set->G && whole; j++)
                    whole = graphs[i + j]->set.get() == set && graphs[i + j]->idx == j;
                if (whole) {
                    count_set_batched(ctx, ctx->work, *set, ctx->stream, res.data() + i);
                    i += set->G;
                    continue;
                }
            }
            // otherwise a contiguous run of one set
            uint32_t j = i + 1;
            while (j < n_graphs && graphs[j]->set.get() == set && graphs[j]->idx == graphs[j - 1]->idx + 1) j++;
            count_sync(ctx, ctx->work, *set, graphs[i]->idx, graphs[j - 1]->idx + 1, 0,
                       default_shape(ctx), ctx->stream, res.data() + i);
            i = j;
        }
        std::copy(res.begin(), res.end(), out_counts);
    });
}

bbc_status bbc_submit(bbc_ctx *ctx, const bbc_graph *g, bbc_ticket *out)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!g || !out) fail(BBC_E_INVAL, "null argument");
        auto r = std::make_shared<Request>();
        r->set = g->set;
        r->idx = g->idx;
        const GraphDesc &d = g->set->desc[g->idx];
        r->m = d.m;
        r->n_s_max = d.n_s;
        r->max_deg = g->set->max_deg;
        *out = enqueue_request(ctx, r);
    });
}

// requests of this many edges or more are copied and measured by up to
// kSubmitThreads threads
constexpr uint64_t kSubmitSplitEdges = 1ull << 18;
constexpr uint32_t kSubmitThreads = 8;

bbc_status bbc_submit_coo(bbc_ctx *ctx, uint32_t n_u, uint32_t n_v, uint64_t n_edges,
                          const uint32_t *eu, const uint32_t *ev, const void *sign, uint32_t flags,
                          bbc_ticket *out)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (!out) fail(BBC_E_INVAL, "null output pointer");
        check_flags(flags);
        if (flags & BBC_IN_DEVICE_PTRS) fail(BBC_E_INVAL, "bbc_submit_coo takes host arrays");
        if (n_edges && (!eu || !ev || !sign)) fail(BBC_E_INVAL, "null edge array");
        auto r = std::make_shared<Request>();
        r->n_u = n_u; r->n_v = n_v; r->m = n_edges; r->flags = flags;
        r->eu.resize(n_edges);
        r->ev.resize(n_edges);
        const uint8_t *sp = (const uint8_t *)sign;
        r->sign.assign(sp, sp + sign_bytes(n_edges, flags));
        // The copy and the degrees (the largest bounds the workspace the count
        // needs, their wedges its size) run on the caller's thread; a large
        // request is split over a few threads, each with its own degree arrays.
        // (all threads' degree arrays together take no more bytes than the
        // copied edge endpoints)
        const uint64_t nvx = std::max<uint64_t>(1, (uint64_t)n_u + n_v);
        const uint32_t nt = n_edges >= kSubmitSplitEdges
                                ? (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(
                                      {kSubmitThreads, std::thread::hardware_concurrency(), 2 * n_edges / nvx}))
                                : 1u;
        std::vector<std::vector<uint32_t>> du(nt), dv(nt);
        auto part = [&](uint32_t t) {
            const uint64_t e0 = n_edges * t / nt, e1 = n_edges * (t + 1) / nt;
            memcpy(r->eu.data() + e0, eu + e0, (e1 - e0) * 4);
            memcpy(r->ev.data() + e0, ev + e0, (e1 - e0) * 4);
            du[t].assign(n_u, 0);
            dv[t].assign(n_v, 0);
            uint32_t *pu = du[t].data(), *pv = dv[t].data();
            for (uint64_t e = e0; e < e1; e++) {
                if (eu[e] < n_u) pu[eu[e]]++;
                if (ev[e] < n_v) pv[ev[e]]++;
            }
        };
        if (nt == 1) {
            part(0);
        } else {
            std::vector<std::thread> th;
            for (uint32_t t = 1; t < nt; t++) th.emplace_back(part, t);
            part(0);
            for (auto &x : th) x.join();
        }
        uint32_t mx = 0;
        uint64_t cu = 0, cv = 0;
        for (uint32_t i = 0; i < n_u; i++) {
            uint32_t x = 0;
            for (uint32_t t = 0; t < nt; t++) x += du[t][i];
            mx = std::max(mx, x);
            cu += (uint64_t)x * (x - (x > 0)) / 2;
        }
        for (uint32_t i = 0; i < n_v; i++) {
            uint32_t x = 0;
            for (uint32_t t = 0; t < nt; t++) x += dv[t][i];
            mx = std::max(mx, x);
            cv += (uint64_t)x * (x - (x > 0)) / 2;
        }
        r->max_deg = mx;
        r->w2_max = std::max(cu, cv);
        r->n_s_max = std::max(n_u, n_v);
        *out = enqueue_request(ctx, r);
    });
}

static bbc_status take_result(bbc_ctx *ctx, bbc_ticket t, int64_t *out_count, bool block)
{
    std::unique_lock<std::mutex> lk(ctx->q_mu);
    auto it = ctx->requests.find(t);
    if (it == ctx->requests.end()) return BBC_E_UNKNOWN_TICKET;
    std::shared_ptr<Request> r = it->second;
    if (block) ctx->done_cv.wait(lk, [&] { return r->done; });
    if (!r->done) return BBC_E_NOT_READY;
    ctx->requests.erase(it);
    if (r->status == BBC_OK && out_count) *out_count = r->result;
    return r->status;
}

bbc_status bbc_poll(bbc_ctx *ctx, bbc_ticket t, int64_t *out_count)
{
    if (!ctx) return BBC_E_INVAL;
    return take_result(ctx, t, out_count, false);
}

bbc_status bbc_wait(bbc_ctx *ctx, bbc_ticket t, int64_t *out_count)
{
    if (!ctx) return BBC_E_INVAL;
    return take_result(ctx, t, out_count, true);
}

bbc_status bbc_set_timing(bbc_ctx *ctx, int enable)
{
    if (!ctx) return BBC_E_INVAL;
    return guard(ctx, [&] {
        if (enable && !ctx->ev[0])
            for (auto &e : ctx->ev) HIP_OK(hipEventCreate(&e));
        ctx->timing = enable != 0;
    });
}

bbc_status bbc_get_memory_stats(bbc_ctx *ctx, bbc_memory_stats *out)
{
    if (!ctx || !out) return BBC_E_INVAL;
    bbc_memory_stats m{};
    m.cap_bytes = ctx->al->cap();
    m.reserved_bytes = ctx->al->used();
    m.peak_reserved_bytes = ctx->al->peak();
    m.live_bytes = ctx->al->live(0) + ctx->al->live(1);
    {
        std::lock_guard<std::mutex> lk(ctx->q_mu);
        m.serve_admitted_bytes = ctx->admitted_bytes;
        m.serve_peak_admitted_bytes = ctx->peak_admitted;
        m.serve_queued = ctx->queue.size();
        m.serve_peak_queued = ctx->peak_queued;
    }
    *out = m;
    return BBC_OK;
}

bbc_status bbc_set_test_hook(bbc_ctx *ctx, int hook, int64_t value)
{
    if (!ctx) return BBC_E_INVAL;
    switch (hook) {
        case BBC_HOOK_NO_WINDOW_TIER: ctx->hook_no_window = value != 0; return BBC_OK;
        case BBC_HOOK_PRELOAD_COUNT: ctx->hook_preload = (uint64_t)value; return BBC_OK;
        case BBC_HOOK_LAUNCH_SHAPE: {
            if (value == 0) { ctx->hook_shape_set = false; return BBC_OK; }
            const uint64_t v = (uint64_t)value;
            Shape sh;
            sh.chunk_base = (uint32_t)(v & 0xffffffffu);
            sh.grid_t_per_cu = (uint32_t)((v >> 32) & 0xffu);
            sh.grid_a_per_cu = (uint32_t)((v >> 40) & 0xffu);
            const bool pow2 = (sh.chunk_base & (sh.chunk_base - 1)) == 0;
            if (!pow2 || sh.chunk_base < 256 || sh.chunk_base > 16384 || sh.grid_t_per_cu < 1 ||
                sh.grid_t_per_cu > 16 || sh.grid_a_per_cu < 1 || sh.grid_a_per_cu > 8 || (v >> 48))
                return BBC_E_INVAL;
            ctx->hook_shape = sh;
            ctx->hook_shape_set = true;
            return BBC_OK;
        }
        default: return BBC_E_INVAL;
    }
}

bbc_status bbc_get_last_stats(bbc_ctx *ctx, bbc_count_stats *out)
{
    if (!ctx || !out) return BBC_E_INVAL;
    *out = ctx->stats;
    return BBC_OK;
}

}  // extern "C"
