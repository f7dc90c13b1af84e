// libatos: C ABI over the persistent worklist kernel and the level-synchronous
// baselines (declarations and contracts in include/atos.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "atos.h"
#include "atos_device.h"
#include "atos_frontier.h"
#include "atos_internal.h"
#include "atos_persistent.h"

using namespace atos;
using namespace atos::host;

namespace {

constexpr uint32_t kDefaultTimeoutMs = 60000;
constexpr uint32_t kDefaultOrderDegree = 8;
constexpr uint32_t kDefaultCombFlush = 131072;  // edges per worker between table flushes
// batches: the 640-instance workload takes 449 ms with 32,768, 461 ms with
// 65,536, 485 ms with 131,072 and 517 ms uncombined
constexpr uint32_t kDefaultBatchCombFlush = 32768;
constexpr uint64_t kMinRing = 1ull << 10;
constexpr uint64_t kDefaultMinRing = 1ull << 16;
constexpr uint64_t kMaxRing = 1ull << 32;

// ------------------------------------------------------------------ config
struct Cfg {
    int strategy, worker, fetch, grid, check_size;
    uint32_t split_degree;  // hub-board threshold in edges; 0 = never split
    uint32_t order_degree;  // colouring: degree of the ordered class; 0 = none
    uint32_t n_queues;  // worklist rings: 1 shared, or one per XCD
    uint64_t capacity;  // slots per ring
    uint32_t timeout_ms;
    bool fetch_fixed;   // pops always take up to `fetch` (else their share of the ring)
    bool push_shallow;  // publish into the shallowest ring (else the worker's own)
    uint32_t discrete_tail;  // discrete runs: queued tasks at which the rest runs persistent
    uint32_t forbid_all;     // colouring: avoid every neighbour's colour (no ordered class)
    const uint32_t* abort_flag;  // host word that stops the run, or null
    uint32_t comb_flush;     // PageRank combining: table flush window in edges (0 = off)
    bool segmented;          // batches: every task into the ring of its vertex's segment
    uint32_t seg_bound[kMaxQueues - 1];  // first vertex of segments 1..7 (set by the batch)
};

atos_status resolve_cfg(const GraphRec& g, int app, const atos_config* in, Cfg& c) {
    atos_config z;
    std::memset(&z, 0, sizeof(z));
    const atos_config& u = in ? *in : z;
    if (u.push_policy != ATOS_PUSH_AUTO && u.push_policy != ATOS_PUSH_OWN &&
        u.push_policy != ATOS_PUSH_SHALLOWEST)
        return ATOS_EINVAL;
    // colouring and persistent PageRank publish into the shallowest ring by
    // default (R-MAT scale 22: colouring 107 ms against 115 ms, PageRank 403 ms
    // against 546 ms; road grid PageRank 52 ms against 77 ms); BFS (road grid
    // 22 ms against 39 ms) and PageRank in rounds (R-MAT scale 22: 388 ms
    // against 550 ms) into the worker's own ring
    c.push_shallow = u.push_policy == ATOS_PUSH_SHALLOWEST ||
                     (u.push_policy == ATOS_PUSH_AUTO &&
                      (app == ATOS_APP_COLOR ||
                       (app == ATOS_APP_PAGERANK && u.strategy == ATOS_PERSISTENT)));
    if (u.fetch_policy != ATOS_FETCH_AUTO && u.fetch_policy != ATOS_FETCH_FIXED &&
        u.fetch_policy != ATOS_FETCH_ADAPTIVE)
        return ATOS_EINVAL;
    // adaptive claims spread the heavy, few ready tasks of colouring's ordered
    // class over many workers; for BFS and PageRank, whose shallow worklists
    // (road-like graphs) hold light tasks, they only add pops
    c.fetch_fixed = u.fetch_policy == ATOS_FETCH_AUTO ? app != ATOS_APP_COLOR
                                                      : u.fetch_policy == ATOS_FETCH_FIXED;
    c.strategy = u.strategy;
    if (c.strategy != ATOS_PERSISTENT && c.strategy != ATOS_BSP && c.strategy != ATOS_DISCRETE &&
        c.strategy != ATOS_ROUNDS)
        return ATOS_EINVAL;
    c.segmented = u.queue_layout == ATOS_QUEUE_SEGMENTED;
    for (int b = 0; b < kMaxQueues - 1; ++b) c.seg_bound[b] = 0xFFFFFFFFu;
    if (u.queue_layout == ATOS_QUEUE_GLOBAL) c.n_queues = 1;
    else if (u.queue_layout == ATOS_QUEUE_AUTO || u.queue_layout == ATOS_QUEUE_PER_XCD ||
             c.segmented)
        c.n_queues = kMaxQueues;
    else return ATOS_EUNSUPPORTED;
    // default workers: 1024 threads, except colouring on a scale-free graph
    // (largest degree above 32 times the average): 512, whose chunks of the
    // ordered chain's long lists are half as long and whose kernel does not
    // spill (R-MAT scale 20/22/23: 39/88/120 ms against 43/106/141 ms; road
    // grids 2048^2/4096^2 stay at 1024: 5.1/17.2 ms against 5.4/19.2 ms)
    const bool scale_free = g.n > 0 && (double)g.max_deg > 32.0 * std::max(1.0, (double)g.m / (double)g.n);
    c.worker = u.worker ? u.worker : (app == ATOS_APP_COLOR && scale_free) ? 512 : 1024;
    if (c.worker != 64 && c.worker != 128 && c.worker != 256 && c.worker != 512 && c.worker != 1024)
        return ATOS_EINVAL;
    c.fetch = u.fetch ? u.fetch : std::min(c.worker, 256);
    if (c.fetch < 1 || c.fetch > c.worker) return ATOS_EINVAL;
    if (u.split_degree < -1) return ATOS_EINVAL;
    // default hub threshold: BFS splits only lists far longer than a batch;
    // PageRank lists over 2 edges per thread (R-MAT scale 22, 1024-thread
    // workers: 388-403 ms against 395-409 ms at 8 per thread, whatever the
    // strategy); colouring every list longer than one chunk (4 edges per
    // thread), since its ordered class is a chain of long lists
    c.split_degree = u.split_degree == -1 ? 0u
                     : u.split_degree > 0 ? (uint32_t)u.split_degree
                     : app == ATOS_APP_COLOR    ? (uint32_t)std::max(4 * c.worker, 1024)
                     : app == ATOS_APP_PAGERANK ? (uint32_t)std::max(2 * c.worker, 2048)
                                                : (uint32_t)std::max(8 * c.worker, 4096);
    if (u.color_order_degree < -2 || u.color_order_degree > 0xFFFF) return ATOS_EINVAL;
    if (u.color_forbid_all != 0 && u.color_forbid_all != 1) return ATOS_EINVAL;
    c.forbid_all = (uint32_t)u.color_forbid_all;
    // forbid-all colouring has no ordered class unless a degree is given
    c.order_degree = (u.color_order_degree == -1 || (c.forbid_all && u.color_order_degree == 0)) ? 0u
                     : u.color_order_degree == -2 ? g.sqrt_class_degree
                     : u.color_order_degree > 0   ? (uint32_t)u.color_order_degree
                                                  : kDefaultOrderDegree;
    if (u.grid < 0) return ATOS_EINVAL;
    // colouring with 512- or 1024-thread workers: one worker per CU by default,
    // however many the registers would let share a CU (R-MAT scale 22 with
    // 512-thread workers: 89 ms with 256 workers, 97 ms with 384, 108 ms with
    // 512: more workers only contend for the ordered class's chain)
    c.grid = u.grid ? u.grid : (app == ATOS_APP_COLOR && c.worker >= 512) ? g.num_cu : 0;
    if (u.pr_check_size < 0) return ATOS_EINVAL;
    c.check_size = u.pr_check_size;
    // Algorithm 4's sweep: global PageRank in one persistent kernel (per launch)
    if (c.check_size != 0 && (app != ATOS_APP_PAGERANK || c.strategy != ATOS_PERSISTENT))
        return ATOS_EUNSUPPORTED;
    if (c.check_size > 65536) return ATOS_EINVAL;
    if (u.queue_capacity < 0) return ATOS_EINVAL;
    uint64_t want = (uint64_t)u.queue_capacity;
    if (want == 0) {
        // all rings together hold 4n (BFS) or 8n (PageRank, colouring) entries
        const uint64_t n = (uint64_t)std::max<int64_t>(g.n, 1);
        want = std::max<uint64_t>(kDefaultMinRing, (app == ATOS_APP_BFS ? 4 * n : 8 * n) / c.n_queues);
    }
    c.capacity = std::max(kMinRing, next_pow2(want));
    if (c.capacity > kMaxRing) return ATOS_EINVAL;
    c.timeout_ms = u.timeout_ms ? u.timeout_ms : kDefaultTimeoutMs;
    c.discrete_tail = u.discrete_tail;
    if (u.pr_combine < -1) return ATOS_EINVAL;
    // PageRank residue combining (PrCombApp): on by default for whole-graph
    // PageRank with 1024-thread workers, whose one workgroup per CU leaves the
    // LDS free for the table (R-MAT scale 22: 286 ms against 387-397 ms for the
    // best plain launch shapes; the road grid has no vertex of degree >= 64 and
    // runs as before); smaller workers would lose co-resident workgroups to it
    const bool comb_ok = app == ATOS_APP_PAGERANK && c.strategy != ATOS_BSP;
    if (u.pr_combine > 0 && !comb_ok) return ATOS_EUNSUPPORTED;
    c.comb_flush = u.pr_combine > 0                                  ? (uint32_t)u.pr_combine
                   : (u.pr_combine == 0 && comb_ok && c.worker == 1024) ? kDefaultCombFlush
                                                                        : 0u;
    c.abort_flag = u.abort_flag;
    return ATOS_OK;
}

// ------------------------------------------------------------------ workspace layout
struct Layout {
    size_t ring = 0, inv_deg = 0, residue = 0, rank64 = 0, queued = 0, key = 0, wait = 0, mask = 0,
           front_a = 0, front_b = 0, comb_tag = 0, comb_vertex = 0, comb_hist = 0, comb_cols = 0,
           total = 0;
};

// PageRank combining: degree classes for picking the combined vertices (exact
// below 32, then 16 classes per octave) and the lowest degree ever combined.
constexpr uint32_t kCombClasses = 512;
constexpr uint32_t kCombMinDegree = 64;

Layout layout(const GraphRec& g, int app, const Cfg& c) {
    Layout L;
    size_t off = align_up(sizeof(WsHeader), 4096);
    const size_t n4 = align_up((size_t)std::max<int64_t>(g.n, 1) * 4, 256);
    if (c.strategy != ATOS_BSP) {
        L.ring = off;
        off += align_up((size_t)c.capacity * 8 * c.n_queues, 256);
    } else {
        L.front_a = off;
        off += n4;
        L.front_b = off;
        off += n4;
    }
    if (app == ATOS_APP_PAGERANK && c.check_size > 0) {  // the clean sweep's finds, queued flags
        L.front_a = off;
        off += n4;
        L.queued = off;
        off += n4;
    }
    if (app == ATOS_APP_PAGERANK) {  // FP64 1/deg, residue and rank
        L.inv_deg = off;
        off += 2 * n4;
        L.residue = off;
        off += 2 * n4;
        L.rank64 = off;
        off += 2 * n4;
    }
    if (app == ATOS_APP_PAGERANK && c.comb_flush != 0 && c.strategy != ATOS_BSP) {
        // combining: each vertex's column tag, the slots' vertices, the degree
        // classes and the tagged copy of the column array
        L.comb_tag = off;
        off += n4;
        L.comb_vertex = off;
        off += align_up((size_t)PrCombApp::kCombSlots * 4, 256);
        L.comb_hist = off;
        off += align_up((size_t)kCombClasses * 4, 256);
        L.comb_cols = off;
        off += align_up((size_t)std::max<int64_t>(g.m, 1) * 4, 256);
    }
    if (app == ATOS_APP_COLOR) {
        L.queued = off;
        off += n4;
        L.key = off;
        off += n4;
        L.wait = off;
        off += n4;
        L.mask = off;  // u64[kColourWords] per vertex, 256-byte aligned as every array here
        off += align_up((size_t)g.n * kColourWords * sizeof(uint64_t), 256);
    }
    L.total = off;
    return L;
}

// ------------------------------------------------------------------ small kernels
template <class OffT>
__global__ void max_degree_kernel(const OffT* offs, int64_t n, unsigned long long* out) {
    unsigned long long best = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        best = std::max(best, (unsigned long long)(offs[v + 1] - offs[v]));
    atomicMax(out, best);
}

// bad[0]: malformed offsets/cols; bad[1]: an edge without its reverse
template <class OffT>
__global__ void validate_kernel(const OffT* offs, const int32_t* cols, int64_t n, int64_t m,
                                int check_sym, uint32_t* bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 == 0 && (offs[0] != 0 || (int64_t)offs[n] != m)) atomicOr(bad, 1u);
    for (int64_t v = t0; v < n; v += stride)
        if (offs[v + 1] < offs[v]) atomicOr(bad, 1u);
    for (int64_t e = t0; e < m; e += stride)
        if (cols[e] < 0 || (int64_t)cols[e] >= n) atomicOr(bad, 1u);
    if (!check_sym) return;
    for (int64_t v = t0; v < n; v += stride) {
        for (OffT e = offs[v]; e < offs[v + 1]; ++e) {
            const int64_t w = cols[e];
            if (w < 0 || w >= n) continue;
            OffT lo = offs[w], hi = offs[w + 1];
            bool found = false;
            while (lo < hi) {  // neighbour lists sorted ascending
                const OffT mid = lo + (hi - lo) / 2;
                if ((int64_t)cols[mid] < v) lo = mid + 1; else hi = mid;
            }
            found = lo < offs[w + 1] && (int64_t)cols[lo] == v;
            if (!found) atomicOr(bad + 1, 1u);
        }
    }
}

// Start of every persistent run: decide where this run's positions begin in
// each ring and whether the rings must be cleared (first use of the
// workspace, another capacity or ring count, or a previous run that stopped
// abnormally), and deal the initial tasks round-robin over the rings.
__global__ void prepare_kernel(WsHeader* H, uint64_t capacity, uint32_t nq, uint64_t n_init) {
    if (blockIdx.x != 0) return;
    for (uint32_t e = threadIdx.x; e < (uint32_t)kBoardEntries; e += blockDim.x) {
        H->board[e].state = kBoardFree;
        H->board[e].finished = 0;
    }
    if (threadIdx.x != 0) return;
    H->board_open = 0;
    for (int w = 0; w < kBoardEntries / 64; ++w) H->board_mask[w] = 0ull;
    H->stat_hub_posts = 0;
    const uint64_t cookie = kCookie ^ capacity ^ ((uint64_t)nq << 56);
    const bool valid = H->cookie == cookie && H->capacity == capacity && H->n_queues == nq;
    for (uint32_t q = 0; q < (uint32_t)kMaxQueues; ++q) {
        QueueCtl* Q = &H->q[q];
        const uint64_t p0 = (valid && q < nq) ? Q->tail : 0ull;
        const uint64_t nq_init = q < nq ? n_init / nq + (q < n_init % nq ? 1 : 0) : 0;
        Q->head = p0;
        Q->tail = p0 + nq_init;
        Q->done = p0;
        Q->init_base = p0;
        Q->n_init = nq_init;
    }
    H->zero_pending = valid ? 0u : 1u;
    H->capacity = capacity;
    H->n_queues = nq;
    H->status = 0u;
    H->check_cursor = 0;
    H->stat_comb_adds = 0;
    H->stat_comb_atomics = 0;
    H->stat_popped = 0;
    H->stat_pushed = 0;
    H->stat_edges = 0;
    H->stat_rounds = 1;
    H->stat_push_retries = 0;
    H->stat_idle = 0;
    H->stat_steals = 0;
    H->scalar_out = 0;
    H->cookie = cookie;
}

// `cap` is the total slot count of all rings.
__device__ inline void maybe_zero_ring(const WsHeader* H, uint64_t* ring, uint64_t cap,
                                       int64_t i0, int64_t stride) {
    if (!H->zero_pending) return;
    for (int64_t i = i0; i < (int64_t)cap; i += stride) ring[i] = 0ull;
}

__global__ void bfs_init_kernel(const WsHeader* H, uint64_t* ring, uint64_t cap, uint32_t* depth,
                                int64_t n, int64_t src) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = i0; v < n; v += stride) depth[v] = v == src ? 0u : 0xFFFFFFFFu;
    if (ring) maybe_zero_ring(H, ring, cap, i0, stride);
}

// PageRank start (all FP64), inv_deg = 1/deg.  Global (source < 0): rank =
// 1-d and residue = 0 everywhere (the residue is then filled by the pull
// pass).  Personalized from `source`: rank = 0 everywhere and residue = 1-d at
// the source, 0 elsewhere, which represents x = (1-d) e_source + d A D^-1 x.
template <class OffT>
__global__ void pr_init_kernel(const WsHeader* H, uint64_t* ring, uint64_t cap, const OffT* offs,
                               int64_t n, double damping, int64_t source, double* rank,
                               double* residue, double* inv_deg) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = i0; v < n; v += stride) {
        const int64_t d = (int64_t)(offs[v + 1] - offs[v]);
        rank[v] = source < 0 ? 1.0 - damping : 0.0;
        residue[v] = v == source ? 1.0 - damping : 0.0;
        inv_deg[v] = d > 0 ? 1.0 / (double)d : 0.0;
    }
    if (ring) maybe_zero_ring(H, ring, cap, i0, stride);
}

// PageRank start, second pass: residue(v) = (1-d)*d * sum_{u in adj(v)} 1/deg(u),
// the residue that makes (rank = 1-d, residue) represent the fixed point.
// Edge-balanced: each thread sums a fixed run of CSR entries and adds one
// partial per vertex boundary it crosses (so hubs are split across threads).
template <class OffT>
__global__ void pr_pull_kernel(const OffT* offs, const int32_t* cols, int64_t n, int64_t m,
                               double coef, const double* inv_deg, double* residue) {
    constexpr int64_t kRun = 32;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t * kRun < m; t += stride) {
        const int64_t e0 = t * kRun;
        const int64_t e1 = std::min(m, e0 + kRun);
        int64_t lo = 0, hi = n;  // vertex v with offs[v] <= e0 < offs[v+1]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)offs[mid] <= e0) lo = mid; else hi = mid;
        }
        int64_t v = lo;
        int64_t vend = (int64_t)offs[v + 1];
        double acc = 0.0;
        // eight neighbours' 1/deg gathered together, then summed in CSR order
        constexpr int kStep = 8;
        for (int64_t eb = e0; eb < e1; eb += kStep) {
            double x[kStep];
#pragma unroll
            for (int j = 0; j < kStep; ++j) x[j] = eb + j < e1 ? inv_deg[cols[eb + j]] : 0.0;
#pragma unroll
            for (int j = 0; j < kStep; ++j) {
                const int64_t e = eb + j;
                if (e >= e1) break;
                while (e >= vend) {
                    if (acc != 0.0) atomicAdd(residue + v, coef * acc);
                    acc = 0.0;
                    ++v;
                    vend = (int64_t)offs[v + 1];
                }
                acc += x[j];
            }
        }
        if (acc != 0.0) atomicAdd(residue + v, coef * acc);
    }
}

// End of PageRank: round the FP64 ranks (and residues, when asked for) to FP32.
__global__ void rank_out_kernel(const double* rank, const double* residue, int64_t n, float* out,
                                float* res_out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        out[v] = (float)rank[v];
        if (res_out) res_out[v] = (float)residue[v];
    }
}

// Colouring start: colour -1, rank key, queued flag (1 when every vertex
// starts queued, as in the persistent run).
// End of PageRank: round the FP64 ranks to the FP32 output.
__global__ void rank_out_kernel(const double* rank, int64_t n, float* out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        out[v] = (float)rank[v];
}

template <class OffT>
__global__ void gc_init_kernel(const WsHeader* H, uint64_t* ring, uint64_t cap, const OffT* offs,
                               int64_t n, uint64_t seed, uint32_t queued_init, int32_t* color,
                               uint32_t* queued, uint32_t* key, uint32_t* wait, uint64_t* mask) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = i0; v < n; v += stride) {
        color[v] = -1;
        queued[v] = queued_init;
        key[v] = colour_key(seed, (uint32_t)v, (uint64_t)(offs[v + 1] - offs[v]));
        wait[v] = 0u;
        if (mask) {
#pragma unroll
            for (int j = 0; j < kColourWords; ++j) mask[(uint64_t)v * kColourWords + j] = 0ull;
        }
    }
    if (ring) maybe_zero_ring(H, ring, cap, i0, stride);
}

// Colouring start, second pass: wait(v) = number of outranking neighbours of
// every vertex of the ordered class (key degree >= order).  Edge-balanced as
// pr_pull_kernel.
template <class OffT>
__global__ void gc_wait_kernel(const OffT* offs, const int32_t* cols, int64_t n, int64_t m,
                               const uint32_t* key, uint32_t order, uint32_t* wait) {
    constexpr int64_t kRun = 32;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t * kRun < m; t += stride) {
        const int64_t e0 = t * kRun;
        const int64_t e1 = std::min(m, e0 + kRun);
        int64_t lo = 0, hi = n;  // vertex v with offs[v] <= e0 < offs[v+1]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)offs[mid] <= e0) lo = mid; else hi = mid;
        }
        int64_t v = lo;
        int64_t vend = (int64_t)offs[v + 1];
        uint32_t acc = 0;
        for (int64_t e = e0; e < e1; ++e) {
            while (e >= vend) {
                if (acc) atomicAdd(wait + v, acc);
                acc = 0;
                ++v;
                vend = (int64_t)offs[v + 1];
            }
            const uint32_t w = (uint32_t)cols[e];
            if (ordered_key(key[v], order) && w != (uint32_t)v && outranks(key, w, (uint32_t)v)) ++acc;
        }
        if (acc) atomicAdd(wait + v, acc);
    }
}

__global__ void color_count_kernel(const int32_t* color, int64_t n, WsHeader* H, int32_t* out) {
    int32_t best = -1;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        best = std::max(best, color[v]);
    atomicMax(&H->scalar_out, best + 1);
}

__global__ void copy_scalar_kernel(const WsHeader* H, int32_t* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = H->scalar_out;
}

__global__ void iota_kernel(uint32_t* out, int64_t n) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        out[v] = (uint32_t)v;
}

__global__ void set_u32_kernel(uint32_t* p, uint32_t v) { *p = v; }

// PageRank combining set-up: count the vertices of degree >= kCombMinDegree
// per degree class; pick the lowest class from which on they fit in the
// table; give each of them a slot and tag its column entries with it.
__host__ __device__ inline uint32_t comb_class(uint64_t d) {
    if (d < 32) return (uint32_t)d;
    const uint32_t e = 63u - (uint32_t)__builtin_clzll(d);  // >= 5
    if (e > 31u) return kCombClasses - 1u;
    return (e - 3u) * 16u + (uint32_t)((d >> (e - 4u)) & 15u);
}
__host__ __device__ inline uint64_t comb_class_min(uint32_t b) {
    if (b < 32u) return b;
    return (uint64_t)(16u + b % 16u) << (b / 16u + 3u - 4u);
}

// Vertices a batch may combine: those of its PageRank instances (all vertices
// of a single graph, ib == nullptr).
struct CombScope {
    const int64_t* ib;
    const int64_t* ie;
    const uint32_t* kind;
    uint32_t n_inst;
};
__device__ inline bool comb_candidate(const CombScope& sc, int64_t v);

template <class OffT>
__global__ void comb_hist_kernel(const OffT* offs, int64_t n, CombScope sc, uint32_t* hist) {
    __shared__ uint32_t h[kCombClasses];
    for (uint32_t j = threadIdx.x; j < kCombClasses; j += blockDim.x) h[j] = 0u;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t d = (uint64_t)(offs[v + 1] - offs[v]);
        if (d >= kCombMinDegree && comb_candidate(sc, v)) atomicAdd(&h[comb_class(d)], 1u);
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < kCombClasses; j += blockDim.x)
        if (h[j]) atomicAdd(&hist[j], h[j]);
}

// one workgroup of kCombClasses threads
__global__ void comb_pick_kernel(const uint32_t* hist, uint32_t slots, WsHeader* H) {
    __shared__ uint32_t suf[kCombClasses];
    __shared__ uint32_t first;
    const uint32_t t = threadIdx.x;
    suf[t] = hist[t];
    if (t == 0) first = kCombClasses;
    __syncthreads();
    // suf[t] = vertices in classes t and above (non-increasing in t)
    for (uint32_t off = 1; off < kCombClasses; off <<= 1) {
        const uint32_t y = t + off < kCombClasses ? suf[t + off] : 0u;
        __syncthreads();
        suf[t] += y;
        __syncthreads();
    }
    if (suf[t] <= slots && (t == 0 || suf[t - 1] > slots)) first = t;  // one t at most
    __syncthreads();
    if (t == 0) {
        // every class from `first` on, then the class below it while slots remain
        auto clamp = [](uint64_t d) {
            return (uint32_t)std::min<uint64_t>(std::max<uint64_t>(d, kCombMinDegree), 0xFFFFFFFFull);
        };
        const uint32_t dmin = first < kCombClasses ? clamp(comb_class_min(first)) : 0xFFFFFFFFu;
        H->comb_min_degree = dmin;
        H->comb_part_degree = first > 0 && first < kCombClasses ? clamp(comb_class_min(first - 1)) : dmin;
        H->comb_base = first < kCombClasses ? suf[first] : 0u;
        H->comb_count = 0u;
        H->comb_part_count = 0u;
    }
}

template <class OffT>
__global__ void comb_slot_kernel(const OffT* offs, int64_t n, CombScope sc, WsHeader* H, uint32_t slots,
                                 uint32_t* tag, uint32_t* vertex) {
    const uint64_t dmin = H->comb_min_degree, dpart = H->comb_part_degree;
    const uint32_t base = H->comb_base;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t d = (uint64_t)(offs[v + 1] - offs[v]);
        uint32_t t = (uint32_t)v;
        uint32_t sl = 0xFFFFFFFFu;
        if (d >= dpart && comb_candidate(sc, v)) {
            if (d >= dmin) sl = atomicAdd(&H->comb_count, 1u);  // < base, by the choice of dmin
            else sl = base + atomicAdd(&H->comb_part_count, 1u);
        }
        if (sl < slots) {
            vertex[sl] = (uint32_t)v;
            t = kCombTag | sl;
        }
        tag[v] = t;
    }
}

// Colouring's sqrt(n) ordered class: the lowest degree class from which on
// at most ceil(sqrt(n)) vertices of degree >= 64 lie (degree classes as for
// combining); 0 when no vertex reaches degree 64.
uint32_t sqrt_class_degree(const uint32_t* hist, int64_t n) {
    const uint64_t k = (uint64_t)std::ceil(std::sqrt((double)std::max<int64_t>(n, 1)));
    uint64_t above = 0;
    for (int b = (int)kCombClasses - 1; b >= 0; --b) {
        if (above + hist[b] > k) {
            // classes above b hold at most k: they form the class (if any)
            return above > 0 ? (uint32_t)std::min<uint64_t>(std::max<uint64_t>(comb_class_min((uint32_t)b + 1), kCombMinDegree), 65535u)
                             : (uint32_t)std::min<uint64_t>(std::max<uint64_t>(comb_class_min((uint32_t)b), kCombMinDegree), 65535u);
        }
        above += hist[b];
    }
    return above > 0 ? kCombMinDegree : 0u;  // every vertex of degree >= 64 fits
}

__global__ void comb_cols_kernel(const int32_t* cols, int64_t m, const uint32_t* tag, uint32_t* out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        out[e] = tag[cols[e]];
}

__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Residue combining set-up of one call (stream-ordered, kernels only): pick
// the combined vertices among `sc`, give them slots and write the tagged copy
// of the column array.  Returns the slot vertices and the tagged columns.
template <class OffT>
atos_status comb_setup(const GraphRec& g, const Layout& L, char* ws, CombScope sc, hipStream_t s,
                       uint32_t** cvert_out, const int32_t** ccols_out) {
    constexpr uint32_t CS = PrCombApp::kCombSlots;
    WsHeader* H = (WsHeader*)ws;
    uint32_t* tag = (uint32_t*)(ws + L.comb_tag);
    uint32_t* cvert = (uint32_t*)(ws + L.comb_vertex);
    uint32_t* hist = (uint32_t*)(ws + L.comb_hist);
    uint32_t* ccols = (uint32_t*)(ws + L.comb_cols);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(kCombClasses), 0, s, hist, (int64_t)kCombClasses, 0u);
    hipLaunchKernelGGL((comb_hist_kernel<OffT>), dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s,
                       (const OffT*)g.offs, g.n, sc, hist);
    hipLaunchKernelGGL(comb_pick_kernel, dim3(1), dim3(kCombClasses), 0, s, (const uint32_t*)hist, CS, H);
    hipLaunchKernelGGL((comb_slot_kernel<OffT>), dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s,
                       (const OffT*)g.offs, g.n, sc, H, CS, tag, cvert);
    if (g.m > 0)
        hipLaunchKernelGGL(comb_cols_kernel, dim3(init_grid(g.m, g.num_cu)), dim3(kInitBlock), 0, s,
                           g.cols, g.m, (const uint32_t*)tag, ccols);
    HIP_TRY(hipGetLastError());
    *cvert_out = cvert;
    *ccols_out = (const int32_t*)ccols;
    return ATOS_OK;
}

// One record of a level-synchronous run's level (trace attached): the level
// number, its frontier size with kTraceBspLevel set, the edges scanned by all
// earlier levels (low 32 bits) and the device clock when the level starts;
// the record after it marks its end.
__global__ void bsp_trace_kernel(TraceBuf* T, uint32_t level, uint32_t n_in, const uint64_t* edges) {
    const uint64_t r = add_agent(&T->count, (uint64_t)1);
    if (r >= T->capacity) return;
    TraceRec* R = &T->rec[r];
    R->t_begin = now_ticks();
    R->t_end = 0;
    R->worker = level;
    R->tasks = kTraceBspLevel | (n_in & ~kTraceBspLevel & ~kTraceHubChunk);
    R->edges = (uint32_t)ld_agent(edges);
    R->vertex = 0xFFFFFFFFu;
}

// Host-side record of a BSP run's counters, written into the header at the end.
__global__ void bsp_stats_kernel(WsHeader* H, uint64_t popped, uint64_t pushed, uint64_t rounds,
                                 uint32_t status) {
    H->stat_popped = popped;
    H->stat_pushed = pushed;
    H->stat_rounds = rounds;
    H->status = status;
}

// Discrete runs: before each round, the positions published so far become
// that round's work.
__global__ void set_limits_kernel(WsHeader* H) {
    for (uint32_t q = threadIdx.x; q < H->n_queues; q += blockDim.x) H->q[q].limit = H->q[q].tail;
}

__global__ void end_discrete_kernel(WsHeader* H, uint64_t rounds, uint32_t status_bits) {
    H->stat_rounds = rounds;
    H->status |= status_bits;
}

// Next launch of a run with Algorithm 4's sweep: the `n_init` vertices its
// clean sweep found become initial tasks, dealt round-robin over the rings at
// their tails (the previous launch ended with every reserved position taken,
// so each ring's head equals its tail), and the cursor starts again.
__global__ void reseed_kernel(WsHeader* H, uint32_t nq, uint64_t n_init) {
    for (uint32_t q = 0; q < nq; ++q) {
        QueueCtl* Q = &H->q[q];
        const uint64_t k = n_init / nq + (q < n_init % nq ? 1 : 0);
        Q->init_base = Q->tail;
        Q->n_init = k;
        Q->tail += k;
    }
    H->check_cursor = 0;
}

__global__ void reset_header_kernel(WsHeader* H) {
    H->status = 0u;
    H->stat_popped = H->stat_pushed = H->stat_edges = 0;
    H->stat_push_retries = H->stat_idle = H->stat_steals = 0;
    H->stat_comb_adds = H->stat_comb_atomics = 0;
    H->stat_rounds = 0;
    H->scalar_out = 0;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false;
    hipStream_t s;
    explicit Timer(bool enabled, hipStream_t st) : s(st) {
        if (enabled && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
            on = hipEventRecord(a, s) == hipSuccess;
        }
    }
    float stop() {
        float ms = 0.0f;
        if (on && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess)
            (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Events bracketing only the persistent worker kernel of a call.
struct KernelEvents {
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false;
    explicit KernelEvents(bool enabled) {
        if (enabled) on = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
    }
    void begin(hipStream_t s) {
        if (on) on = hipEventRecord(a, s) == hipSuccess;
    }
    void end(hipStream_t s) {
        if (on) on = hipEventRecord(b, s) == hipSuccess;
    }
    float ms() {
        float t = 0.0f;
        if (on && hipEventSynchronize(b) == hipSuccess) (void)hipEventElapsedTime(&t, a, b);
        return on ? t : -1.0f;
    }
    ~KernelEvents() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// ------------------------------------------------------------------ launch helpers
// Seed kernel, then the worker kernel; `ke` brackets the worker kernel alone.
// The attached per-batch trace buffer (atos_trace_attach) and its device.
std::mutex g_trace_mu;
TraceBuf* g_trace = nullptr;
int g_trace_device = -1;

TraceBuf* trace_for(int device) {
    std::lock_guard<std::mutex> lock(g_trace_mu);
    return g_trace_device == device ? g_trace : nullptr;
}

// Whether the host set the run's abort word (read between levels and rounds).
bool host_aborted(const Cfg& c) {
    return c.abort_flag != nullptr &&
           __atomic_load_n(c.abort_flag, __ATOMIC_ACQUIRE) != 0u;
}

// a level record of a traced level-synchronous run (no-op without a trace)
void bsp_trace(const GraphRec& g, WsHeader* H, uint64_t level, uint32_t n_in, hipStream_t s) {
    TraceBuf* T = trace_for(g.device);
    if (T)
        hipLaunchKernelGGL(bsp_trace_kernel, dim3(1), dim3(1), 0, s, T, (uint32_t)level, n_in,
                           (const uint64_t*)&H->stat_edges);
}

template <int B, class App, class OffT>
atos_status launch_persistent_b(const GraphRec& g, const Cfg& c, const App& app, WsHeader* H,
                                uint64_t* ring, uint64_t n_init, hipStream_t s, KernelEvents* ke) {
    auto kern = persistent_kernel<B, App, OffT>;
    const int grid = c.grid ? c.grid : occupancy(kern, B) * g.num_cu;
    PersistArgs<OffT> a;
    a.offs = (const OffT*)g.offs;
    a.cols = g.cols;
    a.n = g.n;
    a.hdr = H;
    a.rings = ring;
    a.log2cap = log2u(c.capacity);
    a.n_queues = c.n_queues;
    a.n_init = n_init;
    a.fetch = c.fetch;
    a.split_degree = c.split_degree;
    a.push_spin_limit = 200000;  // about 25 ms of s_sleep(2) before declaring overflow
    a.timeout_ticks = (uint64_t)c.timeout_ms * (uint64_t)g.clock_khz;
    // bulk claims only while a ring holds more than every worker could claim at once
    a.bulk_margin = (uint64_t)c.fetch * (uint64_t)grid;
    a.trace = trace_for(g.device);
    a.fetch_share = c.fetch_fixed ? 0u : (uint32_t)std::max<int>(1, grid / (int)c.n_queues);
    a.discrete = c.strategy == ATOS_DISCRETE ? 1u : c.strategy == ATOS_ROUNDS ? 2u : 0u;
    a.push_shallow = c.push_shallow ? 1u : 0u;
    a.segmented = c.segmented ? 1u : 0u;
    for (int b = 0; b < kMaxQueues - 1; ++b) a.seg_bound[b] = c.seg_bound[b];
    a.abort_flag = c.abort_flag;
    a.comb_flush_edges = c.comb_flush;
    if (n_init > 0)
        hipLaunchKernelGGL((seed_tasks_kernel<App, OffT>), dim3(init_grid((int64_t)n_init, g.num_cu)),
                           dim3(kInitBlock), 0, s, a, app);
    if (a.discrete == 2u)  // the first round: the initial tasks
        hipLaunchKernelGGL(set_limits_kernel, dim3(1), dim3(64), 0, s, H);
    if (ke) ke->begin(s);
    if (a.discrete != 1u) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(B), 0, s, a, app);
        if (ke) ke->end(s);
        return hipGetLastError() == hipSuccess ? ATOS_OK : ATOS_EHIP;
    }
    // Discrete kernels (paper section 3.4, the non-persistent strategy): the same
    // workers, one launch per round; a round takes the tasks published before it
    // and pushes the next round's.  The host reads the counters after each round
    // and stops when every reserved task is done, on a device error, or at the
    // deadline.
    const auto t0 = std::chrono::steady_clock::now();
    uint64_t rounds = 0;
    uint32_t status_bits = 0;
    QueueCtl q[kMaxQueues];
    for (;;) {
        hipLaunchKernelGGL(set_limits_kernel, dim3(1), dim3(64), 0, s, H);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(B), 0, s, a, app);
        ++rounds;
        uint32_t status = 0;
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(q, H->q, sizeof(q), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&status, &H->status, sizeof(status), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (status != 0u) break;
        if (host_aborted(c)) {
            status_bits = (uint32_t)kStatusAbort;
            break;
        }
        uint64_t d = 0, t = 0;
        for (uint32_t i = 0; i < c.n_queues; ++i) {
            d += q[i].done;
            t += q[i].tail;
        }
        if (d == t) break;
        if (t - d <= (uint64_t)c.discrete_tail) {
            // the few tasks left: one persistent launch finishes the run
            a.discrete = 0u;
            hipLaunchKernelGGL(kern, dim3(grid), dim3(B), 0, s, a, app);
            ++rounds;
            HIP_TRY(hipGetLastError());
            break;
        }
        const auto ms = std::chrono::duration_cast<std::chrono::milliseconds>(
            std::chrono::steady_clock::now() - t0).count();
        if ((uint64_t)ms > (uint64_t)c.timeout_ms) {
            status_bits = (uint32_t)kStatusTimeout;
            break;
        }
    }
    if (ke) ke->end(s);
    hipLaunchKernelGGL(end_discrete_kernel, dim3(1), dim3(1), 0, s, H, rounds, status_bits);
    return hipGetLastError() == hipSuccess ? ATOS_OK : ATOS_EHIP;
}

template <class App, class OffT>
atos_status launch_persistent(const GraphRec& g, const Cfg& c, const App& app, WsHeader* H,
                              uint64_t* ring, uint64_t n_init, hipStream_t s,
                              KernelEvents* ke = nullptr) {
    switch (c.worker) {
        case 64: return launch_persistent_b<64, App, OffT>(g, c, app, H, ring, n_init, s, ke);
        case 128: return launch_persistent_b<128, App, OffT>(g, c, app, H, ring, n_init, s, ke);
        case 256: return launch_persistent_b<256, App, OffT>(g, c, app, H, ring, n_init, s, ke);
        case 512: return launch_persistent_b<512, App, OffT>(g, c, app, H, ring, n_init, s, ke);
        case 1024: return launch_persistent_b<1024, App, OffT>(g, c, app, H, ring, n_init, s, ke);
        default: return ATOS_EINVAL;
    }
}

template <int B, class App, class OffT>
atos_status launch_frontier_b(const GraphRec& g, const App& app, const uint32_t* in, uint32_t n_in,
                              uint32_t* out, uint32_t* out_count, uint64_t* edges, hipStream_t s) {
    if (n_in == 0) return ATOS_OK;
    FrontierArgs<OffT> a;
    a.offs = (const OffT*)g.offs;
    a.cols = g.cols;
    a.in = in;
    a.n_in = n_in;
    a.out = out;
    a.out_count = out_count;
    a.edges = edges;
    const uint32_t grid = (n_in + B - 1) / B;
    hipLaunchKernelGGL((frontier_kernel<B, App, OffT>), dim3(grid), dim3(B), 0, s, a, app);
    return hipGetLastError() == hipSuccess ? ATOS_OK : ATOS_EHIP;
}

template <class App, class OffT>
atos_status launch_frontier(const GraphRec& g, int worker, const App& app, const uint32_t* in,
                            uint32_t n_in, uint32_t* out, uint32_t* out_count, uint64_t* edges,
                            hipStream_t s) {
    switch (worker) {
        case 64: return launch_frontier_b<64, App, OffT>(g, app, in, n_in, out, out_count, edges, s);
        case 128: return launch_frontier_b<128, App, OffT>(g, app, in, n_in, out, out_count, edges, s);
        case 256: return launch_frontier_b<256, App, OffT>(g, app, in, n_in, out, out_count, edges, s);
        case 512: return launch_frontier_b<512, App, OffT>(g, app, in, n_in, out, out_count, edges, s);
        case 1024: return launch_frontier_b<1024, App, OffT>(g, app, in, n_in, out, out_count, edges, s);
        default: return ATOS_EINVAL;
    }
}

// ------------------------------------------------------------------ run bracket
atos_status status_from_bits(uint32_t bits) {
    if (bits & kStatusCorrupt) return ATOS_EHIP;
    if (bits & kStatusOverflow) return ATOS_EOVERFLOW;
    if (bits & kStatusTimeout) return ATOS_ETIMEOUT;
    if (bits & kStatusAbort) return ATOS_EABORTED;
    return ATOS_OK;
}

atos_status read_stats(const void* d_ws, hipStream_t s, atos_stats* st) {
    WsHeader h;
    HIP_TRY(hipMemcpyAsync(&h, d_ws, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    st->status = (int32_t)status_from_bits(h.status);
    st->reserved0 = 0;
    st->tasks_popped = h.stat_popped;
    st->tasks_pushed = h.stat_pushed;
    st->edges_scanned = h.stat_edges;
    st->rounds = h.stat_rounds;
    st->kernel_ms = 0.0f;
    st->push_retries = h.stat_push_retries;
    st->hub_posts = h.stat_hub_posts;
    st->combined_updates = h.stat_comb_adds;
    st->combine_atomics = h.stat_comb_atomics;
    st->idle_iterations = h.stat_idle;
    st->steals = h.stat_steals;
    return ATOS_OK;
}

atos_status finish_call(atos_status launched, Timer& tm, KernelEvents& ke, const void* d_ws,
                        hipStream_t s, atos_stats* st) {
    if (launched != ATOS_OK) return launched;
    if (!st) return ATOS_OK;
    const float ms = tm.stop();
    atos_status r = read_stats(d_ws, s, st);
    st->device_ms = ms;
    const float kms = ke.ms();
    st->kernel_ms = kms >= 0.0f ? kms : ms;
    return r;
}

atos_status check_common(atos_graph_t g, int app, void* d_ws, size_t ws_bytes,
                         const atos_config* cfg, Cfg& c, Layout& L) {
    if (!g || !d_ws) return ATOS_EINVAL;
    if (((uintptr_t)d_ws & 255u) != 0u) return ATOS_EINVAL;
    atos_status r = resolve_cfg(g->r, app, cfg, c);
    if (r != ATOS_OK) return r;
    if (c.segmented) return ATOS_EUNSUPPORTED;  // a batch layout
    L = layout(g->r, app, c);
    if (ws_bytes < L.total) return ATOS_ENOMEM;
    return ATOS_OK;
}

// ------------------------------------------------------------------ BFS
template <class OffT>
atos_status run_bfs(KernelEvents& ke, const GraphRec& g, const Cfg& c, const Layout& L, int64_t source,
                    int32_t* d_depth, char* ws, hipStream_t s) {
    WsHeader* H = (WsHeader*)ws;
    uint32_t* depth = (uint32_t*)d_depth;
    if (c.strategy != ATOS_BSP) {
        uint64_t* ring = (uint64_t*)(ws + L.ring);
        hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(64), 0, s, H, c.capacity, c.n_queues, (uint64_t)1);
        hipLaunchKernelGGL(bfs_init_kernel, dim3(init_grid(std::max<int64_t>(g.n, (int64_t)(c.capacity * c.n_queues)), g.num_cu)),
                           dim3(kInitBlock), 0, s, (const WsHeader*)H, ring, c.capacity * c.n_queues, depth, g.n,
                           source);
        HIP_TRY(hipGetLastError());
        BfsApp app{depth, (uint32_t)source};
        atos_status r = launch_persistent<BfsApp, OffT>(g, c, app, H, ring, 1, s, &ke);
        return r;
    }
    // Algorithm 1: one frontier expansion per level, host-synchronised.
    uint32_t* fa = (uint32_t*)(ws + L.front_a);
    uint32_t* fb = (uint32_t*)(ws + L.front_b);
    uint32_t* count = &H->bsp_count;
    hipLaunchKernelGGL(reset_header_kernel, dim3(1), dim3(1), 0, s, H);
    hipLaunchKernelGGL(bfs_init_kernel, dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s,
                       (const WsHeader*)H, (uint64_t*)nullptr, (uint64_t)0, depth, g.n, source);
    hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(1), 0, s, fa, (uint32_t)source);
    HIP_TRY(hipGetLastError());
    uint32_t n_in = 1;
    uint64_t popped = 0, pushed = 0, rounds = 0;
    BspBfs app{depth};
    uint32_t bits = 0;
    while (n_in > 0) {
        if (host_aborted(c)) {
            bits = (uint32_t)kStatusAbort;
            break;
        }
        bsp_trace(g, H, rounds, n_in, s);
        HIP_TRY(hipMemsetAsync(count, 0, sizeof(uint32_t), s));
        atos_status r = launch_frontier<BspBfs, OffT>(g, c.worker, app, fa, n_in, fb, count, &H->stat_edges, s);
        if (r != ATOS_OK) return r;
        uint32_t n_out = 0;
        HIP_TRY(hipMemcpyAsync(&n_out, count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        popped += n_in;
        pushed += n_out;
        ++rounds;
        std::swap(fa, fb);
        n_in = n_out;
    }
    bsp_trace(g, H, rounds, 0u, s);
    hipLaunchKernelGGL(bsp_stats_kernel, dim3(1), dim3(1), 0, s, H, popped, pushed, rounds, bits);
    HIP_TRY(hipGetLastError());
    return ATOS_OK;
}

// ------------------------------------------------------------------ PageRank
// Algorithm 4 as printed: every vertex starts queued; a task pushes its
// residue without enqueueing anyone, then sweeps Check_Size positions of the
// round-robin cursor and enqueues what it finds above eps.  The paper leaves
// the end of the sweep open ("while not frontier.empty()" can hold while some
// residue > eps sits behind the cursor): when a launch's worklist has drained,
// a clean sweep of every vertex collects the residues still above eps and
// they start the next launch; the run ends when the clean sweep finds none.
// stats.rounds counts the launches.
template <class OffT>
atos_status pagerank_sweep(KernelEvents& ke, const GraphRec& g, const Cfg& c, const Layout& L,
                           double d, double e, double* rank64, double* residue, WsHeader* H,
                           uint64_t* ring, char* ws, hipStream_t s) {
    uint32_t* list = (uint32_t*)(ws + L.front_a);
    uint32_t* queued = (uint32_t*)(ws + L.queued);
    uint32_t* count = &H->bsp_count;
    PrSweepApp app{rank64, residue, queued, d, e, nullptr, (uint32_t)c.check_size};
    // residue combining: the tagged column array is read by every launch
    GraphRec gc = g;
    PrSweepCombApp capp;
    if (c.comb_flush != 0) {
        uint32_t* cvert = nullptr;
        const int32_t* ccols = nullptr;
        atos_status rs = comb_setup<OffT>(g, L, ws, CombScope{nullptr, nullptr, nullptr, 0u}, s,
                                          &cvert, &ccols);
        if (rs != ATOS_OK) return rs;
        gc.cols = ccols;
        capp.comb_vertex = cvert;
        capp.comb = nullptr;  // the worker's LDS table, set by the kernel
    }
    // every vertex starts queued (Algorithm 3's initial frontier)
    hipLaunchKernelGGL(fill_u32_kernel, dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s,
                       queued, g.n, 1u);
    const auto t0 = std::chrono::steady_clock::now();
    uint64_t n_init = (uint64_t)g.n, launches = 0;
    uint32_t status_bits = 0;
    ke.begin(s);
    for (;;) {
        atos_status r;
        if (c.comb_flush != 0) {
            static_cast<PrSweepApp&>(capp) = app;
            r = launch_persistent<PrSweepCombApp, OffT>(gc, c, capp, H, ring, n_init, s, nullptr);
        } else {
            r = launch_persistent<PrSweepApp, OffT>(g, c, app, H, ring, n_init, s, nullptr);
        }
        if (r != ATOS_OK) return r;
        ++launches;
        hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(1), 0, s, count, 0u);
        hipLaunchKernelGGL(pr_filter_kernel, dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s,
                           (const double*)residue, g.n, e, list, count);
        HIP_TRY(hipGetLastError());
        uint32_t found = 0, status = 0;
        HIP_TRY(hipMemcpyAsync(&found, count, sizeof(found), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(&status, &H->status, sizeof(status), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (status != 0u || found == 0u) break;
        if (host_aborted(c)) {
            status_bits = (uint32_t)kStatusAbort;
            break;
        }
        const auto ms = std::chrono::duration_cast<std::chrono::milliseconds>(
            std::chrono::steady_clock::now() - t0).count();
        if ((uint64_t)ms > (uint64_t)c.timeout_ms) {
            status_bits = (uint32_t)kStatusTimeout;
            break;
        }
        hipLaunchKernelGGL(reseed_kernel, dim3(1), dim3(1), 0, s, H, c.n_queues, (uint64_t)found);
        app.list = list;
        n_init = found;
    }
    ke.end(s);
    hipLaunchKernelGGL(end_discrete_kernel, dim3(1), dim3(1), 0, s, H, launches, status_bits);
    return hipGetLastError() == hipSuccess ? ATOS_OK : ATOS_EHIP;
}

template <class OffT>
atos_status run_pagerank(KernelEvents& ke, const GraphRec& g, const Cfg& c, const Layout& L, float damping,
                         float eps, int64_t source, float* rank, float* residual_out, char* ws,
                         hipStream_t s) {
    WsHeader* H = (WsHeader*)ws;
    double* inv_deg = (double*)(ws + L.inv_deg);
    double* residue = (double*)(ws + L.residue);
    double* rank64 = (double*)(ws + L.rank64);
    const double d = (double)damping, e = (double)eps;
    const double coef = (1.0 - d) * d;
    const int out_grid = init_grid(g.n, g.num_cu);
    const int pull_grid = init_grid((g.m + 31) / 32, g.num_cu);
    if (c.strategy != ATOS_BSP) {
        uint64_t* ring = (uint64_t*)(ws + L.ring);
        if ((uint64_t)g.n > c.capacity * c.n_queues) return ATOS_EINVAL;
        if (c.comb_flush != 0 && source >= 0) return ATOS_EUNSUPPORTED;  // whole-graph PageRank only
        const uint64_t n_init = source < 0 ? (uint64_t)g.n : 1ull;
        hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(64), 0, s, H, c.capacity, c.n_queues, n_init);
        hipLaunchKernelGGL((pr_init_kernel<OffT>), dim3(init_grid(std::max<int64_t>(g.n, (int64_t)(c.capacity * c.n_queues)), g.num_cu)),
                           dim3(kInitBlock), 0, s, (const WsHeader*)H, ring, c.capacity * c.n_queues,
                           (const OffT*)g.offs, g.n, d, source, rank64, residue, inv_deg);
        if (g.m > 0 && source < 0)
            hipLaunchKernelGGL((pr_pull_kernel<OffT>), dim3(pull_grid), dim3(kInitBlock), 0, s,
                               (const OffT*)g.offs, g.cols, g.n, g.m, coef, (const double*)inv_deg, residue);
        HIP_TRY(hipGetLastError());
        if (c.check_size > 0) {
            atos_status r = pagerank_sweep<OffT>(ke, g, c, L, d, e, rank64, residue, H, ring, ws, s);
            if (r != ATOS_OK) return r;
        } else if (c.comb_flush != 0) {
            // the combined vertices, their slots and the tagged column array
            uint32_t* cvert = nullptr;
            const int32_t* ccols = nullptr;
            atos_status rs = comb_setup<OffT>(g, L, ws, CombScope{nullptr, nullptr, nullptr, 0u}, s,
                                              &cvert, &ccols);
            if (rs != ATOS_OK) return rs;
            GraphRec gc = g;
            gc.cols = ccols;
            PrCombApp app;
            app.rank = rank64;
            app.residue = residue;
            app.damping = d;
            app.eps = e;
            app.first = 0u;
            app.comb_vertex = cvert;
            app.comb = nullptr;  // the worker's LDS table, set by the kernel
            atos_status r = launch_persistent<PrCombApp, OffT>(gc, c, app, H, ring, n_init, s, &ke);
            if (r != ATOS_OK) return r;
        } else {
            PrApp app{rank64, residue, d, e, source < 0 ? 0u : (uint32_t)source};
            atos_status r = launch_persistent<PrApp, OffT>(g, c, app, H, ring, n_init, s, &ke);
            if (r != ATOS_OK) return r;
        }
        hipLaunchKernelGGL(rank_out_kernel, dim3(out_grid), dim3(kInitBlock), 0, s,
                           (const double*)rank64, (const double*)residue, g.n, rank, residual_out);
        HIP_TRY(hipGetLastError());
        return ATOS_OK;
    }
    // Algorithm 3: push round over the frontier, then the residue > eps filter.
    uint32_t* fa = (uint32_t*)(ws + L.front_a);
    uint32_t* fb = (uint32_t*)(ws + L.front_b);
    uint32_t* count = &H->bsp_count;
    hipLaunchKernelGGL(reset_header_kernel, dim3(1), dim3(1), 0, s, H);
    hipLaunchKernelGGL((pr_init_kernel<OffT>), dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s,
                       (const WsHeader*)H, (uint64_t*)nullptr, (uint64_t)0, (const OffT*)g.offs, g.n,
                       d, source, rank64, residue, inv_deg);
    uint32_t n_in;
    if (source < 0) {
        if (g.m > 0)
            hipLaunchKernelGGL((pr_pull_kernel<OffT>), dim3(pull_grid), dim3(kInitBlock), 0, s,
                               (const OffT*)g.offs, g.cols, g.n, g.m, coef, (const double*)inv_deg, residue);
        hipLaunchKernelGGL(iota_kernel, dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s, fa, g.n);
        n_in = (uint32_t)g.n;
    } else {
        hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(1), 0, s, fa, (uint32_t)source);
        n_in = 1;
    }
    HIP_TRY(hipGetLastError());
    uint64_t popped = 0, pushed = 0, rounds = 0;
    BspPrPush app{rank64, residue, d};
    const int filt_grid = init_grid(g.n, g.num_cu);
    const uint64_t deadline_rounds = 1000000;
    bool aborted = false;
    while (n_in > 0 && rounds < deadline_rounds) {
        if (host_aborted(c)) {
            aborted = true;
            break;
        }
        bsp_trace(g, H, rounds, n_in, s);
        atos_status r = launch_frontier<BspPrPush, OffT>(g, c.worker, app, fa, n_in, nullptr, nullptr, &H->stat_edges, s);
        if (r != ATOS_OK) return r;
        HIP_TRY(hipMemsetAsync(count, 0, sizeof(uint32_t), s));
        hipLaunchKernelGGL(pr_filter_kernel, dim3(filt_grid), dim3(kInitBlock), 0, s,
                           (const double*)residue, g.n, e, fb, count);
        HIP_TRY(hipGetLastError());
        uint32_t n_out = 0;
        HIP_TRY(hipMemcpyAsync(&n_out, count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        popped += n_in;
        pushed += n_out;
        ++rounds;
        std::swap(fa, fb);
        n_in = n_out;
    }
    bsp_trace(g, H, rounds, 0u, s);
    hipLaunchKernelGGL(bsp_stats_kernel, dim3(1), dim3(1), 0, s, H, popped, pushed, rounds,
                       aborted ? (uint32_t)kStatusAbort : n_in == 0 ? 0u : (uint32_t)kStatusTimeout);
    hipLaunchKernelGGL(rank_out_kernel, dim3(out_grid), dim3(kInitBlock), 0, s,
                       (const double*)rank64, (const double*)residue, g.n, rank, residual_out);
    HIP_TRY(hipGetLastError());
    return ATOS_OK;
}

// ------------------------------------------------------------------ colouring
template <class OffT>
atos_status run_color(KernelEvents& ke, const GraphRec& g, const Cfg& c, const Layout& L, uint64_t seed,
                      int32_t* color, int32_t* n_colors, char* ws, hipStream_t s) {
    WsHeader* H = (WsHeader*)ws;
    uint32_t* queued = (uint32_t*)(ws + L.queued);
    uint32_t* key = (uint32_t*)(ws + L.key);
    uint32_t* wait = (uint32_t*)(ws + L.wait);
    uint64_t* mask = (uint64_t*)(ws + L.mask);
    const int wait_grid = init_grid((g.m + 31) / 32, g.num_cu);
    if (c.strategy != ATOS_BSP) {
        uint64_t* ring = (uint64_t*)(ws + L.ring);
        if ((uint64_t)g.n > c.capacity * c.n_queues) return ATOS_EINVAL;
        hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(64), 0, s, H, c.capacity, c.n_queues, (uint64_t)g.n);
        hipLaunchKernelGGL((gc_init_kernel<OffT>), dim3(init_grid(std::max<int64_t>(g.n, (int64_t)(c.capacity * c.n_queues)), g.num_cu)),
                           dim3(kInitBlock), 0, s, (const WsHeader*)H, ring, c.capacity * c.n_queues,
                           (const OffT*)g.offs, g.n, seed, 1u, color, queued, key, wait, mask);
        if (g.m > 0 && c.order_degree)
            hipLaunchKernelGGL((gc_wait_kernel<OffT>), dim3(wait_grid), dim3(kInitBlock), 0, s,
                               (const OffT*)g.offs, g.cols, g.n, g.m, (const uint32_t*)key,
                               c.order_degree, wait);
        HIP_TRY(hipGetLastError());
        GcApp app{color, queued, key, wait, mask, c.order_degree, c.forbid_all};
        atos_status r = launch_persistent<GcApp, OffT>(g, c, app, H, ring, (uint64_t)g.n, s, &ke);
        if (r != ATOS_OK) return r;
    } else {
        // Algorithm 5: assign kernel, then conflict kernel, per round.
        uint32_t* fa = (uint32_t*)(ws + L.front_a);
        uint32_t* fb = (uint32_t*)(ws + L.front_b);
        uint32_t* count = &H->bsp_count;
        hipLaunchKernelGGL(reset_header_kernel, dim3(1), dim3(1), 0, s, H);
        hipLaunchKernelGGL((gc_init_kernel<OffT>), dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s,
                           (const WsHeader*)H, (uint64_t*)nullptr, (uint64_t)0, (const OffT*)g.offs,
                           g.n, seed, 0u, color, queued, key, wait, (uint64_t*)nullptr);
        if (g.m > 0 && c.order_degree)
            hipLaunchKernelGGL((gc_wait_kernel<OffT>), dim3(wait_grid), dim3(kInitBlock), 0, s,
                               (const OffT*)g.offs, g.cols, g.n, g.m, (const uint32_t*)key,
                               c.order_degree, wait);
        hipLaunchKernelGGL(iota_kernel, dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s, fa, g.n);
        HIP_TRY(hipGetLastError());
        uint32_t n_in = (uint32_t)g.n;
        uint64_t popped = 0, pushed = 0, rounds = 0;
        BspGcAssign assign{color, key, queued, wait, c.order_degree, c.forbid_all};
        BspGcCheck check{color, key, queued, wait, c.order_degree};
        uint32_t bits = 0;
        while (n_in > 0) {
            if (host_aborted(c)) {
                bits = (uint32_t)kStatusAbort;
                break;
            }
            bsp_trace(g, H, rounds, n_in, s);
            atos_status r = launch_frontier<BspGcAssign, OffT>(g, c.worker, assign, fa, n_in, nullptr, nullptr, &H->stat_edges, s);
            if (r != ATOS_OK) return r;
            HIP_TRY(hipMemsetAsync(count, 0, sizeof(uint32_t), s));
            r = launch_frontier<BspGcCheck, OffT>(g, c.worker, check, fa, n_in, fb, count, &H->stat_edges, s);
            if (r != ATOS_OK) return r;
            uint32_t n_out = 0;
            HIP_TRY(hipMemcpyAsync(&n_out, count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            popped += n_in;
            pushed += n_out;
            ++rounds;
            std::swap(fa, fb);
            n_in = n_out;
        }
        bsp_trace(g, H, rounds, 0u, s);
        hipLaunchKernelGGL(bsp_stats_kernel, dim3(1), dim3(1), 0, s, H, popped, pushed, rounds, bits);
    }
    hipLaunchKernelGGL(color_count_kernel, dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock), 0, s,
                       (const int32_t*)color, g.n, H, n_colors);
    if (n_colors) hipLaunchKernelGGL(copy_scalar_kernel, dim3(1), dim3(1), 0, s, (const WsHeader*)H, n_colors);
    HIP_TRY(hipGetLastError());
    return ATOS_OK;
}


// ------------------------------------------------------------------ batching
// Device tables of a batch plan (one allocation, laid out by BatchLayout).
struct BatchLayout {
    size_t bfs_src = 0, pr_begin = 0, pr_prefix = 0, pr_edge_begin = 0, pr_edge_prefix = 0,
           inst_begin = 0, inst_end = 0, inst_kind = 0, inst_src = 0, bad = 0, total = 0;
};

BatchLayout batch_layout(size_t n_inst, size_t n_bfs, size_t n_pr) {
    BatchLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    L.bfs_src = take(std::max<size_t>(n_bfs, 1) * 4);
    L.pr_begin = take(std::max<size_t>(n_pr, 1) * 4);
    L.pr_prefix = take((n_pr + 1) * 8);
    L.pr_edge_begin = take(std::max<size_t>(n_pr, 1) * 8);
    L.pr_edge_prefix = take((n_pr + 1) * 8);
    L.inst_begin = take(std::max<size_t>(n_inst, 1) * 8);
    L.inst_end = take(std::max<size_t>(n_inst, 1) * 8);
    L.inst_kind = take(std::max<size_t>(n_inst, 1) * 4);
    L.inst_src = take(std::max<size_t>(n_inst, 1) * 8);
    L.bad = take(8);
    L.total = off;
    return L;
}

// instance containing v, or -1 (instances sorted by begin, disjoint)
__device__ inline int64_t find_instance(const int64_t* ib, const int64_t* ie, uint32_t n_inst,
                                        int64_t v) {
    if (n_inst == 0 || v < ib[0]) return -1;
    uint32_t lo = 0, hi = n_inst;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ib[mid] <= v) lo = mid; else hi = mid;
    }
    return v < ie[lo] ? (int64_t)lo : -1;
}

__device__ inline bool comb_candidate(const CombScope& sc, int64_t v) {
    if (sc.ib == nullptr) return true;
    const int64_t k = find_instance(sc.ib, sc.ie, sc.n_inst, v);
    return k >= 0 && sc.kind[k] == (uint32_t)ATOS_APP_PAGERANK;
}

// Every edge of an instance's vertices must stay inside the instance.
template <class OffT>
__global__ void batch_validate_kernel(const OffT* offs, const int32_t* cols, int64_t n,
                                      const int64_t* ib, const int64_t* ie, uint32_t n_inst,
                                      uint32_t* bad) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = find_instance(ib, ie, n_inst, v);
        if (k < 0) continue;
        for (OffT e = offs[v]; e < offs[v + 1]; ++e) {
            const int64_t w = cols[e];
            if (w < ib[k] || w >= ie[k]) atomicOr(bad, 1u);
        }
    }
}

// Per-vertex state of a batch: BFS depths, PageRank rank = 1-d (FP64), residue 0, 1/deg.
template <class OffT>
__global__ void batch_init_kernel(const WsHeader* H, uint64_t* ring, uint64_t cap, const OffT* offs,
                                  int64_t n, const int64_t* ib, const int64_t* ie,
                                  const uint32_t* kind, const int64_t* src, uint32_t n_inst,
                                  double damping, uint32_t* state, double* rank, double* residue,
                                  double* inv_deg) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t v = i0; v < n; v += stride) {
        const int64_t k = find_instance(ib, ie, n_inst, v);
        if (k < 0) continue;
        if (kind[k] == (uint32_t)ATOS_APP_BFS) {
            state[v] = v == src[k] ? 0u : 0xFFFFFFFFu;
        } else {
            const int64_t d = (int64_t)(offs[v + 1] - offs[v]);
            rank[v] = 1.0 - damping;
            residue[v] = 0.0;
            inv_deg[v] = d > 0 ? 1.0 / (double)d : 0.0;
        }
    }
    maybe_zero_ring(H, ring, cap, i0, stride);
}

// End of a batch: FP32 rank bits of PageRank vertices into `state`, and their
// residues into `res_out` when asked for.
__global__ void batch_rank_out_kernel(const double* rank, const double* residue, int64_t n,
                                      const int64_t* ib, const int64_t* ie, const uint32_t* kind,
                                      uint32_t n_inst, uint32_t* state, float* res_out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = find_instance(ib, ie, n_inst, v);
        if (k >= 0 && kind[k] == (uint32_t)ATOS_APP_PAGERANK) {
            state[v] = __float_as_uint((float)rank[v]);
            if (res_out) res_out[v] = (float)residue[v];
        }
    }
}

// PageRank residue initialisation over the PageRank instances' edge ranges
// only (the concatenation of [pr_edge_begin[k], + size_k)), edge-balanced as
// in pr_pull_kernel.
template <class OffT>
__global__ void batch_pull_kernel(const OffT* offs, const int32_t* cols, int64_t n,
                                  const uint64_t* ebeg, const uint64_t* epre, uint32_t n_pr,
                                  double coef, const double* inv_deg, double* residue) {
    constexpr uint64_t kRun = 32;
    const uint64_t total = epre[n_pr];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t * kRun < total; t += stride) {
        const uint64_t j0 = t * kRun, j1 = std::min(total, j0 + kRun);
        uint32_t lo = 0, hi = n_pr;  // range holding j0
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (epre[mid] <= j0) lo = mid; else hi = mid;
        }
        uint32_t k = lo;
        int64_t v = -1, vend = 0;
        double acc = 0.0;
        for (uint64_t j = j0; j < j1; ++j) {
            bool jumped = v < 0;
            while (j >= epre[k + 1]) {
                ++k;
                jumped = true;
            }
            const int64_t e = (int64_t)(ebeg[k] + (j - epre[k]));
            if (jumped) {  // entered a PageRank range: locate the vertex holding e
                if (v >= 0 && acc != 0.0) atomicAdd(residue + v, coef * acc);
                acc = 0.0;
                int64_t a = 0, b = n;
                while (b - a > 1) {
                    const int64_t mid = (a + b) >> 1;
                    if ((int64_t)offs[mid] <= e) a = mid; else b = mid;
                }
                v = a;
                vend = (int64_t)offs[v + 1];
            }
            while (e >= vend) {  // consecutive edges of one range: advance vertex by vertex
                if (acc != 0.0) atomicAdd(residue + v, coef * acc);
                acc = 0.0;
                ++v;
                vend = (int64_t)offs[v + 1];
            }
            acc += inv_deg[cols[e]];
        }
        if (v >= 0 && acc != 0.0) atomicAdd(residue + v, coef * acc);
    }
}

}  // namespace

struct atos_batch {
    atos_graph_t g;
    std::vector<atos_batch_instance> inst;
    float damping, eps;
    Cfg cfg;
    BatchLayout L;
    char* d_tab;
    uint32_t n_bfs, n_pr;
    uint64_t n_init, pr_edges;
};

// Segments of a batch (ATOS_QUEUE_SEGMENTED): boundaries at instance starts,
// each the first instance start at or past k*n/8, so that every instance
// lies in one segment and the segments hold about n/8 vertices each.
static void segment_bounds(const atos_batch* b, Cfg& c) {
    const uint64_t n = (uint64_t)b->g->r.n;
    size_t i = 0;
    for (int k = 1; k < kMaxQueues; ++k) {
        const uint64_t target = n * (uint64_t)k / kMaxQueues;
        while (i < b->inst.size() && (uint64_t)b->inst[i].vertex_begin < target) ++i;
        c.seg_bound[k - 1] = i < b->inst.size() ? (uint32_t)b->inst[i].vertex_begin : 0xFFFFFFFFu;
    }
}

struct atos_exec {
    hipGraphExec_t exec;
};

namespace {

Layout batch_ws_layout(const atos_batch* b) {
    Layout L;
    size_t off = align_up(sizeof(WsHeader), 4096);
    const size_t n4 = align_up((size_t)std::max<int64_t>(b->g->r.n, 1) * 4, 256);
    L.ring = off;
    off += align_up((size_t)b->cfg.capacity * 8 * b->cfg.n_queues, 256);
    L.inv_deg = off;  // FP64 1/deg, residue and rank
    off += 2 * n4;
    L.residue = off;
    off += 2 * n4;
    L.rank64 = off;
    off += 2 * n4;
    if (b->n_pr > 0) {
        // residue combining of the PageRank instances (used when the batch's
        // configuration asks for it; kept whatever the configuration, so that
        // atos_batch_set_config can switch it on and off)
        L.comb_tag = off;
        off += n4;
        L.comb_vertex = off;
        off += align_up((size_t)PrCombApp::kCombSlots * 4, 256);
        L.comb_hist = off;
        off += align_up((size_t)kCombClasses * 4, 256);
        L.comb_cols = off;
        off += align_up((size_t)std::max<int64_t>(b->g->r.m, 1) * 4, 256);
    }
    L.total = off;
    return L;
}

template <class OffT>
atos_status run_batch(KernelEvents& ke, const atos_batch* b, const Layout& L, uint32_t* state,
                      float* residual_out, char* ws, hipStream_t s) {
    const GraphRec& g = b->g->r;
    const Cfg& c = b->cfg;
    WsHeader* H = (WsHeader*)ws;
    uint64_t* ring = (uint64_t*)(ws + L.ring);
    double* inv_deg = (double*)(ws + L.inv_deg);
    double* residue = (double*)(ws + L.residue);
    double* rank64 = (double*)(ws + L.rank64);
    const double damping = (double)b->damping;
    const char* T = b->d_tab;
    const BatchLayout& BL = b->L;
    const uint32_t n_inst = (uint32_t)b->inst.size();
    hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(64), 0, s, H, c.capacity, c.n_queues, b->n_init);
    hipLaunchKernelGGL((batch_init_kernel<OffT>),
                       dim3(init_grid(std::max<int64_t>(g.n, (int64_t)(c.capacity * c.n_queues)), g.num_cu)),
                       dim3(kInitBlock), 0, s, (const WsHeader*)H, ring, c.capacity * c.n_queues,
                       (const OffT*)g.offs, g.n, (const int64_t*)(T + BL.inst_begin),
                       (const int64_t*)(T + BL.inst_end), (const uint32_t*)(T + BL.inst_kind),
                       (const int64_t*)(T + BL.inst_src), n_inst, damping, state, rank64,
                       residue, inv_deg);
    if (b->pr_edges > 0)
        hipLaunchKernelGGL((batch_pull_kernel<OffT>),
                           dim3(init_grid((int64_t)((b->pr_edges + 31) / 32), g.num_cu)),
                           dim3(kInitBlock), 0, s, (const OffT*)g.offs, g.cols, g.n,
                           (const uint64_t*)(T + BL.pr_edge_begin),
                           (const uint64_t*)(T + BL.pr_edge_prefix), b->n_pr,
                           (1.0 - damping) * damping, (const double*)inv_deg, residue);
    HIP_TRY(hipGetLastError());
    BatchTables t;
    t.bfs_src = (const uint32_t*)(T + BL.bfs_src);
    t.pr_prefix = (const uint64_t*)(T + BL.pr_prefix);
    t.pr_begin = (const uint32_t*)(T + BL.pr_begin);
    t.n_bfs = b->n_bfs;
    t.n_pr = b->n_pr;
    BatchApp app{state, rank64, residue, damping, (double)b->eps, t};
    atos_status r;
    if (c.comb_flush != 0 && b->n_pr > 0) {
        // the PageRank instances' combined vertices, their slots, and the column
        // array with their entries tagged (BFS instances' entries unchanged)
        const CombScope pr{(const int64_t*)(T + BL.inst_begin), (const int64_t*)(T + BL.inst_end),
                           (const uint32_t*)(T + BL.inst_kind), n_inst};
        uint32_t* cvert = nullptr;
        const int32_t* ccols = nullptr;
        atos_status rs = comb_setup<OffT>(g, L, ws, pr, s, &cvert, &ccols);
        if (rs != ATOS_OK) return rs;
        GraphRec gc = g;
        gc.cols = ccols;
        BatchCombApp capp;
        static_cast<BatchApp&>(capp) = app;
        capp.comb_vertex = cvert;
        capp.comb = nullptr;  // the worker's LDS table, set by the kernel
        r = launch_persistent<BatchCombApp, OffT>(gc, c, capp, H, ring, b->n_init, s, &ke);
    } else {
        r = launch_persistent<BatchApp, OffT>(g, c, app, H, ring, b->n_init, s, &ke);
    }
    if (r != ATOS_OK) return r;
    if (b->n_pr > 0) {
        hipLaunchKernelGGL(batch_rank_out_kernel, dim3(init_grid(g.n, g.num_cu)), dim3(kInitBlock),
                           0, s, (const double*)rank64, (const double*)residue, g.n,
                           (const int64_t*)(T + BL.inst_begin), (const int64_t*)(T + BL.inst_end),
                           (const uint32_t*)(T + BL.inst_kind), n_inst, state, residual_out);
        HIP_TRY(hipGetLastError());
    }
    return ATOS_OK;
}

}  // namespace

// ------------------------------------------------------------------ BFS call
namespace {

atos_status bfs_call(atos_graph_t g, int64_t source, int32_t* d_depth, void* d_ws, size_t ws_bytes,
                     const atos_config* cfg, void* stream, atos_stats* st, bool timed) {
    Cfg c;
    Layout L;
    atos_status r = check_common(g, ATOS_APP_BFS, d_ws, ws_bytes, cfg, c, L);
    if (r != ATOS_OK) return r;
    if (!d_depth || source < 0 || source >= g->r.n) return ATOS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    Timer tm(timed && st != nullptr, s);
    KernelEvents ke(timed && st != nullptr && c.strategy != ATOS_BSP);
    r = g->r.off64 ? run_bfs<int64_t>(ke, g->r, c, L, source, d_depth, (char*)d_ws, s)
                   : run_bfs<int32_t>(ke, g->r, c, L, source, d_depth, (char*)d_ws, s);
    return finish_call(r, tm, ke, d_ws, s, st);
}

// ------------------------------------------------------------------ no-allocation scratch
// The workspace of atos_bfs_noalloc: one file-scope device array, so that the
// call needs no device allocation.  Each GPU the library runs on holds its own
// copy at its own address until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol):
// the per-device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is used afterwards.
constexpr size_t kNoallocScratchBytes = ATOS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxNoallocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxNoallocDevices] = {};

__global__ void zero_words_kernel(uint64_t* p, int64_t n_words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// Address of `scratch` on `device` (the current device).  On first use on the
// device its workspace header is cleared by a kernel on `s` (a fill kernel,
// not a memset node, so that the call stays capturable), which every later
// call's work follows in stream order or, on other streams, by the documented
// rule that concurrent calls on one GPU race.
atos_status noalloc_scratch(int device, hipStream_t s, void** out) {
    if (device < 0 || device >= kMaxNoallocDevices) return ATOS_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != device) return ATOS_EINVAL;  // the graph lives on another device
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255u) != 0u) return ATOS_EHIP;
        hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(256), 0, s, (uint64_t*)p,
                           (int64_t)(ATOS_WORKSPACE_HEADER_BYTES / sizeof(uint64_t)));
        HIP_TRY(hipGetLastError());
        g_noalloc_ptr[device] = p;
    }
    *out = g_noalloc_ptr[device];
    return ATOS_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

atos_status atos_trace_attach(void* d_buf, size_t bytes) {
    if (d_buf == nullptr) {
        std::lock_guard<std::mutex> lock(g_trace_mu);
        g_trace = nullptr;
        g_trace_device = -1;
        return ATOS_OK;
    }
    if (bytes < 96 || ((uintptr_t)d_buf & 255u) != 0) return ATOS_EINVAL;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, d_buf) != hipSuccess) {
        (void)hipGetLastError();  // not a pointer HIP knows: clear the error it recorded
        return ATOS_EINVAL;
    }
    if (attr.type != hipMemoryTypeDevice) return ATOS_EINVAL;
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, attr.device));
    const uint64_t hdr[3] = {0ull, (uint64_t)((bytes - 64) / sizeof(TraceRec)), (uint64_t)khz};
    HIP_TRY(hipMemcpy(d_buf, hdr, sizeof(hdr), hipMemcpyHostToDevice));
    std::lock_guard<std::mutex> lock(g_trace_mu);
    g_trace = (TraceBuf*)d_buf;
    g_trace_device = attr.device;
    return ATOS_OK;
}

const char* atos_strerror(atos_status s) {
    switch (s) {
        case ATOS_OK: return "ok";
        case ATOS_EINVAL: return "invalid argument";
        case ATOS_ENOMEM: return "workspace too small";
        case ATOS_EOVERFLOW: return "worklist ring overflow";
        case ATOS_ETIMEOUT: return "device deadline expired";
        case ATOS_EABORTED: return "run aborted";
        case ATOS_EHIP: return "HIP runtime error";
        case ATOS_ENOTSYMMETRIC: return "graph not loaded as symmetric";
        case ATOS_EUNSUPPORTED: return "configuration not supported";
        case ATOS_EAGAIN: return "no free query slot, memory or worklist capacity";
    }
    return "unknown status";
}

const char* atos_version(void) { return "0.1.0"; }

atos_status atos_graph_load(const void* d_offsets, int32_t offsets_are_int64,
                            const int32_t* d_cols, int64_t n_vertices, int64_t n_edges,
                            uint32_t flags, void* stream, atos_graph_t* out) {
    if (!out || !d_offsets || n_vertices < 0 || n_edges < 0) return ATOS_EINVAL;
    if (n_edges > 0 && !d_cols) return ATOS_EINVAL;
    if (n_vertices >= (int64_t)0x7FFFFFFF) return ATOS_EINVAL;
    if (!offsets_are_int64 && n_edges >= (int64_t)0x7FFFFFFF) return ATOS_EINVAL;
    if (flags & ~(ATOS_GRAPH_SYMMETRIC | ATOS_GRAPH_VALIDATE)) return ATOS_EINVAL;
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    GraphRec r;
    r.offs = d_offsets;
    r.off64 = offsets_are_int64 ? 1 : 0;
    r.cols = d_cols;
    r.n = n_vertices;
    r.m = n_edges;
    r.flags = flags;
    HIP_TRY(hipGetDevice(&r.device));
    HIP_TRY(hipDeviceGetAttribute(&r.num_cu, hipDeviceAttributeMultiprocessorCount, r.device));
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, r.device));
    r.clock_khz = khz > 0 ? khz : 100000;

    // scratch: max degree (8 B) + validation flags (8 B), then the degree-class
    // counts of the vertices of degree >= 64 (for colouring's sqrt(n) class)
    constexpr size_t kHistOff = 64;
    constexpr size_t kScratch = kHistOff + kCombClasses * 4;
    void* scratch = nullptr;
    HIP_TRY(hipMalloc(&scratch, kScratch));
    atos_status status = ATOS_OK;
    do {
        if (hipMemsetAsync(scratch, 0, kScratch, s) != hipSuccess) { status = ATOS_EHIP; break; }
        unsigned long long* d_max = (unsigned long long*)scratch;
        uint32_t* d_bad = (uint32_t*)((char*)scratch + 8);
        uint32_t* d_hist = (uint32_t*)((char*)scratch + kHistOff);
        const CombScope all{nullptr, nullptr, nullptr, 0u};
        const int grid = init_grid(std::max<int64_t>(std::max(n_vertices, n_edges), 1), r.num_cu);
        if (n_vertices > 0) {
            if (r.off64) {
                hipLaunchKernelGGL((max_degree_kernel<int64_t>), dim3(grid), dim3(kInitBlock), 0, s,
                                   (const int64_t*)d_offsets, n_vertices, d_max);
                hipLaunchKernelGGL((comb_hist_kernel<int64_t>), dim3(grid), dim3(kInitBlock), 0, s,
                                   (const int64_t*)d_offsets, n_vertices, all, d_hist);
            } else {
                hipLaunchKernelGGL((max_degree_kernel<int32_t>), dim3(grid), dim3(kInitBlock), 0, s,
                                   (const int32_t*)d_offsets, n_vertices, d_max);
                hipLaunchKernelGGL((comb_hist_kernel<int32_t>), dim3(grid), dim3(kInitBlock), 0, s,
                                   (const int32_t*)d_offsets, n_vertices, all, d_hist);
            }
        }
        if (flags & ATOS_GRAPH_VALIDATE) {
            const int sym = (flags & ATOS_GRAPH_SYMMETRIC) ? 1 : 0;
            if (r.off64)
                hipLaunchKernelGGL((validate_kernel<int64_t>), dim3(grid), dim3(kInitBlock), 0, s,
                                   (const int64_t*)d_offsets, d_cols, n_vertices, n_edges, sym, d_bad);
            else
                hipLaunchKernelGGL((validate_kernel<int32_t>), dim3(grid), dim3(kInitBlock), 0, s,
                                   (const int32_t*)d_offsets, d_cols, n_vertices, n_edges, sym, d_bad);
        }
        if (hipGetLastError() != hipSuccess) { status = ATOS_EHIP; break; }
        unsigned long long host[2] = {0, 0};
        uint32_t hist[kCombClasses];
        if (hipMemcpyAsync(host, scratch, 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(hist, d_hist, sizeof(hist), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            status = ATOS_EHIP;
            break;
        }
        r.max_deg = (int64_t)host[0];
        r.sqrt_class_degree = sqrt_class_degree(hist, n_vertices);
        const uint32_t bad0 = (uint32_t)(host[1] & 0xFFFFFFFFull);
        const uint32_t bad1 = (uint32_t)(host[1] >> 32);
        if (bad0) status = ATOS_EINVAL;
        else if (bad1) status = ATOS_ENOTSYMMETRIC;
    } while (0);
    (void)hipFree(scratch);
    if (status != ATOS_OK) return status;
    atos_graph_t g = new (std::nothrow) atos_graph;
    if (!g) return ATOS_EINVAL;
    g->r = r;
    *out = g;
    return ATOS_OK;
}

atos_status atos_graph_free(atos_graph_t g) {
    if (!g) return ATOS_EINVAL;
    delete g;
    return ATOS_OK;
}

atos_status atos_graph_info(atos_graph_t g, int64_t* n_vertices, int64_t* n_edges,
                            int64_t* max_degree) {
    if (!g) return ATOS_EINVAL;
    if (n_vertices) *n_vertices = g->r.n;
    if (n_edges) *n_edges = g->r.m;
    if (max_degree) *max_degree = g->r.max_deg;
    return ATOS_OK;
}

atos_status atos_workspace_bytes(atos_graph_t g, int32_t app, const atos_config* cfg,
                                 size_t* bytes) {
    if (!g || !bytes) return ATOS_EINVAL;
    if (app != ATOS_APP_BFS && app != ATOS_APP_PAGERANK && app != ATOS_APP_COLOR) return ATOS_EINVAL;
    Cfg c;
    atos_status r = resolve_cfg(g->r, app, cfg, c);
    if (r != ATOS_OK) return r;
    *bytes = layout(g->r, app, c).total;
    return ATOS_OK;
}

atos_status atos_workspace_stats(const void* d_ws, void* stream, atos_stats* st) {
    if (!d_ws || !st) return ATOS_EINVAL;
    std::memset(st, 0, sizeof(*st));
    return read_stats(d_ws, (hipStream_t)stream, st);
}

atos_status atos_bfs(atos_graph_t g, int64_t source, int32_t* d_depth, void* d_ws, size_t ws_bytes,
                     const atos_config* cfg, void* stream, atos_stats* st) {
    return bfs_call(g, source, d_depth, d_ws, ws_bytes, cfg, stream, st, true);
}

atos_status atos_bfs_noalloc(atos_graph_t g, int64_t source, int32_t* d_depth,
                             const atos_config* cfg, void* stream, atos_stats* st) {
    if (!g) return ATOS_EINVAL;
    size_t need = 0;
    atos_status r = atos_workspace_bytes(g, ATOS_APP_BFS, cfg, &need);
    if (r != ATOS_OK) return r;
    if (need > kNoallocScratchBytes) return ATOS_ENOMEM;
    void* ws = nullptr;
    r = noalloc_scratch(g->r.device, (hipStream_t)stream, &ws);
    if (r != ATOS_OK) return r;
    // no timing events either: st, when given, carries the status and counters only
    return bfs_call(g, source, d_depth, ws, kNoallocScratchBytes, cfg, stream, st, false);
}

atos_status atos_pagerank(atos_graph_t g, float damping, float epsilon, float* d_rank,
                          float* d_residual, void* d_ws, size_t ws_bytes, const atos_config* cfg,
                          void* stream, atos_stats* st) {
    Cfg c;
    Layout L;
    atos_status r = check_common(g, ATOS_APP_PAGERANK, d_ws, ws_bytes, cfg, c, L);
    if (r != ATOS_OK) return r;
    if (!d_rank || !(damping > 0.0f && damping < 1.0f) || !(epsilon > 0.0f)) return ATOS_EINVAL;
    if (!(g->r.flags & ATOS_GRAPH_SYMMETRIC)) return ATOS_ENOTSYMMETRIC;
    hipStream_t s = (hipStream_t)stream;
    Timer tm(st != nullptr, s);
    KernelEvents ke(st != nullptr && c.strategy != ATOS_BSP);
    r = g->r.off64 ? run_pagerank<int64_t>(ke, g->r, c, L, damping, epsilon, -1, d_rank, d_residual, (char*)d_ws, s)
                   : run_pagerank<int32_t>(ke, g->r, c, L, damping, epsilon, -1, d_rank, d_residual, (char*)d_ws, s);
    return finish_call(r, tm, ke, d_ws, s, st);
}

atos_status atos_ppr(atos_graph_t g, int64_t source, float damping, float epsilon, float* d_rank,
                     float* d_residual, void* d_ws, size_t ws_bytes, const atos_config* cfg,
                     void* stream, atos_stats* st) {
    Cfg c;
    Layout L;
    atos_status r = check_common(g, ATOS_APP_PAGERANK, d_ws, ws_bytes, cfg, c, L);
    if (r != ATOS_OK) return r;
    if (!d_rank || !(damping > 0.0f && damping < 1.0f) || !(epsilon > 0.0f)) return ATOS_EINVAL;
    if (source < 0 || source >= g->r.n) return ATOS_EINVAL;
    if (!(g->r.flags & ATOS_GRAPH_SYMMETRIC)) return ATOS_ENOTSYMMETRIC;
    // the sweep and the combining set-up cover the whole graph
    if (c.check_size != 0 || (cfg && cfg->pr_combine > 0)) return ATOS_EUNSUPPORTED;
    c.comb_flush = 0;
    // a personalized run's few tasks stay in the worker's own ring by default
    // (R-MAT scale 22: 11.3 ms against 11.5 ms a query; road grid 0.43 against 0.44)
    if (!cfg || cfg->push_policy == ATOS_PUSH_AUTO) c.push_shallow = false;
    hipStream_t s = (hipStream_t)stream;
    Timer tm(st != nullptr, s);
    KernelEvents ke(st != nullptr && c.strategy != ATOS_BSP);
    r = g->r.off64 ? run_pagerank<int64_t>(ke, g->r, c, L, damping, epsilon, source, d_rank, d_residual, (char*)d_ws, s)
                   : run_pagerank<int32_t>(ke, g->r, c, L, damping, epsilon, source, d_rank, d_residual, (char*)d_ws, s);
    return finish_call(r, tm, ke, d_ws, s, st);
}

atos_status atos_color(atos_graph_t g, uint64_t priority_seed, int32_t* d_color, int32_t* d_n_colors,
                       void* d_ws, size_t ws_bytes, const atos_config* cfg, void* stream,
                       atos_stats* st) {
    Cfg c;
    Layout L;
    atos_status r = check_common(g, ATOS_APP_COLOR, d_ws, ws_bytes, cfg, c, L);
    if (r != ATOS_OK) return r;
    if (!d_color) return ATOS_EINVAL;
    if (!(g->r.flags & ATOS_GRAPH_SYMMETRIC)) return ATOS_ENOTSYMMETRIC;
    hipStream_t s = (hipStream_t)stream;
    Timer tm(st != nullptr, s);
    KernelEvents ke(st != nullptr && c.strategy != ATOS_BSP);
    r = g->r.off64 ? run_color<int64_t>(ke, g->r, c, L, priority_seed, d_color, d_n_colors, (char*)d_ws, s)
                   : run_color<int32_t>(ke, g->r, c, L, priority_seed, d_color, d_n_colors, (char*)d_ws, s);
    return finish_call(r, tm, ke, d_ws, s, st);
}

atos_status atos_batch_plan(atos_graph_t g, const atos_batch_instance* instances, int32_t n_instances,
                            float damping, float epsilon, const atos_config* cfg, void* stream,
                            atos_batch_t* out) {
    if (!g || !out || (n_instances > 0 && !instances) || n_instances < 0) return ATOS_EINVAL;
    *out = nullptr;
    const int64_t n = g->r.n;
    uint32_t n_bfs = 0, n_pr = 0;
    uint64_t n_init = 0, pr_edges = 0;
    int64_t prev_end = 0;
    for (int32_t i = 0; i < n_instances; ++i) {
        const atos_batch_instance& x = instances[i];
        if (x.reserved != 0 || x.vertex_begin < prev_end || x.vertex_end <= x.vertex_begin ||
            x.vertex_end > n)
            return ATOS_EINVAL;
        prev_end = x.vertex_end;
        if (x.app == ATOS_APP_BFS) {
            if (x.source < x.vertex_begin || x.source >= x.vertex_end) return ATOS_EINVAL;
            ++n_bfs;
            ++n_init;
        } else if (x.app == ATOS_APP_PAGERANK) {
            ++n_pr;
            n_init += (uint64_t)(x.vertex_end - x.vertex_begin);
        } else {
            return ATOS_EINVAL;
        }
    }
    if (n_pr > 0) {
        if (!(damping > 0.0f && damping < 1.0f) || !(epsilon > 0.0f)) return ATOS_EINVAL;
        if (!(g->r.flags & ATOS_GRAPH_SYMMETRIC)) return ATOS_ENOTSYMMETRIC;
    }
    Cfg c;
    atos_config z;
    std::memset(&z, 0, sizeof(z));
    if (cfg) z = *cfg;
    if (z.strategy != ATOS_PERSISTENT || z.pr_check_size != 0) return ATOS_EUNSUPPORTED;
    atos_status r = resolve_cfg(g->r, ATOS_APP_PAGERANK, &z, c);
    if (r != ATOS_OK) return r;
    if (z.pr_combine == 0 && c.comb_flush != 0) c.comb_flush = kDefaultBatchCombFlush;
    if (z.queue_capacity == 0) {  // all rings together: 2 x max(initial tasks, vertices)
        z.queue_capacity = (int64_t)std::max<uint64_t>(
            kDefaultMinRing, 2 * std::max<uint64_t>(n_init, (uint64_t)n) / c.n_queues);
        r = resolve_cfg(g->r, ATOS_APP_PAGERANK, &z, c);
    }
    if (r != ATOS_OK) return r;
    if (n_init > c.capacity * c.n_queues) return ATOS_EINVAL;

    // host copies of the device tables
    std::vector<uint32_t> bfs_src, pr_begin, kind;
    std::vector<uint64_t> pr_prefix(1, 0), pr_edge_begin, pr_edge_prefix(1, 0);
    std::vector<int64_t> ib, ie, src;
    std::vector<int64_t> offs_h;  // offsets at PageRank range bounds
    hipStream_t s = (hipStream_t)stream;
    for (int32_t i = 0; i < n_instances; ++i) {
        const atos_batch_instance& x = instances[i];
        ib.push_back(x.vertex_begin);
        ie.push_back(x.vertex_end);
        kind.push_back((uint32_t)x.app);
        src.push_back(x.app == ATOS_APP_BFS ? x.source : -1);
        if (x.app == ATOS_APP_BFS) {
            bfs_src.push_back((uint32_t)x.source);
        } else {
            pr_begin.push_back((uint32_t)x.vertex_begin);
            pr_prefix.push_back(pr_prefix.back() + (uint64_t)(x.vertex_end - x.vertex_begin));
            // edge range of the instance: read its two bounding offsets
            int64_t lohi[2] = {0, 0};
            if (g->r.off64) {
                HIP_TRY(hipMemcpy(&lohi[0], (const int64_t*)g->r.offs + x.vertex_begin, 8, hipMemcpyDeviceToHost));
                HIP_TRY(hipMemcpy(&lohi[1], (const int64_t*)g->r.offs + x.vertex_end, 8, hipMemcpyDeviceToHost));
            } else {
                int32_t a = 0, bnd = 0;
                HIP_TRY(hipMemcpy(&a, (const int32_t*)g->r.offs + x.vertex_begin, 4, hipMemcpyDeviceToHost));
                HIP_TRY(hipMemcpy(&bnd, (const int32_t*)g->r.offs + x.vertex_end, 4, hipMemcpyDeviceToHost));
                lohi[0] = a;
                lohi[1] = bnd;
            }
            pr_edge_begin.push_back((uint64_t)lohi[0]);
            pr_edge_prefix.push_back(pr_edge_prefix.back() + (uint64_t)(lohi[1] - lohi[0]));
        }
    }
    pr_edges = pr_edge_prefix.back();

    atos_batch* b = new (std::nothrow) atos_batch;
    if (!b) return ATOS_EINVAL;
    b->g = g;
    b->inst.assign(instances, instances + n_instances);
    b->damping = damping;
    b->eps = epsilon;
    b->cfg = c;
    if (c.segmented) segment_bounds(b, b->cfg);
    b->L = batch_layout((size_t)n_instances, n_bfs, n_pr);
    b->n_bfs = n_bfs;
    b->n_pr = n_pr;
    b->n_init = n_init;
    b->pr_edges = pr_edges;
    b->d_tab = nullptr;
    auto fail = [&](atos_status st) {
        if (b->d_tab) (void)hipFree(b->d_tab);
        delete b;
        return st;
    };
    if (hipMalloc((void**)&b->d_tab, b->L.total) != hipSuccess) return fail(ATOS_EHIP);
    auto put = [&](size_t off, const void* src_h, size_t bytes) {
        return bytes == 0 || hipMemcpy(b->d_tab + off, src_h, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = put(b->L.bfs_src, bfs_src.data(), bfs_src.size() * 4) &&
              put(b->L.pr_begin, pr_begin.data(), pr_begin.size() * 4) &&
              put(b->L.pr_prefix, pr_prefix.data(), pr_prefix.size() * 8) &&
              put(b->L.pr_edge_begin, pr_edge_begin.data(), pr_edge_begin.size() * 8) &&
              put(b->L.pr_edge_prefix, pr_edge_prefix.data(), pr_edge_prefix.size() * 8) &&
              put(b->L.inst_begin, ib.data(), ib.size() * 8) &&
              put(b->L.inst_end, ie.data(), ie.size() * 8) &&
              put(b->L.inst_kind, kind.data(), kind.size() * 4) &&
              put(b->L.inst_src, src.data(), src.size() * 8) &&
              hipMemset(b->d_tab + b->L.bad, 0, 8) == hipSuccess;
    if (!ok) return fail(ATOS_EHIP);
    // every edge of an instance must stay inside it
    const int grid = init_grid(std::max<int64_t>(n, 1), g->r.num_cu);
    if (g->r.off64)
        hipLaunchKernelGGL((batch_validate_kernel<int64_t>), dim3(grid), dim3(kInitBlock), 0, s,
                           (const int64_t*)g->r.offs, g->r.cols, n, (const int64_t*)(b->d_tab + b->L.inst_begin),
                           (const int64_t*)(b->d_tab + b->L.inst_end), (uint32_t)n_instances,
                           (uint32_t*)(b->d_tab + b->L.bad));
    else
        hipLaunchKernelGGL((batch_validate_kernel<int32_t>), dim3(grid), dim3(kInitBlock), 0, s,
                           (const int32_t*)g->r.offs, g->r.cols, n, (const int64_t*)(b->d_tab + b->L.inst_begin),
                           (const int64_t*)(b->d_tab + b->L.inst_end), (uint32_t)n_instances,
                           (uint32_t*)(b->d_tab + b->L.bad));
    uint32_t bad = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&bad, b->d_tab + b->L.bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(ATOS_EHIP);
    if (bad) return fail(ATOS_EINVAL);
    // prime the occupancy cache so that later runs make no runtime queries (graph capture)
    (void)(g->r.off64 ? occupancy(persistent_kernel<256, BatchApp, int64_t>, 256)
                      : occupancy(persistent_kernel<256, BatchApp, int32_t>, 256));
    *out = b;
    return ATOS_OK;
}

atos_status atos_batch_free(atos_batch_t b) {
    if (!b) return ATOS_EINVAL;
    if (b->d_tab) (void)hipFree(b->d_tab);
    delete b;
    return ATOS_OK;
}

atos_status atos_batch_workspace_bytes(atos_batch_t b, size_t* bytes) {
    if (!b || !bytes) return ATOS_EINVAL;
    *bytes = batch_ws_layout(b).total;
    return ATOS_OK;
}

atos_status atos_batch_run(atos_batch_t b, uint32_t* d_state, float* d_residual, void* d_ws,
                           size_t ws_bytes, void* stream, atos_stats* st) {
    if (!b || !d_state || !d_ws || ((uintptr_t)d_ws & 255u) != 0u) return ATOS_EINVAL;
    const Layout L = batch_ws_layout(b);
    if (ws_bytes < L.total) return ATOS_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    Timer tm(st != nullptr, s);
    KernelEvents ke(st != nullptr);
    atos_status r = b->g->r.off64 ? run_batch<int64_t>(ke, b, L, d_state, d_residual, (char*)d_ws, s)
                                  : run_batch<int32_t>(ke, b, L, d_state, d_residual, (char*)d_ws, s);
    return finish_call(r, tm, ke, d_ws, s, st);
}

atos_status atos_batch_capture(atos_batch_t b, uint32_t* d_state, float* d_residual, void* d_ws,
                               size_t ws_bytes, void* stream, atos_exec_t* out) {
    if (!out || !stream) return ATOS_EINVAL;
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    atos_status r = atos_batch_run(b, d_state, d_residual, d_ws, ws_bytes, stream, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (r != ATOS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (e != hipSuccess || !graph) return ATOS_EHIP;
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return ATOS_EHIP;
    atos_exec* x = new (std::nothrow) atos_exec;
    if (!x) {
        (void)hipGraphExecDestroy(exec);
        return ATOS_EINVAL;
    }
    x->exec = exec;
    *out = x;
    return ATOS_OK;
}

atos_status atos_exec_launch(atos_exec_t x, void* stream) {
    if (!x) return ATOS_EINVAL;
    HIP_TRY(hipGraphLaunch(x->exec, (hipStream_t)stream));
    return ATOS_OK;
}

atos_status atos_exec_free(atos_exec_t x) {
    if (!x) return ATOS_EINVAL;
    (void)hipGraphExecDestroy(x->exec);
    delete x;
    return ATOS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ autotuning
namespace {

// Candidate launch shapes: worker size x fetch granularity (fetch <= worker,
// powers of two up to 256) x queue layout.
std::vector<atos_config> tune_candidates(const atos_config& base, bool batch) {
    std::vector<atos_config> out;
    const int workers[] = {64, 128, 256, 512, 1024};
    std::vector<int> layouts = {ATOS_QUEUE_PER_XCD, ATOS_QUEUE_GLOBAL};
    if (batch) layouts.push_back(ATOS_QUEUE_SEGMENTED);
    for (int layout : layouts) {
        for (int w : workers) {
            for (int f = 1; f <= std::min(w, 256); f *= 2) {
                atos_config c = base;
                c.strategy = ATOS_PERSISTENT;
                c.worker = w;
                c.fetch = f;
                c.queue_layout = layout;
                out.push_back(c);
            }
        }
    }
    return out;
}

// Second stage at the first stage's winning launch shape: the kernel
// strategies (persistent, discrete launches, rounds in one launch; batches
// run persistent only) each with own-ring and shallowest-ring pushes.
std::vector<atos_config> tune_refinements(const atos_config& won, bool all_strategies) {
    std::vector<atos_config> out;
    const int strategies[] = {ATOS_PERSISTENT, ATOS_DISCRETE, ATOS_ROUNDS};
    for (int strategy : strategies) {
        if (strategy != ATOS_PERSISTENT && !all_strategies) continue;
        for (int push : {ATOS_PUSH_OWN, ATOS_PUSH_SHALLOWEST}) {
            atos_config c = won;
            c.strategy = strategy;
            c.push_policy = push;
            out.push_back(c);
        }
    }
    return out;
}

// Progress callback of the tuner (atos_tune_set_progress), or null.
std::mutex g_tune_mu;
atos_tune_progress_fn g_tune_cb = nullptr;
void* g_tune_user = nullptr;

template <class Run>
atos_status tune_loop(const atos_config* base, int32_t reps, void* stream, bool all_strategies,
                      Run run, atos_tune_result* results, int32_t max_results, int32_t* n_results,
                      atos_config* best) {
    atos_tune_progress_fn cb;
    void* user;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        cb = g_tune_cb;
        user = g_tune_user;
    }
    if (reps < 1 || !best || (max_results > 0 && !results)) return ATOS_EINVAL;
    atos_config z;
    std::memset(&z, 0, sizeof(z));
    std::vector<atos_config> cands = tune_candidates(base ? *base : z, !all_strategies);
    const size_t n_stage1 = cands.size();
    hipStream_t s = (hipStream_t)stream;
    float best_ms = -1.0f;
    int32_t n = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        atos_config c = cands[i];
        // once a point has run, a point more than five times slower cannot win:
        // its runs stop at that deadline (ETIMEOUT) instead of running to the end
        if (best_ms >= 0.0f) {
            const uint32_t own = c.timeout_ms ? c.timeout_ms : kDefaultTimeoutMs;
            const uint32_t cut = (uint32_t)std::max(1000.0f, 5.0f * best_ms);
            c.timeout_ms = std::min(own, cut);
        }
        std::vector<float> times;
        int32_t status = ATOS_OK;
        for (int32_t r = 0; r <= reps && status == ATOS_OK; ++r) {  // r == 0 warms up
            atos_stats st;
            std::memset(&st, 0, sizeof(st));
            const atos_status e = run(c, s, &st);
            if (e != ATOS_OK) status = e;
            else if (st.status != ATOS_OK) status = st.status;
            else if (r > 0) times.push_back(st.device_ms);
        }
        float ms = -1.0f;
        if (status == ATOS_OK && !times.empty()) {
            std::sort(times.begin(), times.end());
            ms = times[times.size() / 2];
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                *best = cands[i];  // with its own deadline, not the sweep's cut
            }
        }
        atos_tune_result tr;
        tr.cfg = cands[i];
        tr.median_ms = ms;
        tr.status = status;
        tr.reserved = 0;
        if (n < max_results) results[n] = tr;
        ++n;
        if (cb) cb(n, (int32_t)(i + 1 < n_stage1 ? n_stage1 : cands.size()), &tr, user);
        if (i + 1 == n_stage1 && best_ms >= 0.0f) {  // the first stage is done
            const std::vector<atos_config> more = tune_refinements(*best, all_strategies);
            cands.insert(cands.end(), more.begin(), more.end());
        }
    }
    if (n_results) *n_results = std::min(n, max_results);
    return best_ms < 0.0f ? ATOS_EUNSUPPORTED : ATOS_OK;
}

}  // namespace

extern "C" {

atos_status atos_tune_set_progress(atos_tune_progress_fn fn, void* user) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cb = fn;
    g_tune_user = user;
    return ATOS_OK;
}

atos_status atos_autotune(atos_graph_t g, int32_t app, int64_t source, float damping, float epsilon,
                          uint64_t seed, void* d_out, float* d_residual, void* d_ws, size_t ws_bytes,
                          const atos_config* base, int32_t reps, void* stream,
                          atos_tune_result* results, int32_t max_results, int32_t* n_results,
                          atos_config* best) {
    if (!g || !d_out) return ATOS_EINVAL;
    if (app == ATOS_APP_BFS) {
        return tune_loop(base, reps, stream, true, [&](const atos_config& c, hipStream_t s, atos_stats* st) {
            return atos_bfs(g, source, (int32_t*)d_out, d_ws, ws_bytes, &c, s, st);
        }, results, max_results, n_results, best);
    }
    if (app == ATOS_APP_PAGERANK) {
        return tune_loop(base, reps, stream, true, [&](const atos_config& c, hipStream_t s, atos_stats* st) {
            return atos_pagerank(g, damping, epsilon, (float*)d_out, d_residual, d_ws, ws_bytes, &c, s, st);
        }, results, max_results, n_results, best);
    }
    if (app == ATOS_APP_COLOR) {
        return tune_loop(base, reps, stream, true, [&](const atos_config& c, hipStream_t s, atos_stats* st) {
            return atos_color(g, seed, (int32_t*)d_out, nullptr, d_ws, ws_bytes, &c, s, st);
        }, results, max_results, n_results, best);
    }
    return ATOS_EINVAL;
}

atos_status atos_batch_set_config(atos_batch_t b, const atos_config* cfg) {
    if (!b || !cfg) return ATOS_EINVAL;
    if (cfg->strategy != ATOS_PERSISTENT || cfg->pr_check_size != 0) return ATOS_EUNSUPPORTED;
    atos_config z = *cfg;
    const uint32_t nq = z.queue_layout == ATOS_QUEUE_GLOBAL ? 1u : (uint32_t)kMaxQueues;
    // keep the total ring size the workspace was sized for
    z.queue_capacity = (int64_t)(b->cfg.capacity * b->cfg.n_queues / nq);
    Cfg c;
    atos_status r = resolve_cfg(b->g->r, ATOS_APP_PAGERANK, &z, c);
    if (r != ATOS_OK) return r;
    if (z.pr_combine == 0 && c.comb_flush != 0) c.comb_flush = kDefaultBatchCombFlush;
    if (c.segmented) segment_bounds(b, c);
    b->cfg = c;
    return ATOS_OK;
}

atos_status atos_batch_autotune(atos_batch_t b, uint32_t* d_state, float* d_residual, void* d_ws,
                                size_t ws_bytes, int32_t reps, void* stream,
                                atos_tune_result* results, int32_t max_results, int32_t* n_results,
                                atos_config* best) {
    if (!b || !d_state) return ATOS_EINVAL;
    const Cfg saved = b->cfg;
    atos_config base;
    std::memset(&base, 0, sizeof(base));
    base.timeout_ms = saved.timeout_ms;
    atos_status r = tune_loop(&base, reps, stream, false, [&](const atos_config& c, hipStream_t s, atos_stats* st) {
        atos_status e = atos_batch_set_config(b, &c);
        if (e != ATOS_OK) return e;
        return atos_batch_run(b, d_state, d_residual, d_ws, ws_bytes, s, st);
    }, results, max_results, n_results, best);
    b->cfg = saved;
    return r;
}

}  // extern "C"
