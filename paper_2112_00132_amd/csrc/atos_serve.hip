// libatos serving: the host side of the resident query daemon
// (declarations and contracts in include/atos.h; device side in atos_serve.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "atos.h"
#include "atos_device.h"
#include "atos_admission.h"
#include "atos_internal.h"
#include "atos_persistent.h"
#include "atos_serve.h"

using namespace atos;
using namespace atos::host;

namespace {

constexpr uint32_t kSrvDefaultSlots = 256;
constexpr uint32_t kSrvDefaultTimeoutMs = 600000;
constexpr uint64_t kSrvMinRing = 1ull << 16;
constexpr uint64_t kSrvMaxRing = 1ull << 31;
constexpr size_t kSrvMinHeap = 1u << 20;

struct SrvCfg {
    int worker, fetch, grid;
    uint32_t slots, nq, n_records;
    uint64_t capacity;  // entries per ring
    uint32_t timeout_ms;
    bool push_shallow;  // publish into the shallowest ring (else the worker's own)
    bool push_query;    // publish every task into the ring of its query's slot
};

struct SrvLayout {
    size_t header = 0, graphs = 0, slots = 0, rings = 0, heap = 0;
};

atos_status resolve_srv(const std::vector<GraphRec>& gs, const atos_server_config* in, SrvCfg& c) {
    atos_server_config z;
    std::memset(&z, 0, sizeof(z));
    const atos_server_config& u = in ? *in : z;
    for (int i = 0; i < 3; ++i)
        if (u.reserved[i] != 0u) return ATOS_EINVAL;
    if (u.push_policy != ATOS_PUSH_AUTO && u.push_policy != ATOS_PUSH_OWN &&
        u.push_policy != ATOS_PUSH_SHALLOWEST && u.push_policy != ATOS_PUSH_QUERY)
        return ATOS_EINVAL;
    if (u.push_policy == ATOS_PUSH_QUERY && u.queue_layout == ATOS_QUEUE_GLOBAL) return ATOS_EINVAL;
    c.push_shallow = u.push_policy == ATOS_PUSH_SHALLOWEST;
    // default: a ring per XCD, every task in the ring of its query
    c.push_query = u.push_policy == ATOS_PUSH_QUERY ||
                   (u.push_policy == ATOS_PUSH_AUTO && u.queue_layout != ATOS_QUEUE_GLOBAL);
    c.worker = u.worker ? u.worker : 1024;
    if (c.worker != 64 && c.worker != 128 && c.worker != 256 && c.worker != 512 && c.worker != 1024)
        return ATOS_EINVAL;
    // a worker claims a whole batch of light tasks (saturated R-MAT + grid mix:
    // 227-288 queries/s with 1024-task claims against 187-239 with 512)
    c.fetch = u.fetch ? u.fetch : c.worker;
    if (c.fetch < 1 || c.fetch > c.worker) return ATOS_EINVAL;
    if (u.grid < 0) return ATOS_EINVAL;
    c.grid = u.grid;
    if (u.max_queries < 0 || u.max_queries > (int32_t)kSrvMaxSlots) return ATOS_EINVAL;
    c.slots = u.max_queries ? (uint32_t)u.max_queries : kSrvDefaultSlots;
    c.n_records = (uint32_t)next_pow2(std::max<uint64_t>(64, 2ull * c.slots));
    // A query's tasks must stay in one FIFO order: when they are spread over
    // rings that other queries have filled to different depths, part of a
    // road-grid BFS runs many levels ahead of the rest and its vertices are
    // expanded again and again (R-MAT + grid mix: 7.0 G tasks per 300 queries
    // with each worker pushing into its own XCD's ring, 2.1-2.6 G with one
    // shared ring or with every task in its query's ring).  One shared ring
    // serialises each BFS level on its head and tail (a lone 4096^2 grid BFS:
    // 240 ms against 64 ms), so the default keeps a ring per XCD and puts each
    // query's tasks in the ring of its slot.
    if (u.queue_layout == ATOS_QUEUE_GLOBAL) c.nq = 1;
    else if (u.queue_layout == ATOS_QUEUE_PER_XCD || u.queue_layout == ATOS_QUEUE_AUTO) c.nq = kMaxQueues;
    else return ATOS_EINVAL;
    if (u.queue_capacity < 0) return ATOS_EINVAL;
    uint64_t want = (uint64_t)u.queue_capacity;
    if (want == 0) {
        // all rings together: 16 entries per resident vertex (a running query
        // reserves 2 per vertex of its graph, so this admits 8 concurrent
        // queries on every graph at once); with a query's tasks in the ring of
        // its slot, 4 entries per resident vertex in every ring
        uint64_t total = 0;
        for (const GraphRec& g : gs) total += (uint64_t)g.n;
        want = std::max<uint64_t>(kSrvMinRing, c.push_query ? 4 * total : 16 * total / c.nq);
    }
    c.capacity = std::max(kSrvMinRing, next_pow2(want));
    if (c.capacity > kSrvMaxRing) return ATOS_EINVAL;
    c.timeout_ms = u.timeout_ms ? u.timeout_ms : kSrvDefaultTimeoutMs;
    return ATOS_OK;
}

SrvLayout srv_layout(size_t n_graphs, const SrvCfg& c) {
    SrvLayout L;
    size_t off = 0;
    L.header = off;
    off = align_up(off + sizeof(SrvHeader), 4096);
    L.graphs = off;
    off = align_up(off + n_graphs * sizeof(SrvGraph), 4096);
    L.slots = off;
    off = align_up(off + (size_t)c.slots * sizeof(SrvSlot), 4096);
    L.rings = off;
    off = align_up(off + (size_t)c.capacity * c.nq * sizeof(uint64_t), 4096);
    L.heap = off;
    return L;
}

atos_status collect_graphs(const atos_graph_t* graphs, int32_t n_graphs, std::vector<GraphRec>& gs) {
    if (!graphs || n_graphs <= 0 || n_graphs > 1024) return ATOS_EINVAL;
    gs.clear();
    for (int32_t i = 0; i < n_graphs; ++i) {
        if (!graphs[i]) return ATOS_EINVAL;
        const GraphRec& r = graphs[i]->r;
        if (r.n <= 0 || (uint64_t)r.n >= kSrvMaxVertices) return ATOS_EINVAL;
        if (i > 0 && r.device != gs[0].device) return ATOS_EINVAL;
        gs.push_back(r);
    }
    return ATOS_OK;
}

// First-fit allocator over the state heap, coalescing on release.
__global__ void srv_reset_kernel(SrvHeader* H, SrvSlot* slots, uint32_t n_slots, uint64_t* rings,
                                 uint64_t n_ring) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t* h = (uint64_t*)H;
    for (uint64_t i = t0; i < sizeof(SrvHeader) / 8; i += stride) h[i] = 0ull;
    uint64_t* sl = (uint64_t*)slots;
    for (uint64_t i = t0; i < (uint64_t)n_slots * (sizeof(SrvSlot) / 8); i += stride) sl[i] = 0ull;
    for (uint64_t i = t0; i < n_ring; i += stride) rings[i] = 0ull;
}

template <int B>
atos_status launch_daemon(const GraphRec& g0, const SrvCfg& c, SrvArgs a, hipStream_t s, int* grid_out) {
    auto kern = serve_kernel<B>;
    const int occ = occupancy(kern, B);
    // leave room for one more workgroup per CU, so that other work can still run
    const int grid = c.grid ? c.grid : g0.num_cu * std::max(1, occ - 1);
    a.bulk_margin = (uint64_t)c.fetch * (uint64_t)grid;
    a.fetch_share = 0u;  // fixed claims (BFS and PageRank tasks are light)
    a.push_shallow = c.push_shallow ? 1u : 0u;
    a.push_query = c.push_query ? 1u : 0u;
    // steal from another ring only what its own workers could not take at once
    a.steal_min = c.push_query ? (uint64_t)c.fetch * (uint64_t)std::max(1, grid / (int)c.nq) : 0ull;
    a.poll_every = (uint32_t)std::max(1, grid / 64);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(B), 0, s, a);
    *grid_out = grid;
    return hipGetLastError() == hipSuccess ? ATOS_OK : ATOS_EHIP;
}

}  // namespace

struct atos_server {
    std::mutex mu;
    std::vector<GraphRec> g;
    SrvCfg c;
    SrvLayout L;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    SrvSubmit* h_sub = nullptr;
    SrvDone* h_done = nullptr;
    SrvHostCtl* h_ctl = nullptr;
    uint64_t* h_snap = nullptr;  // snapshot words, written by the daemon
    size_t snap_words = 0;
    hipStream_t aux = nullptr;  // non-blocking stream for copies when the daemon is not running
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool running = false, stopping = false;
    uint64_t sub_next = 0, done_next = 0, next_id = 1;
    // slots, worklist budgets (one pool per ring when a query's tasks all go
    // to the ring of its slot, else one for all rings) and the state heap
    Admission adm;
    int grid = 0;
    uint64_t epoch = 0;  // launch number of the current daemon
    struct Query {
        uint64_t tag;
        uint32_t slot;
        int32_t app, graph;
        size_t off, bytes;
        uint64_t ring;
        bool done;
    };
    std::map<uint64_t, Query> queries;
};

namespace {

void free_host(atos_server* s) {
    if (s->h_sub) (void)hipHostFree(s->h_sub);
    if (s->h_done) (void)hipHostFree(s->h_done);
    if (s->h_ctl) (void)hipHostFree(s->h_ctl);
    if (s->h_snap) (void)hipHostFree(s->h_snap);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    if (s->aux) (void)hipStreamDestroy(s->aux);
    s->h_sub = nullptr;
    s->h_done = nullptr;
    s->h_ctl = nullptr;
    s->h_snap = nullptr;
    s->ev0 = s->ev1 = nullptr;
    s->aux = nullptr;
}

size_t state_bytes(int32_t app, int64_t n) {
    return align_up((size_t)n * (app == ATOS_APP_BFS ? 4u : 16u), 256);
}

}  // namespace

extern "C" {

atos_status atos_server_arena_bytes(const atos_graph_t* graphs, int32_t n_graphs,
                                    const atos_server_config* cfg, size_t* bytes) {
    if (!bytes) return ATOS_EINVAL;
    std::vector<GraphRec> gs;
    atos_status r = collect_graphs(graphs, n_graphs, gs);
    if (r != ATOS_OK) return r;
    SrvCfg c;
    r = resolve_srv(gs, cfg, c);
    if (r != ATOS_OK) return r;
    *bytes = srv_layout(gs.size(), c).heap;
    return ATOS_OK;
}

atos_status atos_server_create(const atos_graph_t* graphs, int32_t n_graphs,
                               const atos_server_config* cfg, void* d_arena, size_t arena_bytes,
                               atos_server_t* out) {
    if (!out || !d_arena || ((uintptr_t)d_arena & 255u) != 0u) return ATOS_EINVAL;
    *out = nullptr;
    atos_server* s = new (std::nothrow) atos_server;
    if (!s) return ATOS_EINVAL;
    atos_status r = collect_graphs(graphs, n_graphs, s->g);
    if (r == ATOS_OK) r = resolve_srv(s->g, cfg, s->c);
    if (r != ATOS_OK) {
        delete s;
        return r;
    }
    s->L = srv_layout(s->g.size(), s->c);
    if (arena_bytes < s->L.heap + kSrvMinHeap) {
        delete s;
        return ATOS_ENOMEM;
    }
    s->arena = (char*)d_arena;
    s->arena_bytes = arena_bytes;
    const unsigned fl = hipHostMallocCoherent | hipHostMallocMapped;
    if (hipHostMalloc((void**)&s->h_sub, s->c.n_records * sizeof(SrvSubmit), fl) != hipSuccess ||
        hipHostMalloc((void**)&s->h_done, s->c.n_records * sizeof(SrvDone), fl) != hipSuccess ||
        hipHostMalloc((void**)&s->h_ctl, sizeof(SrvHostCtl), fl) != hipSuccess ||
        hipHostMalloc((void**)&s->h_snap,
                      (s->snap_words = 13 + 3ull * s->c.nq + 4ull * s->c.slots +
                                       (uint64_t)kSrvSnapRingWords * s->c.nq) * sizeof(uint64_t),
                      fl) != hipSuccess ||
        hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess) {
        free_host(s);
        delete s;
        return ATOS_EHIP;
    }
    std::memset((void*)s->h_sub, 0, s->c.n_records * sizeof(SrvSubmit));
    std::memset((void*)s->h_done, 0, s->c.n_records * sizeof(SrvDone));
    std::memset((void*)s->h_ctl, 0, sizeof(SrvHostCtl));
    s->adm.init(s->c.slots, s->c.push_query ? s->c.nq : 1u,
                s->c.push_query ? s->c.capacity : s->c.capacity * s->c.nq, s->L.heap,
                arena_bytes - s->L.heap);
    *out = s;
    return ATOS_OK;
}

atos_status atos_server_start(atos_server_t s, void* stream) {
    if (!s) return ATOS_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->running) return ATOS_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    std::vector<SrvGraph> tab(s->g.size());
    for (size_t i = 0; i < s->g.size(); ++i) {
        tab[i].offs = s->g[i].offs;
        tab[i].cols = s->g[i].cols;
        tab[i].n = s->g[i].n;
        tab[i].offs64 = s->g[i].off64 ? 1u : 0u;
        tab[i].pad = 0;
    }
    std::memset((void*)s->h_sub, 0, s->c.n_records * sizeof(SrvSubmit));
    std::memset((void*)s->h_done, 0, s->c.n_records * sizeof(SrvDone));
    std::memset((void*)s->h_ctl, 0, sizeof(SrvHostCtl));
    s->sub_next = s->done_next = 0;
    HIP_TRY(hipMemcpyAsync(s->arena + s->L.graphs, tab.data(), tab.size() * sizeof(SrvGraph),
                           hipMemcpyHostToDevice, st));
    const uint64_t n_ring = s->c.capacity * s->c.nq;
    hipLaunchKernelGGL(srv_reset_kernel, dim3(init_grid((int64_t)n_ring, s->g[0].num_cu)),
                       dim3(kInitBlock), 0, st, (SrvHeader*)(s->arena + s->L.header),
                       (SrvSlot*)(s->arena + s->L.slots), s->c.slots,
                       (uint64_t*)(s->arena + s->L.rings), n_ring);
    HIP_TRY(hipGetLastError());
    SrvArgs a;
    std::memset(&a, 0, sizeof(a));
    a.hdr = (SrvHeader*)(s->arena + s->L.header);
    a.graphs = (const SrvGraph*)(s->arena + s->L.graphs);
    a.n_graphs = (uint32_t)s->g.size();
    a.n_slots = s->c.slots;
    a.slots = (SrvSlot*)(s->arena + s->L.slots);
    a.rings = (uint64_t*)(s->arena + s->L.rings);
    a.log2cap = log2u(s->c.capacity);
    a.n_queues = s->c.nq;
    HIP_TRY(hipHostGetDevicePointer((void**)&a.sub, s->h_sub, 0));
    HIP_TRY(hipHostGetDevicePointer((void**)&a.done, s->h_done, 0));
    HIP_TRY(hipHostGetDevicePointer((void**)&a.ctl, s->h_ctl, 0));
    HIP_TRY(hipHostGetDevicePointer((void**)&a.snap, s->h_snap, 0));
    a.n_records = s->c.n_records;
    a.fetch = (uint32_t)s->c.fetch;
    a.timeout_ticks = (uint64_t)s->c.timeout_ms * (uint64_t)s->g[0].clock_khz;
    a.push_spin_limit = 200000;
    static std::atomic<uint64_t> launches{0};
    a.epoch = ++launches;
    s->epoch = a.epoch;
    HIP_TRY(hipEventRecord(s->ev0, st));
    atos_status r;
    switch (s->c.worker) {
        case 64: r = launch_daemon<64>(s->g[0], s->c, a, st, &s->grid); break;
        case 128: r = launch_daemon<128>(s->g[0], s->c, a, st, &s->grid); break;
        case 256: r = launch_daemon<256>(s->g[0], s->c, a, st, &s->grid); break;
        case 512: r = launch_daemon<512>(s->g[0], s->c, a, st, &s->grid); break;
        default: r = launch_daemon<1024>(s->g[0], s->c, a, st, &s->grid); break;
    }
    if (r != ATOS_OK) return r;
    HIP_TRY(hipEventRecord(s->ev1, st));
    s->stream = st;
    s->running = true;
    s->stopping = false;
    return ATOS_OK;
}

atos_status atos_server_submit(atos_server_t s, const atos_query* q, uint64_t* query_id) {
    if (!s || !q || !query_id) return ATOS_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    if (!s->running || s->stopping) return ATOS_EINVAL;
    if (q->graph < 0 || (size_t)q->graph >= s->g.size()) return ATOS_EINVAL;
    const GraphRec& g = s->g[(size_t)q->graph];
    if (q->source < 0 || q->source >= g.n) return ATOS_EINVAL;
    if (q->app == ATOS_APP_PAGERANK) {
        if (!(g.flags & ATOS_GRAPH_SYMMETRIC)) return ATOS_ENOTSYMMETRIC;
        if (!(q->damping > 0.0f && q->damping < 1.0f) || !(q->epsilon > 0.0f)) return ATOS_EINVAL;
    } else if (q->app != ATOS_APP_BFS) {
        return ATOS_EINVAL;
    }
    const uint64_t ring = 2ull * (uint64_t)g.n;
    const size_t bytes = state_bytes(q->app, g.n);
    size_t off = 0;
    uint32_t slot = 0;
    if (!s->adm.admit(ring, bytes, slot, off)) return ATOS_EAGAIN;
    const uint64_t id = s->next_id++;
    s->queries[id] = atos_server::Query{q->tag, slot, q->app, q->graph, off, bytes, ring, false};
    SrvSubmit* rec = &s->h_sub[s->sub_next & (s->c.n_records - 1u)];
    rec->query_id = id;
    rec->state = (uint64_t)(uintptr_t)(s->arena + off);
    rec->slot = slot;
    rec->graph = (uint32_t)q->graph;
    rec->app = (uint32_t)q->app;
    rec->source = (uint32_t)q->source;
    rec->damping = q->damping;
    rec->eps = q->epsilon;
    rec->out = 0;
    if (q->out) {
        void* dp = q->out;  // pinned host memory is addressed through its device mapping
        if (hipHostGetDevicePointer(&dp, q->out, 0) != hipSuccess) dp = q->out;
        rec->out = (uint64_t)(uintptr_t)dp;
    }
    __atomic_store_n(&rec->seq, s->sub_next + 1, __ATOMIC_RELEASE);  // fields before seq
    ++s->sub_next;
    *query_id = id;
    return ATOS_OK;
}

atos_status atos_server_poll(atos_server_t s, atos_completion* out, int32_t max, int32_t* n_out) {
    if (!s || !n_out || max < 0 || (max > 0 && !out)) return ATOS_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    int32_t n = 0;
    while (n < max) {
        SrvDone* rec = &s->h_done[s->done_next & (s->c.n_records - 1u)];
        if (__atomic_load_n(&rec->seq, __ATOMIC_ACQUIRE) != s->done_next + 1) break;
        const uint64_t id = rec->query_id;
        auto it = s->queries.find(id);
        ++s->done_next;
        if (it == s->queries.end()) return ATOS_EHIP;  // not a query of this server
        atos_server::Query& Q = it->second;
        Q.done = true;
        atos_completion& c = out[n++];
        c.query_id = id;
        c.tag = Q.tag;
        c.status = rec->status == 0u ? ATOS_OK : ATOS_EHIP;
        c.app = Q.app;
        c.graph = Q.graph;
        c.reserved = 0;
        c.state_offset = Q.off;
        c.tasks = rec->tasks;
        c.edges = rec->edges;
        c.device_us = (double)(rec->t_done - rec->t_admit) * 1000.0 / (double)s->g[0].clock_khz;
    }
    *n_out = n;
    if (n == 0) {
        // the daemon ended on an error: no further completion will come
        const uint32_t bits = __atomic_load_n(&s->h_ctl->status, __ATOMIC_ACQUIRE);
        if (bits & kStatusCorrupt) return ATOS_EHIP;
        if (bits & kStatusOverflow) return ATOS_EOVERFLOW;
        if (bits & kStatusTimeout) return ATOS_ETIMEOUT;
    }
    return ATOS_OK;
}

atos_status atos_server_release(atos_server_t s, uint64_t query_id) {
    if (!s) return ATOS_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->queries.find(query_id);
    if (it == s->queries.end() || !it->second.done) return ATOS_EINVAL;
    const atos_server::Query& Q = it->second;
    s->adm.release(Q.slot, Q.ring, Q.off, Q.bytes);
    s->queries.erase(it);
    return ATOS_OK;
}

atos_status atos_server_stop(atos_server_t s, atos_stats* st) {
    if (!s) return ATOS_EINVAL;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        if (!s->running) return ATOS_EINVAL;
        s->stopping = true;
        __atomic_store_n(&s->h_ctl->stop, 1u, __ATOMIC_RELEASE);
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::lock_guard<std::mutex> lock(s->mu);
    s->running = false;
    SrvHeader h;
    HIP_TRY(hipMemcpyAsync(&h, s->arena + s->L.header, sizeof(h), hipMemcpyDeviceToHost, s->aux));
    HIP_TRY(hipStreamSynchronize(s->aux));
    const uint32_t bits = h.status & ~kStatusStopped;
    atos_status r = ATOS_OK;
    if (bits & kStatusCorrupt) r = ATOS_EHIP;
    else if (bits & kStatusOverflow) r = ATOS_EOVERFLOW;
    else if (bits & kStatusTimeout) r = ATOS_ETIMEOUT;
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->status = r;
        st->tasks_popped = h.stat_popped;
        st->tasks_pushed = h.stat_pushed;
        st->edges_scanned = h.stat_edges;
        st->rounds = h.completed;
        st->push_retries = h.stat_push_retries;
        st->idle_iterations = h.stat_idle;
        st->steals = h.stat_steals;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, s->ev0, s->ev1);
        st->device_ms = ms;
        st->kernel_ms = ms;
    }
    return r;
}

atos_status atos_server_snapshot(atos_server_t s, int32_t ring_words, uint64_t* out,
                                 int64_t max_words, int64_t* n_words) {
    if (!s || !out || !n_words || ring_words < 0 || ring_words > (int32_t)kSrvSnapRingWords)
        return ATOS_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    if (!s->running) return ATOS_EINVAL;
    const int64_t need = 15 + 3ll * s->c.nq + 4ll * s->c.slots + (int64_t)ring_words * s->c.nq;
    if (max_words < need) return ATOS_EINVAL;
    // ask a worker of the daemon for a copy (a copy on another stream could
    // share the daemon's hardware queue and wait for it to end)
    const uint32_t req = __atomic_add_fetch(&s->h_ctl->snap_req, 1u, __ATOMIC_RELEASE);
    const auto t0 = std::chrono::steady_clock::now();
    while (__atomic_load_n(&s->h_ctl->snap_done, __ATOMIC_ACQUIRE) != req) {
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(5)) return ATOS_ETIMEOUT;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    const uint64_t* d = s->h_snap;
    int64_t w = 0;
    for (int i = 0; i < 11; ++i) out[w++] = d[i];  // status .. t_timeout
    out[w++] = (uint64_t)s->g[0].clock_khz;
    out[w++] = s->epoch;
    out[w++] = d[11];  // epoch that started
    out[w++] = d[12];  // epoch that timed out
    const uint64_t* r = d + 13;
    for (uint32_t q = 0; q < s->c.nq; ++q)
        for (int k = 0; k < 3; ++k) out[w++] = *r++;
    for (uint32_t sl = 0; sl < s->c.slots; ++sl)
        for (int k = 0; k < 4; ++k) out[w++] = *r++;
    for (uint32_t q = 0; q < s->c.nq; ++q)
        for (uint32_t i = 0; i < kSrvSnapRingWords; ++i, ++r)
            if ((int32_t)i < ring_words) out[w++] = *r;
    *n_words = w;
    return ATOS_OK;
}

atos_status atos_host_alloc(size_t bytes, void** out) {
    if (!out || bytes == 0) return ATOS_EINVAL;
    *out = nullptr;
    HIP_TRY(hipHostMalloc(out, bytes, hipHostMallocCoherent | hipHostMallocMapped));
    return ATOS_OK;
}

atos_status atos_host_free(void* p) {
    if (!p) return ATOS_EINVAL;
    HIP_TRY(hipHostFree(p));
    return ATOS_OK;
}

atos_status atos_server_destroy(atos_server_t s) {
    if (!s) return ATOS_EINVAL;
    if (s->running) (void)atos_server_stop(s, nullptr);
    free_host(s);
    delete s;
    return ATOS_OK;
}

}  // extern "C"
