// Serving daemon: one persistent worker kernel that stays resident and runs
// BFS and personalized PageRank queries on a set of resident graphs as they
// arrive (continuous batching on the worklist of section 3).
//
// The host writes a query record into a submit ring in host memory; an idle
// worker admits it into a free query slot: it fills the slot's entry and
// pushes the query's state-initialisation tasks (one per chunk of vertices)
// into the same worklist that carries every running query's vertex tasks.
// The last initialisation task of a query pushes its start task (the BFS
// source, or the PageRank source with residue 1 - damping).  Every task
// carries its query slot, so one popped batch can mix queries and graphs.
// Each slot counts its tasks in flight (`pending`): children are counted
// before they are published and a task is uncounted after its children, so
// pending reaches zero exactly once, when the query is complete; the worker
// that brings it there writes a completion record into a ring in host
// memory.  The kernel ends when the host has asked it to stop and every
// admitted query is complete, on error, or at its deadline.
//
// A query submitted with an output buffer (device-accessible host memory)
// gets its result written there by finalisation tasks (one per chunk of
// vertices) once its last task is done; the last of them posts the
// completion, so the host reads the result with no GPU call of its own (a
// copy on another stream could share the daemon's hardware queue and wait
// behind it).
//
// Per-query state is reused memory, so every read of it is an agent-scope
// (coherent) load: a plain load could hit a line a previous query left in
// this XCD's L2.
#pragma once

#include "atos_device.h"
#include "atos_persistent.h"

namespace atos {

// Task payload (the 48 payload bits of a ring word):
//   [47:37] query slot  [36:35] kind  [34:10] vertex or chunk  [9:0] BFS depth tag
constexpr uint32_t kSrvSlotBits = 11;
constexpr uint32_t kSrvMaxSlots = 1u << kSrvSlotBits;
constexpr uint32_t kSrvVertexBits = 25;
constexpr uint64_t kSrvMaxVertices = 1ull << kSrvVertexBits;
constexpr uint32_t kSrvTagMask = 0x3FFu;
enum : uint32_t { kSrvBfs = 0u, kSrvPpr = 1u, kSrvInit = 2u, kSrvFinal = 3u };
constexpr uint32_t kSrvChunk = 16384;  // vertices initialised (or finalised) by one task
constexpr uint32_t kStatusStopped = 16u;  // normal end: stop requested, all queries done

ATOS_DEV uint64_t srv_payload(uint32_t slot, uint32_t kind, uint32_t v, uint32_t tag) {
    return ((uint64_t)slot << 37) | ((uint64_t)kind << 35) | ((uint64_t)v << 10) |
           (uint64_t)(tag & kSrvTagMask);
}
ATOS_DEV uint32_t srv_slot(uint64_t w) { return (uint32_t)(w >> 37) & (kSrvMaxSlots - 1u); }
ATOS_DEV uint32_t srv_kind(uint64_t w) { return (uint32_t)(w >> 35) & 3u; }
ATOS_DEV uint32_t srv_vertex(uint64_t w) { return (uint32_t)(w >> 10) & (uint32_t)(kSrvMaxVertices - 1u); }
ATOS_DEV uint32_t srv_tag(uint64_t w) { return (uint32_t)w & kSrvTagMask; }

// A resident graph (written before the daemon starts, constant while it runs).
struct SrvGraph {
    const void* offs;
    const int32_t* cols;
    int64_t n;
    uint32_t offs64;
    uint32_t pad;
};

// Query record in host memory, written by the host; `seq` (= record index
// + 1) is written last and marks the record ready.
struct alignas(64) SrvSubmit {
    uint64_t query_id;
    uint64_t state;  // device address of the query's state
    uint32_t slot, graph, app, source;
    float damping, eps;
    uint64_t out;    // device address of the result buffer, 0 = none
    uint64_t seq;
};

// Completion record in host memory, written by the device; `seq` last.
struct alignas(64) SrvDone {
    uint64_t query_id;
    uint32_t slot, status;
    uint64_t tasks, edges;
    uint64_t t_admit, t_done;  // device wall-clock ticks
    uint64_t seq;
};

// Host-memory control word.
struct alignas(64) SrvHostCtl {
    uint32_t stop;       // set by the host: end once every admitted query is complete
    uint32_t status;     // set by the device when the daemon ends on an error (kStatus* bits)
    uint32_t snap_req;   // host: snapshot requests made
    uint32_t snap_done;  // device: snapshot requests served (written after the snapshot)
    uint32_t pad[12];
};

// One query slot (device memory).
struct alignas(128) SrvSlot {
    uint64_t state;
    uint64_t query_id;
    uint32_t graph, app, source, n_chunks;
    double damping, eps;
    uint64_t t_admit;
    uint64_t out;        // result buffer (0 = none)
    uint64_t pad0[8];
    uint64_t pending;    // tasks of the query reserved and not finished
    uint64_t init_left;  // initialisation tasks not finished
    uint64_t tasks, edges;
    uint64_t fin_left;   // finalisation tasks not finished
    uint64_t pad1[11];
};
static_assert(sizeof(SrvSlot) == 256, "slot size");

// Daemon control block (device memory).
struct alignas(256) SrvHeader {
    uint32_t status;  // kStatus* bits; kStatusStopped on a normal end
    uint32_t pad0;
    uint64_t submit_head;  // next submit record to admit
    uint64_t comp_tail;    // next completion record to write
    uint64_t active;       // admitted, not completed queries
    uint64_t admitted, completed;
    uint64_t stat_popped, stat_pushed, stat_edges, stat_idle, stat_steals, stat_push_retries;
    uint64_t t_start;    // device clock when the daemon started (first worker to run)
    uint64_t t_timeout;  // device clock when a worker found the deadline passed
    uint64_t epoch;      // launch number of the daemon that wrote t_start
    uint64_t epoch_timeout;  // launch number of the daemon that wrote t_timeout
    uint32_t snap_served;    // snapshot requests taken by a worker
    uint32_t pad2;
    uint64_t pad1[15];
    QueueCtl q[kMaxQueues];
};

struct SrvArgs {
    SrvHeader* hdr;
    const SrvGraph* graphs;
    uint32_t n_graphs;
    uint32_t n_slots;
    SrvSlot* slots;
    uint64_t* rings;
    uint32_t log2cap;
    uint32_t n_queues;
    SrvSubmit* sub;      // host memory, n_records entries
    SrvDone* done;       // host memory, n_records entries
    SrvHostCtl* ctl;     // host memory
    uint32_t n_records;  // power of two
    uint32_t fetch;
    uint64_t bulk_margin;
    uint32_t fetch_share;  // workers per ring: a pop takes its share of what the ring holds
    uint32_t push_shallow; // 1: publish into the shallowest ring (as last probed), 0: own ring
    uint32_t push_query;   // 1: publish every task into the ring of its query's slot
    uint64_t steal_min;    // take from another ring only when it holds at least this many
    uint64_t timeout_ticks;
    uint32_t push_spin_limit;
    uint32_t poll_every;  // workers with blockIdx % poll_every == 0 poll for new queries
    uint64_t epoch;       // launch number (diagnostics)
    uint64_t* snap;       // host memory: snapshot words (see srv_snapshot)
};

template <class T>
ATOS_DEV T ld_sys(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
template <class T>
ATOS_DEV void st_sys(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

constexpr uint32_t kSrvLdsGraphs = 64;  // graph table entries the daemon keeps in LDS

ATOS_DEV int64_t srv_offset(const SrvGraph& G, uint32_t v) {
    return G.offs64 ? ((const int64_t*)G.offs)[v] : (int64_t)((const int32_t*)G.offs)[v];
}

constexpr uint32_t kSrvSnapRingWords = 8;

// Words of a snapshot (host memory, written by one thread): status,
// submit_head, comp_tail, active, admitted, completed, rings, ring capacity,
// slots, t_start, t_timeout, epoch, epoch_timeout; per ring head, tail, done;
// per slot query_id, pending, init_left, app << 32 | graph; then
// kSrvSnapRingWords slot words of every ring from its head.
ATOS_DEV void srv_snapshot(const SrvArgs& a) {
    const SrvHeader* H = a.hdr;
    uint64_t* o = a.snap;
    uint64_t w = 0;
    st_sys(o + w++, (uint64_t)ld_agent(&H->status));
    st_sys(o + w++, ld_agent(&H->submit_head));
    st_sys(o + w++, ld_agent(&H->comp_tail));
    st_sys(o + w++, ld_agent(&H->active));
    st_sys(o + w++, ld_agent(&H->admitted));
    st_sys(o + w++, ld_agent(&H->completed));
    st_sys(o + w++, (uint64_t)a.n_queues);
    st_sys(o + w++, (uint64_t)1 << a.log2cap);
    st_sys(o + w++, (uint64_t)a.n_slots);
    st_sys(o + w++, ld_agent(&H->t_start));
    st_sys(o + w++, ld_agent(&H->t_timeout));
    st_sys(o + w++, ld_agent(&H->epoch));
    st_sys(o + w++, ld_agent(&H->epoch_timeout));
    for (uint32_t q = 0; q < a.n_queues; ++q) {
        st_sys(o + w++, ld_agent(&H->q[q].head));
        st_sys(o + w++, ld_agent(&H->q[q].tail));
        st_sys(o + w++, ld_agent(&H->q[q].done));
    }
    for (uint32_t sl = 0; sl < a.n_slots; ++sl) {
        const SrvSlot* S = &a.slots[sl];
        st_sys(o + w++, ld_agent(&S->query_id));
        st_sys(o + w++, ld_agent(&S->pending));
        st_sys(o + w++, ld_agent(&S->init_left));
        st_sys(o + w++, ((uint64_t)ld_agent(&S->app) << 32) | ld_agent(&S->graph));
    }
    const uint64_t mask = (1ull << a.log2cap) - 1ull;
    for (uint32_t q = 0; q < a.n_queues; ++q) {
        const uint64_t h = ld_agent(&H->q[q].head);
        for (uint32_t i = 0; i < kSrvSnapRingWords; ++i)
            st_sys(o + w++, ld_agent(a.rings + ((uint64_t)q << a.log2cap) + ((h + i) & mask)));
    }
}

// Post the completion of the query in slot `sl` (one thread).
ATOS_DEV void srv_complete(const SrvArgs& a, uint32_t sl) {
    SrvHeader* H = a.hdr;
    SrvSlot* S = &a.slots[sl];
    const uint64_t idx = add_agent(&H->comp_tail, (uint64_t)1);
    SrvDone* D = &a.done[idx & (a.n_records - 1u)];
    st_sys(&D->query_id, ld_agent(&S->query_id));
    st_sys(&D->slot, sl);
    st_sys(&D->status, 0u);
    st_sys(&D->tasks, ld_agent(&S->tasks));
    st_sys(&D->edges, ld_agent(&S->edges));
    st_sys(&D->t_admit, ld_agent(&S->t_admit));
    st_sys(&D->t_done, now_ticks());
    __hip_atomic_store(&D->seq, idx + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    add_agent(&H->completed, (uint64_t)1);
    add_agent(&H->active, ~(uint64_t)0);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void serve_kernel(SrvArgs a) {
    constexpr int PUSH_CAP = (2 * BLOCK < 512) ? 512 : 2 * BLOCK;
    constexpr int NW = BLOCK / kWave;

    __shared__ uint32_t s_slot[BLOCK];
    __shared__ uint32_t s_kind[BLOCK];
    __shared__ uint32_t s_vert[BLOCK];
    __shared__ uint32_t s_val[BLOCK];   // BFS: depth of the neighbours (d + 1)
    __shared__ uint32_t s_deg[BLOCK];
    __shared__ uint32_t s_active[BLOCK];
    __shared__ int64_t s_start[BLOCK];
    __shared__ const int32_t* s_cols[BLOCK];
    __shared__ uint64_t s_state[BLOCK];  // BFS: depth array; PageRank: residue array
    __shared__ uint64_t s_acc[BLOCK];    // PageRank: push amount (FP64 bits)
    __shared__ double s_eps[BLOCK];
    __shared__ uint32_t s_scan[BLOCK + 1];
    __shared__ uint64_t s_push[PUSH_CAP];
    __shared__ uint32_t s_wsum[NW + 1];
    __shared__ uint32_t s_push_n;
    __shared__ uint32_t s_k;
    __shared__ uint32_t s_stop;
    __shared__ PopLds s_pop;
    __shared__ uint32_t s_admit;  // admitted a query this iteration
    __shared__ SrvSubmit s_rec;   // its record
    __shared__ uint64_t s_ist;    // init / finalise: state address of the chunk's query
    __shared__ uint64_t s_iout;   // finalise: its result buffer
    __shared__ uint32_t s_iapp;
    __shared__ int64_t s_in;
    __shared__ uint32_t s_fin[BLOCK];  // queries whose last task finished in this batch
    __shared__ uint32_t s_nfin;
    __shared__ SrvGraph s_graphs[kSrvLdsGraphs];  // the first graphs of the (immutable) table
    __shared__ uint32_t s_ucnt[kSrvMaxSlots];  // per query: tasks of this batch (zero between batches)
    __shared__ uint64_t s_uedg[kSrvMaxSlots];  // per query: edges of this batch

    const int tid = threadIdx.x;
    SrvHeader* H = a.hdr;
    const uint32_t F = a.fetch;
    const uint32_t NQ = a.n_queues;
    const uint32_t my_q = xcc_id() % NQ;
    __shared__ uint32_t s_push_q;  // ring the current flush publishes into (one-ring flushes)
    __shared__ uint32_t s_qcnt[kMaxQueues];  // tasks of the current flush per ring
    __shared__ uint64_t s_qbase[kMaxQueues]; // their first reserved position per ring
    Deadline deadline;  // checked by thread 0 only
    deadline.start(a.timeout_ticks);
    const uint64_t t0 = deadline.last;
    const bool poller = (blockIdx.x % a.poll_every) == 0u;
    if (tid == 0 && blockIdx.x == 0) {
        st_agent(&H->t_start, t0);
        st_agent(&H->epoch, a.epoch);
    }

    if (tid == 0) {
        s_push_n = 0;
        s_k = 0;
        s_nfin = 0;
    }
    if ((uint32_t)tid < (uint32_t)kMaxQueues) {  // no probe yet: every ring counts as empty
        s_pop.head[tid] = 0;
        s_pop.tail[tid] = 0;
    }
    for (uint32_t i = tid; i < kSrvMaxSlots; i += BLOCK) {
        s_ucnt[i] = 0u;
        s_uedg[i] = 0ull;
    }
    for (uint32_t i = tid; i < kSrvLdsGraphs && i < a.n_graphs; i += BLOCK) s_graphs[i] = a.graphs[i];
    uint32_t spin = 0, iter = 0;
    bool was_idle = true;
    uint64_t st_pop = 0, st_push = 0, st_edges = 0, st_idle = 0, st_steal = 0;

    // Publish s_push into this XCD's ring.  With count_pending, every task is
    // first counted in its query's pending counter (before it can be popped).
    auto flush = [&](bool count_pending) {
        __syncthreads();
        const uint32_t n = s_push_n;
        if (n == 0) return;
        if (count_pending) {
            for (uint32_t b = 0; b < n; b += BLOCK) {
                const uint32_t i = b + (uint32_t)tid;
                const bool has = i < n;
                const uint32_t sl = has ? srv_slot(s_push[i]) : 0u;
                uint64_t m = ballot(has);
                while (m) {  // one atomic per distinct slot in the wavefront
                    const int leader = __builtin_ctzll(m);
                    const uint32_t ls = __shfl(sl, leader, kWave);
                    const uint64_t same = ballot(has && sl == ls) & m;
                    if (lane_id() == (uint32_t)leader) add_agent(&a.slots[ls].pending, (uint64_t)__popcll(same));
                    m &= ~same;
                }
            }
        }
        // target ring of every task, and its rank among this flush's tasks for
        // that ring (a thread handles tasks tid, tid + BLOCK, ...)
        constexpr uint32_t PER = (PUSH_CAP + BLOCK - 1) / BLOCK;
        uint32_t rank[PER], ring[PER];
        if ((uint32_t)tid < (uint32_t)kMaxQueues) s_qcnt[tid] = 0u;
        __syncthreads();
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t i = j * BLOCK + (uint32_t)tid;
            ring[j] = 0u;
            rank[j] = i;
            if (a.push_query && i < n) {
                ring[j] = srv_slot(s_push[i]) % NQ;
                rank[j] = atomicAdd(&s_qcnt[ring[j]], 1u);
            }
        }
        wait_vmem();  // counters and task data complete before any task is published
        __syncthreads();
        if (a.push_query) {
            if ((uint32_t)tid < NQ && s_qcnt[tid] != 0u)
                s_qbase[tid] = add_agent(&H->q[tid].tail, (uint64_t)s_qcnt[tid]);
        } else if (tid == 0) {
            uint32_t pq = my_q;
            if (a.push_shallow) pq = (my_q + shallowest_ring(s_pop, NQ)) % NQ;
            s_push_q = pq;
            s_qbase[pq] = add_agent(&H->q[pq].tail, (uint64_t)n);
        }
        __syncthreads();
        uint64_t retries = 0;
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t i = j * BLOCK + (uint32_t)tid;
            if (i >= n) continue;
            const uint32_t r = a.push_query ? ring[j] : s_push_q;
            RingView R;
            R.slots = a.rings + ((uint64_t)r << a.log2cap);
            R.mask = (1ull << a.log2cap) - 1ull;
            R.log2cap = a.log2cap;
            const uint64_t pos = s_qbase[r] + rank[j];
            const uint64_t want = R.free_word(pos);
            const uint64_t full = R.full_word(pos, s_push[i]);
            uint32_t tries = 0;
            while (!cas_agent(R.slot(pos), want, full)) {
                ++retries;
                if (ld_agent(&H->status) != 0u) break;
                if (++tries > a.push_spin_limit) {
                    or_agent(&H->status, (uint32_t)kStatusOverflow);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (retries) add_agent(&H->stat_push_retries, retries);
        if (tid == 0) st_push += n;
        __syncthreads();
        if (tid == 0) s_push_n = 0;
        __syncthreads();
    };
    auto nearly_full = [&]() -> bool {
        __syncthreads();
        return __syncthreads_or(tid == 0 && s_push_n + BLOCK > (uint32_t)PUSH_CAP) != 0;
    };
    auto append = [&](bool push, uint64_t payload) {
        const uint64_t m = ballot(push);
        if (m) {
            uint32_t wbase = 0;
            if (lane_id() == (uint32_t)__builtin_ctzll(m))
                wbase = atomicAdd(&s_push_n, (uint32_t)__popcll(m));
            wbase = __shfl(wbase, __builtin_ctzll(m), kWave);
            if (push) s_push[wbase + mbcnt(m)] = payload;
        }
    };
    // the run ends: stop requested, every admitted query complete, no record waiting
    auto drained = [&]() -> bool {
        if (ld_sys(&a.ctl->stop) == 0u) return false;
        if (ld_agent(&H->active) != 0ull) return false;
        const uint64_t h = ld_agent(&H->submit_head);
        return ld_sys(&a.sub[h & (a.n_records - 1u)].seq) != h + 1ull;
    };

    __syncthreads();
    for (;; ++iter) {
        // ---- admission: take the next submit record, if one is ready
        if (tid == 0) {
            s_admit = 0u;
            s_stop = 0u;
            // (a busy worker looks at the status word every 8th batch; the pop
            // and idle paths look at it too)
            if ((was_idle || (iter & 7u) == 0u) && ld_agent(&H->status) != 0u) {
                s_stop = 1u;
            } else if (deadline.passed()) {
                st_agent(&H->t_timeout, now_ticks());
                st_agent(&H->epoch_timeout, a.epoch);
                or_agent(&H->status, (uint32_t)kStatusTimeout);
                s_stop = 1u;
            } else if (poller && (was_idle || (iter & 7u) == 0u)) {
                const uint32_t want = ld_sys(&a.ctl->snap_req);
                const uint32_t served = ld_agent(&H->snap_served);
                if (want != served && cas_agent(&H->snap_served, served, want)) {
                    srv_snapshot(a);
                    __hip_atomic_store(&a.ctl->snap_done, want, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_SYSTEM);
                }
                const uint64_t h = ld_agent(&H->submit_head);
                SrvSubmit* r = &a.sub[h & (a.n_records - 1u)];
                if (ld_sys(&r->seq) == h + 1ull && cas_agent(&H->submit_head, h, h + (uint64_t)1)) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // record fields after its seq
                    s_rec.query_id = ld_sys(&r->query_id);
                    s_rec.state = ld_sys(&r->state);
                    s_rec.slot = ld_sys(&r->slot);
                    s_rec.graph = ld_sys(&r->graph);
                    s_rec.app = ld_sys(&r->app);
                    s_rec.source = ld_sys(&r->source);
                    s_rec.damping = ld_sys(&r->damping);
                    s_rec.eps = ld_sys(&r->eps);
                    s_rec.out = ld_sys(&r->out);
                    s_admit = 1u;
                    if (s_rec.slot >= a.n_slots || s_rec.graph >= a.n_graphs ||
                        (int64_t)s_rec.source >= a.graphs[s_rec.graph].n ||
                        (s_rec.app != (uint32_t)ATOS_APP_BFS && s_rec.app != (uint32_t)ATOS_APP_PAGERANK)) {
                        or_agent(&H->status, (uint32_t)kStatusCorrupt);  // the host validates records
                        s_admit = 0u;
                        s_stop = 1u;
                    }
                }
            }
        }
        __syncthreads();
        if (s_stop) break;
        if (s_admit) {
            const int64_t n = a.graphs[s_rec.graph].n;
            const uint32_t n_chunks = (uint32_t)((n + kSrvChunk - 1) / kSrvChunk);
            const uint32_t slot = s_rec.slot;
            if (tid == 0) {
                SrvSlot* S = &a.slots[slot];
                st_agent(&S->state, s_rec.state);
                st_agent(&S->query_id, s_rec.query_id);
                st_agent(&S->graph, s_rec.graph);
                st_agent(&S->app, s_rec.app);
                st_agent(&S->source, s_rec.source);
                st_agent(&S->n_chunks, n_chunks);
                st_agent(&S->damping, (double)s_rec.damping);
                st_agent(&S->eps, (double)s_rec.eps);
                st_agent(&S->t_admit, now_ticks());
                st_agent(&S->out, s_rec.out);
                st_agent(&S->tasks, (uint64_t)0);
                st_agent(&S->edges, (uint64_t)0);
                st_agent(&S->init_left, (uint64_t)n_chunks);
                st_agent(&S->pending, (uint64_t)n_chunks);  // the init tasks pushed below
                add_agent(&H->active, (uint64_t)1);
                add_agent(&H->admitted, (uint64_t)1);
            }
            for (uint32_t b = 0; b < n_chunks; b += BLOCK) {
                const uint32_t c = b + (uint32_t)tid;
                append(c < n_chunks, srv_payload(slot, kSrvInit, c, 0u));
                if (nearly_full()) flush(false);
            }
            flush(false);
        }

        // ---- pop
        auto stop_wait = [&](uint32_t wait) -> bool {
            if (ld_agent(&H->status) != 0u) return true;
            if (deadline.passed()) {
                st_agent(&H->t_timeout, now_ticks());
                st_agent(&H->epoch_timeout, a.epoch);
                or_agent(&H->status, (uint32_t)kStatusTimeout);
                return true;
            }
            if ((wait & 255u) == 0u && drained()) {
                or_agent(&H->status, kStatusStopped);
                return true;
            }
            return false;
        };
        uint64_t word = 0;
        bool got = pop_tasks<BLOCK>(H->q, a.rings, a.log2cap, NQ, my_q, F, a.bulk_margin, a.fetch_share,
                                    false, a.steal_min, s_pop,
                                    word, st_steal, stop_wait);
        if (s_pop.stop) break;
        if (tid == 0) s_k = 0;
        __syncthreads();
        if (got) {
            const uint32_t idx = atomicAdd(&s_k, 1u);
            s_slot[idx] = srv_slot(word);
            s_kind[idx] = srv_kind(word);
            s_vert[idx] = srv_vertex(word);
            s_val[idx] = srv_tag(word);
        }
        __syncthreads();
        const uint32_t k = s_k;
        if (k == 0) {
            // ---- idle: stop on error, at the deadline, or once drained
            was_idle = true;
            if (tid == 0) {
                ++st_idle;
                uint32_t stop = 0;
                if (ld_agent(&H->status) != 0u) {
                    stop = 1;
                } else if (deadline.passed()) {
                    st_agent(&H->t_timeout, now_ticks());
                st_agent(&H->epoch_timeout, a.epoch);
                    or_agent(&H->status, (uint32_t)kStatusTimeout);
                    stop = 1;
                } else if ((st_idle & 15u) == 0u && drained()) {
                    or_agent(&H->status, kStatusStopped);
                    stop = 1;
                }
                s_stop = stop;
            }
            __syncthreads();
            if (s_stop) break;
            backoff(spin);
            // pollers keep checking for new queries at a short interval
            if (poller && spin > 64) spin = 64;
            continue;
        }
        was_idle = false;
        spin = 0;

        // ---- initialisation and finalisation tasks: the whole worker takes
        //      each chunk (fill the state, or copy the result out)
        if (__syncthreads_or((uint32_t)tid < k && s_kind[tid] >= kSrvInit)) {
            for (uint32_t i = 0; i < k; ++i) {
                if (s_kind[i] < kSrvInit) continue;
                if (tid == 0) {
                    const SrvSlot* S = &a.slots[s_slot[i]];
                    s_ist = ld_agent(&S->state);
                    s_iout = ld_agent(&S->out);
                    s_iapp = ld_agent(&S->app);
                    s_in = a.graphs[ld_agent(&S->graph)].n;
                }
                __syncthreads();
                const int64_t v0 = (int64_t)s_vert[i] * kSrvChunk;
                const int64_t v1 = v0 + kSrvChunk < s_in ? v0 + kSrvChunk : s_in;
                const bool bfs = s_iapp == (uint32_t)ATOS_APP_BFS;
                if (s_kind[i] == kSrvInit) {
                    if (bfs) {
                        uint32_t* depth = (uint32_t*)s_ist;
                        for (int64_t v = v0 + tid; v < v1; v += BLOCK) st_agent(depth + v, 0xFFFFFFFFu);
                    } else {
                        double* rank = (double*)s_ist;
                        double* residue = rank + s_in;
                        for (int64_t v = v0 + tid; v < v1; v += BLOCK) {
                            st_agent(rank + v, 0.0);
                            st_agent(residue + v, 0.0);
                        }
                    }
                } else if (bfs) {  // result: int32 depths (unreached = -1)
                    const uint32_t* depth = (const uint32_t*)s_ist;
                    uint32_t* out = (uint32_t*)s_iout;
                    for (int64_t v = v0 + tid; v < v1; v += BLOCK) st_sys(out + v, ld_agent(depth + v));
                } else {  // result: FP32 ranks, then FP32 residues
                    const double* rank = (const double*)s_ist;
                    float* out = (float*)s_iout;
                    for (int64_t v = v0 + tid; v < v1; v += BLOCK) {
                        st_sys(out + v, (float)ld_agent(rank + v));
                        st_sys(out + s_in + v, (float)ld_agent(rank + s_in + v));
                    }
                }
                __syncthreads();
            }
            wait_vmem();  // this worker's fills and copies are complete before its chunks are counted
            __syncthreads();
            if ((uint32_t)tid < k && s_kind[tid] == kSrvFinal &&
                add_agent(&a.slots[s_slot[tid]].fin_left, ~(uint64_t)0) == (uint64_t)1)
                srv_complete(a, s_slot[tid]);  // last chunk of the result: post the completion
            bool push = false;
            uint64_t payload = 0;
            if ((uint32_t)tid < k && s_kind[tid] == kSrvInit) {
                SrvSlot* S = &a.slots[s_slot[tid]];
                if (add_agent(&S->init_left, ~(uint64_t)0) == (uint64_t)1) {
                    // last chunk of the query: its start task
                    const uint32_t src = ld_agent(&S->source);
                    const uint64_t st = ld_agent(&S->state);
                    if (ld_agent(&S->app) == (uint32_t)ATOS_APP_BFS) {
                        st_agent((uint32_t*)st + src, 0u);
                        payload = srv_payload(s_slot[tid], kSrvBfs, src, 0u);
                    } else {
                        const int64_t n = a.graphs[ld_agent(&S->graph)].n;
                        st_agent((double*)st + n + src, 1.0 - ld_agent(&S->damping));
                        payload = srv_payload(s_slot[tid], kSrvPpr, src, 0u);
                    }
                    push = true;
                }
            }
            append(push, payload);
        }

        // ---- per vertex task: neighbour range and the application's prepare
        if ((uint32_t)tid < k) {
            bool active = false;
            uint32_t deg = 0;
            const uint32_t kind = s_kind[tid];
            if (kind < kSrvInit) {
                const SrvSlot* S = &a.slots[s_slot[tid]];
                const uint32_t gi = ld_agent(&S->graph);
                const SrvGraph G = gi < kSrvLdsGraphs ? s_graphs[gi] : a.graphs[gi];
                const uint32_t v = s_vert[tid];
                if ((int64_t)v >= G.n) {
                    or_agent(&H->status, (uint32_t)kStatusCorrupt);  // never dereference it
                } else {
                    const int64_t beg = srv_offset(G, v), end = srv_offset(G, v + 1);
                    deg = (uint32_t)(end - beg);
                    s_start[tid] = beg;
                    s_cols[tid] = G.cols;
                    const uint64_t st = ld_agent(&S->state);
                    if (kind == kSrvBfs) {
                        uint32_t* depth = (uint32_t*)st;
                        const uint32_t d = ld_agent(depth + v);
                        active = (d & kSrvTagMask) == s_val[tid] && deg > 0;  // else a stale duplicate
                        s_val[tid] = d + 1u;
                        s_state[tid] = st;
                    } else {
                        double* rank = (double*)st;
                        double* residue = rank + G.n;
                        const double r = exch_agent(residue + v, 0.0);
                        if (r > 0.0) {
                            add_agent(rank + v, r);
                            if (deg > 0) {
                                s_acc[tid] = (uint64_t)__double_as_longlong(ld_agent(&S->damping) * r / (double)deg);
                                s_eps[tid] = ld_agent(&S->eps);
                                s_state[tid] = (uint64_t)residue;
                                active = true;
                            }
                        }
                    }
                }
            }
            s_deg[tid] = deg;
            s_active[tid] = active ? 1u : 0u;
        }
        __syncthreads();

        // ---- load-balancing search over the batch's edges (tasks of any query)
        {
            const uint32_t cnt = ((uint32_t)tid < k && s_active[tid]) ? s_deg[tid] : 0u;
            uint32_t total;
            const uint32_t ex = block_exclusive_scan<BLOCK>(cnt, s_wsum, total);
            if ((uint32_t)tid < k) s_scan[tid] = ex;
            if (tid == 0) s_scan[k] = total;
            __syncthreads();
            if (tid == 0) st_edges += total;
            const bool may_overflow = s_push_n + total + BLOCK > (uint32_t)PUSH_CAP;
            // EPT edges per thread per step, in phases: neighbour ids, then BFS
            // neighbour depths, then (with no load outstanding) every update, so a
            // thread's atomics are in flight together, then the push decisions
            constexpr int EPT = kEdgesPerThread;
            for (uint32_t eb = 0; eb < total; eb += BLOCK * EPT) {
                uint32_t wv[EPT], iv[EPT], dv[EPT], ub[EPT];
                double up[EPT];
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    const uint32_t e = eb + (uint32_t)(j * BLOCK + tid);
                    iv[j] = 0xFFFFFFFFu;
                    wv[j] = 0u;
                    if (e < total) {
                        const uint32_t i = lbs_search(s_scan, k, e);
                        wv[j] = (uint32_t)s_cols[i][s_start[i] + (int64_t)(e - s_scan[i])];
                        iv[j] = i;
                    }
                }
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    dv[j] = 0u;
                    if (iv[j] != 0xFFFFFFFFu && s_kind[iv[j]] == kSrvBfs)
                        dv[j] = ld_agent((const uint32_t*)s_state[iv[j]] + wv[j]);
                }
                wait_vmem();
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    ub[j] = 0u;
                    up[j] = 0.0;
                    if (iv[j] != 0xFFFFFFFFu) {
                        const uint32_t i = iv[j];
                        if (s_kind[i] == kSrvBfs) {
                            if (s_val[i] < dv[j]) ub[j] = min_agent((uint32_t*)s_state[i] + wv[j], s_val[i]);
                        } else {
                            up[j] = add_agent((double*)s_state[i] + wv[j],
                                              __longlong_as_double((long long)s_acc[i]));
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < EPT; ++j) {
                    bool push = false;
                    uint64_t payload = 0;
                    if (iv[j] != 0xFFFFFFFFu) {
                        const uint32_t i = iv[j];
                        if (s_kind[i] == kSrvBfs) {
                            const uint32_t nd = s_val[i];
                            push = nd < dv[j] && nd < ub[j];
                            payload = srv_payload(s_slot[i], kSrvBfs, wv[j], nd);
                        } else {
                            const double delta = __longlong_as_double((long long)s_acc[i]);
                            push = up[j] <= s_eps[i] && up[j] + delta > s_eps[i];
                            payload = srv_payload(s_slot[i], kSrvPpr, wv[j], 0u);
                        }
                    }
                    append(push, payload);
                    if (may_overflow && nearly_full()) flush(true);
                }
            }
        }
        flush(true);

        // ---- uncount the batch's tasks per query (after their children were
        //      counted and published, and after every update they made completed);
        //      the worker that brings a query's pending to zero completes it
        wait_vmem();
        __syncthreads();
        {
            // Tasks and edges per query of this batch, summed in LDS; the first
            // task of each query in the batch then updates that query's counters,
            // all queries in parallel.  (Finalisation tasks are not counted in
            // pending.)
            const bool has = (uint32_t)tid < k && s_kind[tid] != kSrvFinal;
            const uint32_t sl = has ? s_slot[tid] : 0u;
            bool leader = false;
            if (has) {
                leader = atomicAdd(&s_ucnt[sl], 1u) == 0u;
                if (s_active[tid]) atomicAdd((unsigned long long*)&s_uedg[sl], (unsigned long long)s_deg[tid]);
            }
            __syncthreads();
            if (leader) {
                SrvSlot* S = &a.slots[sl];
                const uint64_t cnt = s_ucnt[sl];
                const uint64_t sum = s_uedg[sl];
                s_ucnt[sl] = 0u;  // clean for the next batch
                s_uedg[sl] = 0ull;
                add_agent(&S->tasks, cnt);
                if (sum) add_agent(&S->edges, sum);
                wait_vmem();
                if (add_agent(&S->pending, (uint64_t)0 - cnt) == cnt) {
                    // the query's last task: copy its result out first, if asked
                    if (ld_agent(&S->out) != 0ull) s_fin[atomicAdd(&s_nfin, 1u)] = sl;
                    else srv_complete(a, sl);
                }
            }
        }
        __syncthreads();
        if (s_nfin) {  // push the finalisation tasks of the queries that just finished
            for (uint32_t f = 0; f < s_nfin; ++f) {
                const uint32_t ls = s_fin[f];
                const uint32_t n_chunks = ld_agent(&a.slots[ls].n_chunks);
                if (tid == 0) st_agent(&a.slots[ls].fin_left, (uint64_t)n_chunks);
                for (uint32_t b = 0; b < n_chunks; b += BLOCK) {
                    const uint32_t c = b + (uint32_t)tid;
                    append(c < n_chunks, srv_payload(ls, kSrvFinal, c, 0u));
                    if (nearly_full()) flush(false);
                }
            }
            flush(false);  // (its wait also completes the fin_left stores before publishing)
            if (tid == 0) s_nfin = 0;
            __syncthreads();
        }
        if (tid == 0) st_pop += k;
        __syncthreads();
    }

    if (tid == 0) {
        add_agent(&H->stat_popped, st_pop);
        add_agent(&H->stat_pushed, st_push);
        add_agent(&H->stat_edges, st_edges);
        if (st_idle) add_agent(&H->stat_idle, st_idle);
        if (st_steal) add_agent(&H->stat_steals, st_steal);
        const uint32_t status = ld_agent(&H->status);
        if (status & ~kStatusStopped) st_sys(&a.ctl->status, status);
    }
}

}  // namespace atos
