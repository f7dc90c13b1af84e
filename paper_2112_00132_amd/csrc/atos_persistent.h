// Persistent worklist kernel (paper section 3, Listing 2; section 3.4).
//
// Every workgroup of the grid is one worker (BLOCK = 64 is the wavefront
// worker, the counterpart of the paper's warp worker; BLOCK = 128..1024 are
// workgroup workers, the counterpart of its CTA worker).  A worker loops:
//
//   claim up to FETCH consecutive positions of this XCD's ring (or, when it
//   is empty, of another XCD's ring) with one atomic on its `head`, take the
//   tasks published there, stage them in LDS and mark the slots FREE for the
//   next lap
//   per task: read its neighbour range, run the application's `prepare`
//   exclusive scan of the tasks' edge counts; load-balancing search maps
//   every edge of the batch to one thread (section 3.3: data parallelism
//   inside the worker on top of task parallelism across workers)
//   per edge: the application's `edge` callback, which may emit a new task
//   new tasks are gathered in LDS with ballot/mbcnt and published into this
//   XCD's ring with one atomic on its `tail` per flush
//   this XCD's `done += tasks taken`
//
// A worker holds no claimed position while it processes tasks: it claims
// either only positions it has seen published (compare-and-swap on head) or,
// when the ring is long, F reserved positions with one atomicAdd and waits
// for their pushers to publish them.  Termination: a ring's `tail` is
// advanced when a task is reserved, before the task that produced it is
// counted in a `done`, so sum(done) == sum(tail) means every task ever
// reserved has been processed and none can appear again; an idle worker
// that observes it (reading all dones first) exits.  Every wait is bounded
// by a device deadline and by the status word.
#pragma once

#include "atos_device.h"

namespace atos {

template <class OffT>
struct PersistArgs {
    const OffT* offs;
    const int32_t* cols;
    int64_t n;
    WsHeader* hdr;
    uint64_t* rings;       // n_queues rings of 2^log2cap slots, back to back
    uint32_t log2cap;
    uint32_t n_queues;     // 1 (one shared ring) or one ring per XCD
    int32_t fetch;         // tasks claimed per pop, 1..BLOCK
    uint32_t split_degree; // tasks with more edges go to the hub board (0 = never)
    uint64_t bulk_margin;  // claim with one atomicAdd when a ring holds at least this many
    uint32_t fetch_share;  // workers sharing a ring (adaptive claims), or 0 (always up to fetch)
    uint32_t discrete;     // 1: one round of a discrete run (take only positions below each
                           // ring's limit, exit when they are taken); 2: rounds inside one
                           // launch (the same limits, advanced by the workers once every
                           // position below them is taken); 0: persistent
    uint32_t push_shallow; // 1: publish into the shallowest ring (as last probed), 0: own ring
    uint32_t segmented;    // 1: publish every task into the ring of its vertex's segment
    uint32_t seg_bound[kMaxQueues - 1];  // first vertex of segments 1..7 (segmented)
    uint32_t push_spin_limit;
    uint64_t n_init;       // initial tasks, dealt round-robin over the rings (seed_tasks_kernel)
    uint64_t timeout_ticks;
    TraceBuf* trace;       // per-batch event records, or null
    const uint32_t* abort_flag;  // host word that stops the run when non-zero, or null
    uint32_t comb_flush_edges;   // combining: flush a worker's table after this many edges

    ATOS_DEV RingView ring_of(uint32_t q) const {
        RingView r;
        r.slots = rings + ((uint64_t)q << log2cap);
        r.mask = (1ull << log2cap) - 1ull;
        r.log2cap = log2cap;
        return r;
    }
};

// Edges a thread handles per step of the load-balancing loop (independent
// loads in flight per thread).
constexpr int kEdgesPerThread = 4;

// Whether an application sweeps vertices after each batch (kHasSweep,
// Algorithm 4's Check_Size rule); false for applications that do not say.
template <class App, class = void>
struct HasSweep {
    static constexpr bool value = false;
};
template <class App>
struct HasSweep<App, decltype((void)App::kHasSweep, void())> {
    static constexpr bool value = App::kHasSweep;
};

// Whether an application combines some of its edge updates in an LDS table
// per worker (kCombSlots > 0, see PrCombApp).  Such a worker defers counting
// its tasks done until it has flushed the table, so a run cannot be seen to
// end while combined updates sit in LDS.
template <class App, class = void>
struct CombSlots {
    static constexpr uint32_t value = 0;
};
template <class App>
struct CombSlots<App, decltype((void)App::kCombSlots, void())> {
    static constexpr uint32_t value = App::kCombSlots;
};

// Result of an application's per-task `finish` hook.
enum FinishResult : uint32_t { kFinishNone = 0, kFinishPush = 1, kFinishRepeat = 2 };

template <int BLOCK>
ATOS_DEV uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_wsum, uint32_t& total) {
    constexpr int NW = BLOCK / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    uint32_t inc = x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t y = __shfl_up(inc, off, kWave);
        if (lane >= off) inc += y;
    }
    if constexpr (NW == 1) {
        total = __shfl(inc, kWave - 1, kWave);
        return inc - x;
    } else {
        if (lane == kWave - 1) s_wsum[wid] = inc;
        __syncthreads();
        if (wid == 0) {
            uint32_t v = lane < NW ? s_wsum[lane] : 0u;
            uint32_t vi = v;
#pragma unroll
            for (int off = 1; off < NW; off <<= 1) {
                uint32_t y = __shfl_up(vi, off, kWave);
                if (lane >= off) vi += y;
            }
            if (lane < NW) s_wsum[lane] = vi - v;  // exclusive wave offsets
            if (lane == NW - 1) s_wsum[NW] = vi;   // block total
        }
        __syncthreads();
        total = s_wsum[NW];
        return s_wsum[wid] + inc - x;
    }
}

// largest i in [0, k) with scan[i] <= e  (scan[0] = 0, scan is non-decreasing)
ATOS_DEV uint32_t lbs_search(const uint32_t* scan, uint32_t k, uint32_t e) {
    uint32_t lo = 0, hi = k;  // invariant: scan[lo] <= e, answer in [lo, hi)
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (scan[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// LDS state of pop_tasks.
struct PopLds {
    uint32_t stop;       // set when a wait was abandoned: the worker must exit
    uint32_t n;          // positions claimed (bulk) or scanned
    uint32_t flag;       // bulk claim / claim succeeded
    uint32_t first_gap;  // first scanned slot that is not FULL
    uint64_t base;       // first position claimed or scanned
    uint32_t keep;       // bulk claim: positions [base, base + keep) were reserved by pushers
    uint32_t skipped;    // bulk claim: positions reserved empty by this worker (count as done)
    uint64_t head[kMaxQueues];  // probe of every ring, in visiting order
    uint64_t tail[kMaxQueues];
};

// Ring (as an offset from the caller's own, in probe order) that held the
// fewest queued tasks at the last probe; the own ring on ties.
ATOS_DEV uint32_t shallowest_ring(const PopLds& P, uint32_t NQ) {
    uint32_t best = 0;
    uint64_t depth = P.tail[0] > P.head[0] ? P.tail[0] - P.head[0] : 0ull;
    for (uint32_t j = 1; j < NQ; ++j) {
        const uint64_t d = P.tail[j] > P.head[j] ? P.tail[j] - P.head[j] : 0ull;
        if (d < depth) {
            depth = d;
            best = j;
        }
    }
    return best;
}

// Pop up to F tasks for this worker (all threads call it), from ring my_q
// first, then from the other rings.  Thread t < (tasks taken) returns true
// with its slot word in `word`; the slots are already marked FREE for the
// next lap.
//   Bulk claim, when a ring holds far more reserved tasks than all workers
//   could claim at once (>= bulk_margin): one atomicAdd of F on head, then
//   one atomicMax of tail to the end of the claim.  Positions below the tail
//   it replaced were reserved by pushers, which are publishing them: the
//   worker waits for each to turn FULL, calling stop_wait(iteration) in
//   thread 0 after every unsuccessful look (a true result abandons the wait
//   and sets P.stop).  Positions at or past that tail (head overtook it) are
//   now reserved by this worker with no task: it marks them FREE for the next
//   lap and reports them in P.skipped, for the caller to count as done.  So
//   a worker never holds tasks it took while waiting for tasks nobody will
//   push.
//   Otherwise scan up to F slots from head, count the leading FULL ones and
//   claim exactly those with a compare-and-swap on head (retried twice when
//   another worker moved head first).
// Either way a worker owns only positions it takes at once: it never goes
// back to work while holding a slot a pusher waits for.
template <int BLOCK, class StopWait>
ATOS_DEV bool pop_tasks(QueueCtl* qctl, uint64_t* rings, uint32_t log2cap, uint32_t NQ,
                        uint32_t my_q, uint32_t F, uint64_t bulk_margin, uint32_t share, bool discrete,
                        uint64_t steal_min, PopLds& P, uint64_t& word, uint64_t& st_steal,
                        StopWait stop_wait) {
    const int tid = threadIdx.x;
    bool got = false;
    word = 0;
    if (tid == 0) {
        P.stop = 0;
        P.skipped = 0;
    }
    // probe every ring at once (one memory round trip instead of one per ring)
    if ((uint32_t)tid < NQ) {
        const uint32_t q = (my_q + (uint32_t)tid) % NQ;
        P.head[tid] = ld_agent(&qctl[q].head);
        const uint64_t t = ld_agent(&qctl[q].tail);
        // a discrete round sees only the positions published before it started
        const uint64_t lim = discrete ? ld_agent(&qctl[q].limit) : 0ull;
        P.tail[tid] = discrete ? (t < lim ? t : lim) : t;
    }
    __syncthreads();
    for (uint32_t j = 0, fails = 0; j < NQ;) {
        if (fails == 0 && (P.tail[j] <= P.head[j] ||
                           (j > 0 && P.tail[j] - P.head[j] < steal_min))) {
            ++j;  // empty when probed, or another ring too shallow to steal from
            continue;
        }
        const uint32_t q = (my_q + j) % NQ;
        QueueCtl* Q = &qctl[q];
        RingView R;
        R.slots = rings + ((uint64_t)q << log2cap);
        R.mask = (1ull << log2cap) - 1ull;
        R.log2cap = log2cap;
        if (tid == 0) {
            P.first_gap = 0xFFFFFFFFu;
            const uint64_t h = fails == 0 ? P.head[j] : ld_agent(&Q->head);
            uint64_t t = fails == 0 ? P.tail[j] : ld_agent(&Q->tail);
            if (discrete) {
                const uint64_t lim = ld_agent(&Q->limit);
                if (t > lim) t = lim;
            }
            if (!discrete && t > h && t - h >= bulk_margin) {
                const uint64_t b = add_agent(&Q->head, (uint64_t)F);
                const uint64_t t_old = max_agent(&Q->tail, b + (uint64_t)F);
                P.base = b;
                P.n = F;
                P.keep = t_old >= b + (uint64_t)F ? F : (t_old > b ? (uint32_t)(t_old - b) : 0u);
                P.skipped += F - P.keep;
                P.flag = 1u;
            } else {
                // take up to F, or with share > 0 only this worker's share of what
                // the ring holds (rounded up): when the ring is shallow its tasks
                // then go to many workers instead of one
                uint32_t f = F;
                if (share > 0u && t > h) {
                    const uint64_t part = (t - h + share - 1u) / share;
                    f = part < (uint64_t)F ? (uint32_t)part : F;
                }
                P.base = h;
                P.n = t > h ? (uint32_t)((t - h) < f ? (t - h) : f) : 0u;
                P.flag = 0u;
            }
        }
        __syncthreads();
        const uint32_t n_scan = P.n;
        const uint64_t h = P.base;
        const bool bulk = P.flag != 0u;
        __syncthreads();
        if (n_scan == 0) {
            ++j;
            fails = 0;
            continue;
        }
        if (bulk) {
            const uint32_t keep = P.keep;
            if ((uint32_t)tid >= keep && (uint32_t)tid < n_scan) {
                // reserved empty: advance the slot to the next lap.  It is FREE for
                // this position unless the ring is full and the previous lap's task
                // there has not been taken yet; then wait for that (bounded: past
                // the limit the slot stays behind and a later push reports overflow).
                const uint64_t pos = h + (uint64_t)tid;
                for (uint32_t tries = 0;
                     !cas_agent(R.slot(pos), R.free_word(pos), R.free_word(pos + R.mask + 1)) &&
                     tries < (1u << 20);
                     ++tries)
                    __builtin_amdgcn_s_sleep(2);
            }
            const bool mine = (uint32_t)tid < keep;
            for (uint32_t wait = 1;; ++wait) {
                if (mine && !got) {
                    word = ld_agent(R.slot(h + (uint64_t)tid));
                    if (R.is_full_for(word, h + (uint64_t)tid)) {
                        got = true;
                        st_agent(R.slot(h + (uint64_t)tid), R.free_word(h + (uint64_t)tid + R.mask + 1));
                    }
                }
                if (__syncthreads_count(mine && !got) == 0) break;
                if (tid == 0) P.stop = stop_wait(wait) ? 1u : 0u;
                __syncthreads();
                if (P.stop) break;
                __builtin_amdgcn_s_sleep(2);
            }
            if (j) ++st_steal;
            break;
        }
        if ((uint32_t)tid < n_scan) {
            word = ld_agent(R.slot(h + (uint64_t)tid));
            if (!R.is_full_for(word, h + (uint64_t)tid)) atomicMin(&P.first_gap, (uint32_t)tid);
        }
        __syncthreads();
        const uint32_t n_full = P.first_gap < n_scan ? P.first_gap : n_scan;
        if (tid == 0) {
            P.flag = 0u;
            if (n_full > 0 && cas_agent(&Q->head, h, h + (uint64_t)n_full)) {
                P.flag = 1u;
                if (j) ++st_steal;
            }
        }
        __syncthreads();
        if (P.flag) {
            got = (uint32_t)tid < n_full;
            if (got) st_agent(R.slot(h + (uint64_t)tid), R.free_word(h + (uint64_t)tid + R.mask + 1));
            break;
        }
        __syncthreads();
        if (n_full > 0 && ++fails <= 2) continue;  // lost the race for this head
        ++j;
        fails = 0;
    }
    if (!got) word = 0;
    return got;
}

// Publish the initial tasks, in a launch of their own before the worker
// kernel (so no worker ever waits on a task that a workgroup not yet
// resident would publish): task i goes to ring i % NQ at position
// init_base + i / NQ of that ring.
template <class App, class OffT>
__global__ void seed_tasks_kernel(PersistArgs<OffT> a, App app) {
    WsHeader* H = a.hdr;
    const uint32_t NQ = a.n_queues;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n_init;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t v, aux;
        app.init_task(i, v, aux);
        const uint32_t q = (uint32_t)(i % NQ);
        const RingView R = a.ring_of(q);
        const uint64_t pos = H->q[q].init_base + i / NQ;
        if (!cas_agent(R.slot(pos), R.free_word(pos), R.full_word(pos, make_payload(v, aux))))
            or_agent(&H->status, (uint32_t)kStatusCorrupt);
    }
}

template <int BLOCK, class App, class OffT>
__global__ __launch_bounds__(BLOCK) void persistent_kernel(PersistArgs<OffT> a, App app) {
    constexpr int PUSH_CAP = (2 * BLOCK < 512) ? 512 : 2 * BLOCK;
    constexpr int NW = BLOCK / kWave;

    __shared__ uint32_t s_vert[BLOCK];
    __shared__ uint32_t s_aux[BLOCK];
    __shared__ uint32_t s_val[BLOCK];
    __shared__ uint32_t s_deg[BLOCK];
    __shared__ uint32_t s_active[BLOCK];
    __shared__ OffT s_start[BLOCK];
    __shared__ uint32_t s_scan[BLOCK + 1];
    constexpr int W = App::kAccWords;  // accumulator words per task
    static_assert(!App::kSplittable || W <= kBoardRedWords, "hub board reduction words");
    __shared__ uint64_t s_acc[BLOCK * W];
    __shared__ uint64_t s_push[PUSH_CAP];
    __shared__ uint32_t s_wsum[NW + 1];
    __shared__ uint32_t s_push_n;
    __shared__ uint32_t s_k;
    __shared__ uint32_t s_stop;
    __shared__ PopLds s_pop;
    __shared__ uint64_t s_push_base;
    __shared__ int32_t s_hub;       // board entry whose chunk this worker claimed, or -1
    __shared__ uint64_t s_board_mask[kBoardEntries / 64];  // open entries at the last poll
    __shared__ uint32_t s_hub_cand;  // lowest scan index of an open entry with work
    __shared__ uint32_t s_posted;    // tasks of this batch posted to the board
    __shared__ uint64_t s_tmax;      // trace: (degree << 32 | vertex) of the batch's largest task
    __shared__ uint32_t s_last;      // this hub chunk completed its task
    __shared__ uint32_t s_fin_r;     // the completed hub task's finish result
    __shared__ uint64_t s_fin_payload;
    __shared__ uint64_t s_sweep_base;  // first cursor position of this batch's sweep
    __shared__ uint32_t s_qcnt[kMaxQueues];   // segmented flush: tasks per ring
    __shared__ uint64_t s_qbase[kMaxQueues];  // their first reserved position per ring
    constexpr uint32_t CS = CombSlots<App>::value;
    __shared__ double s_comb[CS > 0 ? CS : 1];  // combined updates per slot (CS > 0)
    __shared__ uint32_t s_comb_due;             // the table is to be flushed now
    __shared__ uint64_t s_done_defer;   // tasks finished since the last flush (counted by it)
    __shared__ uint64_t s_comb_edges0;  // st_edges at the last flush

    const int tid = threadIdx.x;
    WsHeader* H = a.hdr;
    const uint32_t F = (uint32_t)a.fetch;
    const uint32_t NQ = a.n_queues;
    const uint32_t my_q = xcc_id() % NQ;
    QueueCtl* const myQ = &H->q[my_q];
    __shared__ uint32_t s_push_q;  // ring the current flush publishes into
    Deadline deadline;  // checked by thread 0 only
    deadline.start(a.timeout_ticks);
    // tasks with more than a.split_degree edges go to the hub board, in chunks of kHubChunk
    constexpr uint32_t kHubChunk = 4 * BLOCK > 1024 ? 4 * BLOCK : 1024;
    constexpr uint64_t kOffMask = (1ull << kBoardOffsetBits) - 1ull;

    if (tid == 0) {
        s_push_n = 0;
        s_k = 0;
        s_posted = 0;
    }
    if ((uint32_t)tid < (uint32_t)kMaxQueues) {  // no probe yet: every ring counts as empty
        s_pop.head[tid] = 0;
        s_pop.tail[tid] = 0;
    }

    uint32_t spin = 0, abort_poll = 0;
    uint64_t st_pop = 0, st_push = 0, st_edges = 0, st_retry = 0, st_idle = 0, st_steal = 0;
    // combining (CS > 0): this thread's combined updates and flush atomics
    uint32_t st_comb = 0, st_comb_atomics = 0;
    if constexpr (CS > 0) {
        for (uint32_t j = (uint32_t)tid; j < CS; j += BLOCK) s_comb[j] = 0.0;
        if (tid == 0) {
            s_done_defer = 0;
            s_comb_edges0 = 0;
            s_comb_due = 0;
        }
        app.comb = s_comb;
    }

    // Publish the tasks gathered in s_push into this XCD's ring: reserve
    // positions with one atomic on tail, then turn each slot FREE -> FULL.
    // Called by all threads.
    auto flush = [&]() {
        __syncthreads();
        const uint32_t n = s_push_n;
        if (n == 0) return;
        wait_vmem();  // this thread's updates are complete before any task is published
        // segmented: the target ring of every task (its vertex's segment) and its
        // rank among this flush's tasks for that ring (tasks tid, tid + BLOCK, ...)
        constexpr uint32_t PER = (PUSH_CAP + BLOCK - 1) / BLOCK;
        uint32_t seg_rank[PER], seg_ring[PER];
        if (a.segmented) {
            if ((uint32_t)tid < (uint32_t)kMaxQueues) s_qcnt[tid] = 0u;
            __syncthreads();
#pragma unroll
            for (uint32_t j = 0; j < PER; ++j) {
                const uint32_t i = j * BLOCK + (uint32_t)tid;
                seg_ring[j] = 0u;
                seg_rank[j] = 0u;
                if (i < n) {
                    const uint32_t v = payload_vertex(s_push[i]);
                    uint32_t r = 0;
#pragma unroll
                    for (int b = 0; b < kMaxQueues - 1; ++b) r += v >= a.seg_bound[b] ? 1u : 0u;
                    seg_ring[j] = r % NQ;
                    seg_rank[j] = atomicAdd(&s_qcnt[seg_ring[j]], 1u);
                }
            }
        }
        __syncthreads();
        if (a.segmented) {
            if ((uint32_t)tid < NQ && s_qcnt[tid] != 0u)
                s_qbase[tid] = add_agent(&H->q[tid].tail, (uint64_t)s_qcnt[tid]);
        } else if (tid == 0) {
            uint32_t pq = my_q;
            if (a.push_shallow) pq = (my_q + shallowest_ring(s_pop, NQ)) % NQ;
            s_push_q = pq;
            s_push_base = add_agent(&H->q[pq].tail, (uint64_t)n);
        }
        __syncthreads();
        const uint64_t base = s_push_base;
        uint64_t retries = 0;
#pragma unroll
        for (uint32_t j = 0; j < PER; ++j) {
            const uint32_t i = j * BLOCK + (uint32_t)tid;
            if (i >= n) continue;
            const uint32_t r = a.segmented ? seg_ring[j] : s_push_q;
            const RingView myR = a.ring_of(r);
            const uint64_t pos = a.segmented ? s_qbase[r] + seg_rank[j] : base + i;
            const uint64_t want = myR.free_word(pos);
            const uint64_t full = myR.full_word(pos, s_push[i]);
            uint32_t tries = 0;
            while (!cas_agent(myR.slot(pos), want, full)) {
                // The previous lap's task in this slot has not been taken yet.
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

    // Uniform decision, taken after every pending append is visible, whether
    // s_push may not have room for one more task per thread.
    auto push_buffer_nearly_full = [&]() -> bool {
        __syncthreads();
        return __syncthreads_or(tid == 0 && s_push_n + BLOCK > (uint32_t)PUSH_CAP) != 0;
    };

    // Append this thread's new task (if any) to s_push, one LDS atomic per wavefront.
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

    // Counts tasks done: at once, or (combining) when the table is next flushed.
    auto count_done = [&](uint64_t n) {
        if constexpr (CS > 0) {
            s_done_defer += n;
        } else {
            add_agent(&myQ->done, n);
        }
    };

    // Combining: apply every non-empty slot of the LDS table with one device
    // atomic (the application's crossing test on the combined amount may push
    // the vertex), publish those pushes, and only then count the deferred
    // tasks done.  Called by all threads between batches (no LDS update is in
    // flight).  Each thread issues its slots' atomics back to back before it
    // waits for any result, as the edge loop does.
    auto comb_flush = [&]() {
        if constexpr (CS > 0) {
            constexpr uint32_t PER = 4;
            __syncthreads();
            for (uint32_t s0 = 0; s0 < CS; s0 += BLOCK * PER) {
                // slot vertices, then every atomic, then the decisions (each slot's
                // amount read again from the table, which is cleared there)
                uint32_t w[PER];
                uint64_t old[PER];
#pragma unroll
                for (uint32_t j = 0; j < PER; ++j) {
                    const uint32_t sl = s0 + j * BLOCK + (uint32_t)tid;
                    w[j] = 0xFFFFFFFFu;
                    if (sl < CS && s_comb[sl] != 0.0) w[j] = app.comb_vertex[sl];
                }
#pragma unroll
                for (uint32_t j = 0; j < PER; ++j) {
                    old[j] = 0ull;
                    if (w[j] != 0xFFFFFFFFu) {
                        old[j] = app.comb_issue(w[j], s_comb[s0 + j * BLOCK + (uint32_t)tid]);
                        ++st_comb_atomics;
                    }
                }
#pragma unroll
                for (uint32_t j = 0; j < PER; ++j) {
                    bool push = false;
                    if (w[j] != 0xFFFFFFFFu) {
                        const uint32_t sl = s0 + j * BLOCK + (uint32_t)tid;
                        push = app.comb_decide(s_comb[sl], old[j]);
                        s_comb[sl] = 0.0;
                    }
                    append(push, make_payload(w[j], App::kCombAux));
                    if (push_buffer_nearly_full()) flush();  // room for the next BLOCK
                }
            }
            flush();  // the pushes are reserved before the deferred tasks count as done
            if (tid == 0) {
                if (s_done_defer) add_agent(&myQ->done, s_done_defer);
                s_done_defer = 0;
                s_comb_edges0 = st_edges;
                s_comb_due = 0;
            }
            __syncthreads();
        }
    };

    __syncthreads();
    for (;;) {
        if constexpr (CS > 0) {
            // the table is due (after the flush window, or with nothing to do)
            if (s_comb_due) comb_flush();
        }
        // ---- hub board: help with a chunk of a posted task before taking new work
        uint32_t k_board = 0;
        if constexpr (App::kSplittable) {
            if (tid == 0) {
                s_hub = -1;
                s_hub_cand = 0xFFFFFFFFu;
            }
            // one load by one thread, decision made uniform by the barrier; then
            // the open-entry mask (one word per 64 entries), and only the entries
            // it marks are read, so a worker polling an open board reads a few
            // words rather than every entry
            if (__syncthreads_or(tid == 0 && ld_agent(&H->board_open) != 0u)) {
                if (tid < kBoardEntries / 64) s_board_mask[tid] = ld_agent(&H->board_mask[tid]);
                __syncthreads();
                for (uint32_t j = tid; j < (uint32_t)kBoardEntries; j += BLOCK) {
                    const uint32_t e = (blockIdx.x + j) % kBoardEntries;
                    if (((s_board_mask[e >> 6] >> (e & 63u)) & 1ull) == 0ull) continue;
                    HubEntry* E = &H->board[e];
                    if (ld_agent(&E->state) == kBoardOpen &&
                        (ld_agent(&E->cursor) & kOffMask) < ld_agent(&E->end))
                        atomicMin(&s_hub_cand, j);
                }
                __syncthreads();
                if (tid == 0 && s_hub_cand != 0xFFFFFFFFu) {
                    const uint32_t e = (blockIdx.x + s_hub_cand) % kBoardEntries;
                    HubEntry* E = &H->board[e];
                    // Claim the next chunk with one fetch-add on the cursor (no lost
                    // races).  The claim is valid when its offset is below the task's
                    // end and the generation is unchanged after the fields were read:
                    // a generation ends (and the entry is re-posted, closing the cursor
                    // first) only once every valid chunk of it has finished, so a
                    // valid claim holds the fields stable, and a claim that finds a
                    // new generation was not valid.  Offsets past the end (and the
                    // closed marker, 2^39) are simply no work.
                    const uint64_t old = add_agent(&E->cursor, (uint64_t)kHubChunk);
                    const uint64_t off = old & kOffMask;
                    if (off < kBoardClosed) {
                        const uint64_t end = ld_agent(&E->end);
                        const uint32_t vtx = ld_agent(&E->vertex);
                        const uint32_t aux = ld_agent(&E->aux);
                        const uint32_t val = ld_agent(&E->val);
                        const uint64_t acc0 = ld_agent(&E->acc);
                        wait_vmem();  // the fields were read before the generation check
                        if (off < end && ((ld_agent(&E->cursor) ^ old) >> kBoardOffsetBits) == 0ull) {
                            const uint64_t len = end - off < kHubChunk ? end - off : kHubChunk;
                            s_hub = (int32_t)e;
                            s_vert[0] = vtx;
                            s_aux[0] = aux;
                            s_val[0] = val;
#pragma unroll
                            for (int j = 1; j < W; ++j) s_acc[j] = 0;
                            s_acc[0] = acc0;
                            s_start[0] = (OffT)off;
                            s_deg[0] = (uint32_t)len;
                            s_active[0] = 1u;
                        }
                    }
                }
            }
            __syncthreads();
            if (s_hub >= 0) k_board = 1;
        }

        uint32_t k = 0;
        uint64_t tr_begin = 0, tr_edges = 0;  // trace (thread 0)
        if (k_board == 0) {
        // ---- pop, from this XCD's ring first, then from the others (pop_tasks)
        bool got = false;
        uint64_t word = 0;
        if (tid == 0) {
            s_stop = 0;
            if (ld_agent(&H->status) != 0u) {
                s_stop = 1;  // another worker stopped the run
            } else if (deadline.passed()) {
                or_agent(&H->status, (uint32_t)kStatusTimeout);
                s_stop = 1;
            } else if (a.abort_flag != nullptr && (++abort_poll & 31u) == 0u &&
                       __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) {
                or_agent(&H->status, (uint32_t)kStatusAbort);  // stopped from the host
                s_stop = 1;
            }
        }
        __syncthreads();
        if (s_stop) break;
        // stop waiting for bulk-claimed positions on error, at the deadline, or
        // when every reserved task is done (positions past tail then stay empty;
        // tasks already taken are reserved and not done, so this cannot hold
        // while this worker holds any)
        auto stop_wait = [&](uint32_t wait) -> bool {
            if (ld_agent(&H->status) != 0u) return true;
            if (deadline.passed()) {
                or_agent(&H->status, (uint32_t)kStatusTimeout);
                return true;
            }
            if ((wait & 63u) != 0u) return false;
            uint64_t d = 0, t = 0;
            for (uint32_t r = 0; r < NQ; ++r) d += ld_agent(&H->q[r].done);
            wait_vmem();
            for (uint32_t r = 0; r < NQ; ++r) t += ld_agent(&H->q[r].tail);
            return d == t;
        };
        got = pop_tasks<BLOCK>(H->q, a.rings, a.log2cap, NQ, my_q, F, a.bulk_margin, a.fetch_share,
                               a.discrete != 0u, 0ull, s_pop, word,
                               st_steal, stop_wait);
        if (s_pop.stop) break;
        if (tid == 0) {
            s_k = 0;
            // positions reserved with no task: consumed, so counted as done at once
            if (s_pop.skipped) add_agent(&myQ->done, (uint64_t)s_pop.skipped);
        }
        __syncthreads();
        if (got && (int64_t)payload_vertex(word) >= a.n) {
            // not a task this library wrote: never dereference it
            or_agent(&H->status, (uint32_t)kStatusCorrupt);
            got = false;
        }
        if (got) {
            const uint32_t idx = atomicAdd(&s_k, 1u);
            s_vert[idx] = payload_vertex(word);
            s_aux[idx] = payload_aux(word);
        }
        __syncthreads();
        k = s_k;
        if constexpr (CS > 0) {
            if (k == 0) {
                // nothing to do: flush the table (and count the deferred tasks
                // done) before looking for the end of the run
                if (tid == 0) s_comb_due = (s_done_defer != 0 || st_edges != s_comb_edges0) ? 1u : 0u;
                __syncthreads();
                if (s_comb_due) continue;  // flushed at the top of the loop
            }
        }
        if (k == 0) {
            // ---- idle: stop on error, on termination, or at the deadline.
            //      Termination: every task ever reserved has completed, i.e.
            //      sum(done) == sum(tail), with all dones read before the tails.
            if (tid == 0) {
                ++st_idle;
                uint32_t stop = 0;
                if (ld_agent(&H->status) != 0u) {
                    stop = 1;
                } else {
                    uint64_t d = 0, t = 0;
                    for (uint32_t q = 0; q < NQ; ++q) d += ld_agent(&H->q[q].done);
                    wait_vmem();
                    for (uint32_t q = 0; q < NQ; ++q) t += ld_agent(&H->q[q].tail);
                    if (d == t) {
                        stop = 1;
                    } else if (deadline.passed()) {
                        or_agent(&H->status, (uint32_t)kStatusTimeout);
                        stop = 1;
                    } else if (a.discrete == 1u) {
                        // a discrete round ends when every position below the limits is
                        // taken (what the taken tasks push is the next round's work)
                        stop = 1;
                        for (uint32_t q = 0; q < NQ; ++q)
                            if (ld_agent(&H->q[q].head) < ld_agent(&H->q[q].limit)) stop = 0;
                    } else if (a.discrete == 2u) {
                        // rounds inside this launch: once every position below the
                        // limits is taken, the next round is everything published
                        // (reserved) by now; batches of the old round still running
                        // push into the round after it
                        bool taken = true;
                        for (uint32_t q = 0; q < NQ; ++q)
                            if (ld_agent(&H->q[q].head) < ld_agent(&H->q[q].limit)) taken = false;
                        if (taken) {
                            bool moved = false;
                            for (uint32_t q = 0; q < NQ; ++q) {
                                const uint64_t t = ld_agent(&H->q[q].tail);
                                if (max_agent(&H->q[q].limit, t) < t) moved = true;
                            }
                            if (moved) add_agent(&H->stat_rounds, (uint64_t)1);
                        }
                    }
                }
                s_stop = stop;
            }
            __syncthreads();
            if (s_stop) break;
            backoff(spin);
            continue;
        }
        spin = 0;
        if (a.trace != nullptr && tid == 0) {
            tr_begin = now_ticks();
            tr_edges = st_edges;
            s_tmax = 0;
        }
        if (a.trace != nullptr) __syncthreads();

        // ---- per task: neighbour range and application prepare
        if ((uint32_t)tid < k) {
            const uint32_t v = s_vert[tid];
            const OffT beg = a.offs[v];
            const OffT end = a.offs[v + 1];
            if (a.trace != nullptr)
                atomicMax((unsigned long long*)&s_tmax, ((unsigned long long)(end - beg) << 32) | v);
            uint32_t val = 0;
            uint64_t* acc = &s_acc[tid * W];
#pragma unroll
            for (int j = 0; j < W; ++j) acc[j] = 0;
            const uint32_t deg = (uint32_t)(end - beg);
            uint32_t aux = s_aux[tid];
            bool active = app.prepare(v, aux, deg, val, acc);  // may turn the task into another pass
            s_aux[tid] = aux;
            if constexpr (App::kSplittable) {
                if (active && a.split_degree != 0u && deg > a.split_degree) {
                    // post to the hub board; on success its edges are processed in
                    // chunks by whichever workers claim them
                    for (uint32_t j = 0; j < 4; ++j) {
                        const uint32_t e = (v * 2654435761u + j * 40503u) % kBoardEntries;
                        HubEntry* E = &H->board[e];
                        if (!cas_agent(&E->state, kBoardFree, kBoardPosting)) continue;
                        // Close the entry under a new generation before changing any
                        // field: a claim taken from the previous cursor then fails its
                        // generation check, and one taken from the closed cursor finds
                        // no edges left (offset kBoardClosed >= any end).
                        const uint64_t gen = ((ld_agent(&E->cursor) >> kBoardOffsetBits) + 1ull) & 0xFFFFFFull;
                        st_agent(&E->cursor, (gen << kBoardOffsetBits) | kBoardClosed);
                        wait_vmem();
                        st_agent(&E->vertex, v);
                        st_agent(&E->aux, s_aux[tid]);
                        st_agent(&E->val, val);
                        st_agent(&E->acc, acc[0]);  // splittable apps use one word
                        st_agent(&E->end, (uint64_t)end);
                        st_agent(&E->finished, (uint64_t)0);
                        st_agent(&E->total, (uint64_t)deg);
                        if constexpr (App::kHasFinish) {
#pragma unroll
                            for (int j = 0; j < W; ++j) st_agent(&H->board_red[e][j], (uint64_t)0);
                        }
                        wait_vmem();
                        st_agent(&E->cursor, (uint64_t)((gen << kBoardOffsetBits) | (uint64_t)beg));
                        wait_vmem();
                        st_agent(&E->state, kBoardOpen);
                        or_agent(&H->board_mask[e >> 6], (uint64_t)1 << (e & 63u));
                        add_agent(&H->board_open, 1u);
                        add_agent(&H->stat_hub_posts, (uint64_t)1);
                        atomicAdd(&s_posted, 1u);
                        active = false;
                        break;
                    }
                }
            }
            s_start[tid] = beg;
            s_deg[tid] = deg;
            s_val[tid] = val;
            s_active[tid] = active ? 1u : 0u;
        }
        __syncthreads();
        }  // k_board == 0
        if (k_board) {
            k = 1;
            if (a.trace != nullptr && tid == 0) {
                tr_begin = now_ticks();
                tr_edges = st_edges;
                s_tmax = ((uint64_t)s_deg[0] << 32) | s_vert[0];
            }
        }

        bool repeat;
        do {
            const uint32_t cnt = ((uint32_t)tid < k && s_active[tid]) ? s_deg[tid] : 0u;
            uint32_t total;
            const uint32_t ex = block_exclusive_scan<BLOCK>(cnt, s_wsum, total);
            if ((uint32_t)tid < k) s_scan[tid] = ex;
            if (tid == 0) s_scan[k] = total;
            __syncthreads();
            if (tid == 0) st_edges += total;

            // ---- load-balancing search over the batch's edges, EPT edges per thread
            //      per step: first every neighbour id, then every neighbour's state
            //      (App::gather), so that a thread has EPT independent loads in
            //      flight before it uses any (a lone worker walking a long
            //      neighbour list is bound by that latency); then the callbacks.
            // (s_push_n is stable here: the last append was before the previous barrier)
            const bool may_overflow = s_push_n + total + BLOCK > (uint32_t)PUSH_CAP;
            for (uint32_t eb = 0; eb < total; eb += BLOCK * kEdgesPerThread) {
                uint32_t wv[kEdgesPerThread], iv[kEdgesPerThread];
                typename App::Nbr nv[kEdgesPerThread];
#pragma unroll
                for (int j = 0; j < kEdgesPerThread; ++j) {
                    const uint32_t e = eb + (uint32_t)(j * BLOCK + tid);
                    iv[j] = 0xFFFFFFFFu;
                    wv[j] = 0u;
                    if (e < total) {
                        const uint32_t i = lbs_search(s_scan, k, e);
                        wv[j] = (uint32_t)a.cols[s_start[i] + (OffT)(e - s_scan[i])];
                        iv[j] = i;
                        if constexpr (CS > 0) st_comb += wv[j] >> 31;  // a combined update
                    }
                }
#pragma unroll
                for (int j = 0; j < kEdgesPerThread; ++j)
                    if (iv[j] != 0xFFFFFFFFu) nv[j] = app.gather(s_vert[iv[j]], s_aux[iv[j]], wv[j]);
                // every id and state has arrived: with no load outstanding, the
                // updates of all EPT edges issue back to back and their atomics are
                // in flight together; the push decisions come after
                wait_vmem();
                if constexpr (App::kHasNotify) {
                    // updates that must be performed before the edge updates (completed
                    // by the wait below)
#pragma unroll
                    for (int j = 0; j < kEdgesPerThread; ++j)
                        if (iv[j] != 0xFFFFFFFFu)
                            app.notify(s_vert[iv[j]], s_aux[iv[j]], s_val[iv[j]], wv[j], nv[j]);
                    wait_vmem();
                }
                uint64_t uw[kEdgesPerThread];
#pragma unroll
                for (int j = 0; j < kEdgesPerThread; ++j) {
                    uw[j] = 0;
                    if (iv[j] != 0xFFFFFFFFu) {
                        const uint32_t i = iv[j];
                        uw[j] = app.edge(s_vert[i], s_aux[i], s_val[i], s_deg[i], wv[j], nv[j],
                                         &s_acc[i * W]);
                    }
                }
#pragma unroll
                for (int j = 0; j < kEdgesPerThread; ++j) {
                    bool push = false;
                    uint64_t payload = 0;
                    if (iv[j] != 0xFFFFFFFFu) {
                        const uint32_t i = iv[j];
                        uint32_t paux = 0;
                        push = app.decide(s_vert[i], s_aux[i], s_val[i], wv[j], nv[j], uw[j], paux,
                                          &s_acc[i * W]);
                        payload = make_payload(wv[j], paux);
                    }
                    append(push, payload);
                    if (may_overflow && push_buffer_nearly_full()) flush();
                }
            }

            // ---- per task: application finish (may emit one task, or ask for another pass)
            repeat = false;
            if constexpr (App::kHasFinish) {
                if (k_board) break;  // a hub chunk: its task finishes with its last chunk
                if (push_buffer_nearly_full()) flush();
                bool push = false;
                uint64_t payload = 0;
                bool again = false;
                if ((uint32_t)tid < k && s_active[tid]) {
                    uint32_t pv = 0, paux = 0;
                    uint32_t val = s_val[tid];
                    uint32_t aux = s_aux[tid];
                    const uint32_t r = app.finish(s_vert[tid], aux, s_deg[tid], val,
                                                  &s_acc[tid * W], pv, paux);
                    if (r == kFinishPush) {
                        push = true;
                        payload = make_payload(pv, paux);
                    } else if (r == kFinishRepeat) {
                        again = true;
                    }
                    s_val[tid] = val;
                    s_aux[tid] = aux;
                }
                if ((uint32_t)tid < k) s_active[tid] = again ? 1u : 0u;
                append(push, payload);
                repeat = __syncthreads_or(again) != 0;
            }
        } while (repeat);

        if constexpr (HasSweep<App>::value) {
            // Algorithm 4's sweep: the batch's tasks take the next positions of the
            // round-robin cursor at once and push every vertex there above eps
            const uint32_t total = app.sweep_positions(k);
            if (tid == 0) s_sweep_base = add_agent(&H->check_cursor, (uint64_t)total);
            __syncthreads();
            const uint64_t sbase = s_sweep_base;
            for (uint32_t i0 = 0; i0 < total; i0 += BLOCK) {
                bool push = false;
                uint32_t v = 0;
                if (i0 + (uint32_t)tid < total) {
                    v = (uint32_t)((sbase + i0 + (uint32_t)tid) % (uint64_t)a.n);
                    push = app.sweep_test(v);
                }
                append(push, make_payload(v, 0u));
                if (push_buffer_nearly_full()) flush();
            }
        }
        flush();
        if (k_board) {
            // a hub chunk: the posted task completes with its last chunk, which
            // (for an application with a finish step) runs finish on the union
            // of every chunk's accumulator words
            HubEntry* E = &H->board[s_hub];
            if (tid == 0) {
                if constexpr (App::kHasFinish) {
#pragma unroll
                    for (int j = 0; j < W; ++j)
                        if (s_acc[j]) or_agent(&H->board_red[s_hub][j], s_acc[j]);
                    wait_vmem();  // merged before this chunk is counted
                }
                const uint64_t len = s_deg[0];
                const uint64_t before = add_agent(&E->finished, len);
                s_last = before + len == ld_agent(&E->total) ? 1u : 0u;
                s_fin_r = kFinishNone;
            }
            __syncthreads();
            if (s_last) {
                if constexpr (App::kHasFinish) {
                    if (tid == 0) {
#pragma unroll
                        for (int j = 0; j < W; ++j) s_acc[j] = ld_agent(&H->board_red[s_hub][j]);
                        uint32_t aux = s_aux[0], val = s_val[0], pv = 0, paux = 0;
                        const uint64_t total = ld_agent(&E->total);
                        const uint32_t r = app.finish(s_vert[0], aux, (uint32_t)total, val, s_acc, pv, paux);
                        s_fin_r = r;
                        s_fin_payload = make_payload(pv, paux);
                        if (r == kFinishRepeat) {
                            // another pass over the whole list: re-open the entry under a
                            // new generation (closed first, as when posting)
                            const uint64_t gen =
                                ((ld_agent(&E->cursor) >> kBoardOffsetBits) + 1ull) & 0xFFFFFFull;
                            st_agent(&E->cursor, (gen << kBoardOffsetBits) | kBoardClosed);
                            wait_vmem();
                            st_agent(&E->aux, aux);
                            st_agent(&E->val, val);
                            st_agent(&E->acc, s_acc[0]);
#pragma unroll
                            for (int j = 0; j < W; ++j) st_agent(&H->board_red[s_hub][j], (uint64_t)0);
                            st_agent(&E->finished, (uint64_t)0);
                            wait_vmem();
                            st_agent(&E->cursor,
                                     (gen << kBoardOffsetBits) | (ld_agent(&E->end) - total));
                        }
                    }
                    __syncthreads();
                    if (s_fin_r == kFinishPush) {
                        append(tid == 0, s_fin_payload);
                        flush();
                    }
                }
                if (tid == 0 && s_fin_r != kFinishRepeat) {
                    count_done(1);
                    // Clear the entry's open bit before freeing it: once the entry is
                    // free another worker may post to it and set the bit again, and a
                    // clear issued after that would hide the new task from every
                    // scanner (its chunks never claimed, the run never done).
                    and_agent(&H->board_mask[(uint32_t)s_hub >> 6], ~((uint64_t)1 << ((uint32_t)s_hub & 63u)));
                    wait_vmem();
                    st_agent(&E->state, kBoardFree);
                    add_agent(&H->board_open, 0xFFFFFFFFu);
                }
            }
        }
        if (tid == 0) {
            if (!k_board) {
                st_pop += k;
                // counted only now: the tasks' children were reserved (tail) before;
                // tasks posted to the board are counted by their last chunk
                count_done((uint64_t)(k - s_posted));
                s_posted = 0;
            }
            if (a.trace != nullptr) {
                const uint64_t r = add_agent(&a.trace->count, (uint64_t)1);
                if (r < a.trace->capacity) {
                    TraceRec* R = &a.trace->rec[r];
                    R->t_begin = tr_begin;
                    R->t_end = now_ticks();
                    R->worker = blockIdx.x;
                    R->tasks = k_board ? (0x80000000u | 1u) : k;
                    R->edges = (uint32_t)(st_edges - tr_edges);
                    R->vertex = (uint32_t)s_tmax;
                }
            }
        }
        if constexpr (CS > 0) {
            if (tid == 0) s_comb_due = st_edges - s_comb_edges0 >= (uint64_t)a.comb_flush_edges ? 1u : 0u;
        }
        __syncthreads();
    }

    if constexpr (CS > 0) {
        if (st_comb) add_agent(&H->stat_comb_adds, (uint64_t)st_comb);
        if (st_comb_atomics) add_agent(&H->stat_comb_atomics, (uint64_t)st_comb_atomics);
    }

    if (tid == 0) {
        add_agent(&H->stat_popped, st_pop);
        add_agent(&H->stat_pushed, st_push);
        add_agent(&H->stat_edges, st_edges);
        if (st_idle) add_agent(&H->stat_idle, st_idle);
        if (st_steal) add_agent(&H->stat_steals, st_steal);
        if (ld_agent(&H->status) != 0u) st_agent(&H->cookie, (uint64_t)0);
    }
    (void)st_retry;
}

// ------------------------------------------------------------------ applications
// Each application supplies:
//   kAccWords                         64-bit accumulator words per task (in LDS,
//                                     zeroed before prepare)
//   init_task(i, v, aux)              vertex and aux word of initial task i
//   prepare(v, aux, deg, val, acc)    per popped task; returns whether the task
//                                     is processed (its edges scanned, finish run);
//                                     may change the task's aux word (which pass)
//   kHasNotify, notify(v, aux, val, w, nbr)  optional per-edge update completed
//                                     before any edge update of the same step
//   Nbr, gather(v, aux, w)            the state of neighbour w (and of v) the
//                                     edge callback reads, loaded ahead of it
//   edge(v, aux, val, deg, w, nbr, acc)  per neighbour w of v (deg = deg(v)):
//                                     applies the update and returns an update
//                                     word, the result of at most one atomic,
//                                     without using it and with no memory load,
//                                     so that the thread's next edges are issued
//                                     before it waits for the result
//   decide(v, aux, val, w, nbr, word, paux, acc)  whether to push w, from the
//                                     update word
//   finish(v, aux, deg, val, acc, pv, paux)  per processed task after its edges
//                                     (optional); may push one task, or ask for
//                                     another pass over the edges (with aux and
//                                     val updated)
//   kSplittable                       whether a task's edges may be processed in
//                                     independent chunks (hub board): every chunk
//                                     starts from the posted accumulator word 0
//                                     (other words zero), and with a finish step
//                                     the chunks' accumulator words must reduce
//                                     by OR (finish runs once, on the union)

// Speculative BFS (Algorithm 2).  A task carries the low 16 bits of the
// depth its pusher set; when the vertex has since been lowered again the
// task is a stale duplicate and is dropped (the newer push expands it).
struct BfsApp {
    uint32_t* depth;
    uint32_t source;
    static constexpr int kAccWords = 1;
    static constexpr bool kHasFinish = false;
    static constexpr bool kHasNotify = false;
    static constexpr bool kSplittable = true;

    ATOS_DEV void init_task(uint64_t, uint32_t& v, uint32_t& aux) const {
        v = source;
        aux = 0u;
    }
    ATOS_DEV bool prepare(uint32_t v, uint32_t aux, uint32_t, uint32_t& val, uint64_t*) const {
        const uint32_t d = ld_agent(depth + v);
        val = d + 1u;
        return (d & 0xFFFFu) == aux;
    }
    // A plain load may return an older value, and depths only decrease, so it
    // never hides an improvement: it only filters hopeless updates.
    using Nbr = uint32_t;
    ATOS_DEV Nbr gather(uint32_t, uint32_t, uint32_t w) const { return depth[w]; }
    // update word: the old depth of w when the plain load let an update through
    ATOS_DEV uint64_t edge(uint32_t, uint32_t, uint32_t nd, uint32_t, uint32_t w, Nbr dw,
                           uint64_t*) const {
        uint32_t old = 0u;
        if (nd < dw) old = min_agent(depth + w, nd);
        return old;
    }
    ATOS_DEV bool decide(uint32_t, uint32_t, uint32_t nd, uint32_t, Nbr dw, uint64_t word,
                         uint32_t& paux, uint64_t*) const {
        paux = nd & 0xFFFFu;
        return nd < dw && nd < (uint32_t)word;
    }
    ATOS_DEV uint32_t finish(uint32_t, uint32_t&, uint32_t, uint32_t&, uint64_t*, uint32_t&,
                             uint32_t&) const {
        return kFinishNone;
    }
};

// Asynchronous push PageRank (Algorithm 4 with threshold-crossing enqueue):
// take the vertex's whole residue, add it to its rank, push damping*res/deg
// to every neighbour, and enqueue a neighbour exactly when this addition
// lifts its residue from <= eps to > eps.  Invariant: every vertex with
// residue > eps is queued or being processed, so termination implies every
// residue <= eps.
//
// Ranks and residues are FP64.  A hub's residue collects one increment per
// neighbour push between two pops of the hub; in FP32 an increment below half
// an ulp of the collected residue (1e-7-sized pushes onto a residue of ~100)
// is lost outright and larger ones are rounded the same way again and again,
// which moves the hub's rank by far more than the accuracy asked of it.  The
// output is rounded to FP32 once at the end.  The per-task push amount
// damping*res/deg travels in the task's 64-bit accumulator word.
struct PrApp {
    double* rank;
    double* residue;
    double damping;
    double eps;
    uint32_t first;  // initial task i is vertex first + i (global: every vertex; personalized: the source)
    static constexpr int kAccWords = 1;
    static constexpr bool kHasFinish = false;
    static constexpr bool kHasNotify = false;
    static constexpr bool kSplittable = true;

    ATOS_DEV void init_task(uint64_t i, uint32_t& v, uint32_t& aux) const {
        v = first + (uint32_t)i;
        aux = 0u;
    }
    ATOS_DEV bool prepare(uint32_t v, uint32_t, uint32_t deg, uint32_t&, uint64_t* acc) const {
        const double r = exch_agent(residue + v, 0.0);
        if (!(r > 0.0)) return false;
        add_agent(rank + v, r);
        if (deg == 0u) return false;
        acc[0] = (uint64_t)__double_as_longlong(damping * r / (double)deg);
        return true;
    }
    using Nbr = uint32_t;  // nothing to read ahead: the update is one atomic
    ATOS_DEV Nbr gather(uint32_t, uint32_t, uint32_t) const { return 0u; }
    // update word: the bits of w's residue before this push
    ATOS_DEV uint64_t edge(uint32_t, uint32_t, uint32_t, uint32_t, uint32_t w, Nbr, uint64_t* acc) const {
        const double delta = __longlong_as_double((long long)*acc);
        return (uint64_t)__double_as_longlong(add_agent(residue + w, delta));
    }
    ATOS_DEV bool decide(uint32_t, uint32_t, uint32_t, uint32_t, Nbr, uint64_t word, uint32_t& paux,
                         uint64_t* acc) const {
        const double delta = __longlong_as_double((long long)*acc);
        const double old = __longlong_as_double((long long)word);
        paux = 0u;
        return old <= eps && old + delta > eps;
    }
    ATOS_DEV uint32_t finish(uint32_t, uint32_t&, uint32_t, uint32_t&, uint64_t*, uint32_t&,
                             uint32_t&) const {
        return kFinishNone;
    }
};

// PageRank with the residue updates of the highest-degree vertices combined
// per worker.  The worker reads a copy of the column array in which every
// entry naming one of those vertices holds kCombTag | its slot (slot < the
// number of combined vertices <= kCombSlots).  An update of such an entry is
// added to the worker's LDS table instead of the device residue; when the
// table is flushed (after a set number of edges, and whenever the worker
// finds no task) each non-empty slot becomes one device atomic whose result
// takes the same threshold-crossing decision on the combined amount.  On a
// scale-free graph the top few thousand vertices receive a fifth to a third
// of all updates, many of them repeatedly within one flush window, so the
// device performs fewer atomics for the same updates.  The sums are exact up
// to the order of FP64 rounding; a vertex's residue reaches the device later,
// which the asynchronous method allows.
constexpr uint32_t kCombTag = 0x80000000u;

struct PrCombApp : PrApp {
    const uint32_t* comb_vertex;  // [kCombSlots] vertex of each slot
    double* comb;                 // the worker's LDS table (set by the kernel)
    static constexpr uint32_t kCombSlots = 12288;
    static constexpr uint32_t kCombAux = 0u;  // aux word of a task a flush pushes

    ATOS_DEV uint64_t edge(uint32_t, uint32_t, uint32_t, uint32_t, uint32_t w, Nbr, uint64_t* acc) const {
        const double delta = __longlong_as_double((long long)*acc);
        if (w & kCombTag) {
            (void)atomicAdd(comb + (w & ~kCombTag), delta);
            return 0ull;
        }
        return (uint64_t)__double_as_longlong(add_agent(residue + w, delta));
    }
    ATOS_DEV bool decide(uint32_t v, uint32_t aux, uint32_t val, uint32_t w, Nbr nb, uint64_t word,
                         uint32_t& paux, uint64_t* acc) const {
        paux = 0u;
        if (w & kCombTag) return false;  // decided when the slot is flushed
        return PrApp::decide(v, aux, val, w, nb, word, paux, acc);
    }
    // flush of a slot of vertex w holding x: the device update and its crossing test
    ATOS_DEV uint64_t comb_issue(uint32_t w, double x) const {
        return (uint64_t)__double_as_longlong(add_agent(residue + w, x));
    }
    ATOS_DEV bool comb_decide(double x, uint64_t word) const {
        const double old = __longlong_as_double((long long)word);
        return old <= eps && old + x > eps;
    }
};

// Asynchronous push PageRank with Algorithm 4's enqueue rule: a task moves
// its residue into its rank and adds damping*res/deg to every neighbour's
// residue without looking at the result (no task is pushed from an edge);
// after each task its worker takes the next Check_Size positions of a
// round-robin cursor over all vertices (one fetch-add per batch for all its
// tasks) and pushes every vertex found with residue > eps that is not
// already queued.  A vertex raised above eps after the cursor passed it is
// found by a later sweep, or, once the worklist has drained, by the caller's
// clean sweep of every vertex, whose finds are the initial tasks of the next
// launch.  Initial task i is vertex i, or list[i] when a list is given.
// The queued flag (set by the push, cleared by the pop before the residue is
// taken) keeps a vertex in the worklist once: without it every sweep that
// passes a vertex still above eps would queue it again, and while most
// residues are above eps each task would queue up to Check_Size more tasks.
struct PrSweepApp {
    double* rank;
    double* residue;
    uint32_t* queued;
    double damping;
    double eps;
    const uint32_t* list;  // initial tasks of a launch after the first, or null
    uint32_t check_size;   // Check_Size: positions swept per task
    static constexpr int kAccWords = 1;
    static constexpr bool kHasFinish = false;
    static constexpr bool kHasNotify = false;
    static constexpr bool kSplittable = true;
    static constexpr bool kHasSweep = true;

    ATOS_DEV void init_task(uint64_t i, uint32_t& v, uint32_t& aux) const {
        v = list ? list[i] : (uint32_t)i;
        aux = 0u;
    }
    ATOS_DEV bool prepare(uint32_t v, uint32_t, uint32_t deg, uint32_t&, uint64_t* acc) const {
        st_agent(queued + v, 0u);
        wait_vmem();  // unqueued before the residue is taken: a later rise is queued again
        const double r = exch_agent(residue + v, 0.0);
        if (!(r > 0.0)) return false;
        add_agent(rank + v, r);
        if (deg == 0u) return false;
        acc[0] = (uint64_t)__double_as_longlong(damping * r / (double)deg);
        return true;
    }
    using Nbr = uint32_t;
    ATOS_DEV Nbr gather(uint32_t, uint32_t, uint32_t) const { return 0u; }
    // the residue addition's old value is not needed: a non-returning atomic
    ATOS_DEV uint64_t edge(uint32_t, uint32_t, uint32_t, uint32_t, uint32_t w, Nbr, uint64_t* acc) const {
        const double delta = __longlong_as_double((long long)*acc);
        (void)add_agent(residue + w, delta);
        return 0ull;
    }
    ATOS_DEV bool decide(uint32_t, uint32_t, uint32_t, uint32_t, Nbr, uint64_t, uint32_t& paux,
                         uint64_t*) const {
        paux = 0u;
        return false;
    }
    ATOS_DEV uint32_t finish(uint32_t, uint32_t&, uint32_t, uint32_t&, uint64_t*, uint32_t&,
                             uint32_t&) const {
        return kFinishNone;
    }
    // positions a batch of k tasks sweeps, and whether vertex v is pushed
    ATOS_DEV uint32_t sweep_positions(uint32_t k) const { return k * check_size; }
    ATOS_DEV bool sweep_test(uint32_t v) const {
        return ld_agent(residue + v) > eps && ld_agent(queued + v) == 0u &&
               exch_agent(queued + v, 1u) == 0u;
    }
};

// Algorithm 4's rule with the residue updates of the highest-degree vertices
// combined per worker (as PrCombApp).  A flush only adds the sums to the
// device residues: the sweeps enqueue, as for every other update.
struct PrSweepCombApp : PrSweepApp {
    const uint32_t* comb_vertex;  // [kCombSlots] vertex of each slot
    double* comb;                 // the worker's LDS table (set by the kernel)
    static constexpr uint32_t kCombSlots = PrCombApp::kCombSlots;
    static constexpr uint32_t kCombAux = 0u;

    ATOS_DEV uint64_t edge(uint32_t v, uint32_t aux, uint32_t val, uint32_t deg, uint32_t w, Nbr nb,
                           uint64_t* acc) const {
        if (w & kCombTag) {
            (void)atomicAdd(comb + (w & ~kCombTag), __longlong_as_double((long long)*acc));
            return 0ull;
        }
        return PrSweepApp::edge(v, aux, val, deg, w, nb, acc);
    }
    ATOS_DEV uint64_t comb_issue(uint32_t w, double x) const {
        (void)add_agent(residue + w, x);
        return 0ull;
    }
    ATOS_DEV bool comb_decide(double, uint64_t) const { return false; }
};

// Colouring rank.  Vertices are totally ordered by (key, id), key packing
// min(degree, 65535) in the high 16 bits and the top 16 bits of a 32-bit hash
// of (seed, id) in the low ones: higher degree outranks lower, the random
// hash breaks ties.  A vertex forbids only the colours of neighbours that
// outrank it; when it collides with a lower-ranked neighbour, that neighbour
// recolours.  The top vertex of any conflict never moves, so runs terminate,
// and every colour is at most the vertex's number of outranking neighbours.
ATOS_DEV uint32_t colour_key(uint64_t seed, uint32_t v, uint64_t deg) {
    const uint32_t d = deg > 0xFFFFull ? 0xFFFFu : (uint32_t)deg;
    return (d << 16) | (priority_hash(seed, v) >> 16);
}
ATOS_DEV bool outranks(const uint32_t* key, uint32_t w, uint32_t v) {
    const uint32_t kw = key[w], kv = key[v];
    return kw != kv ? kw > kv : w > v;
}
// Ordered class: vertices with at least `order` neighbours (order > 0).  All
// outranking neighbours of a class vertex have at least its degree, so they
// are in the class too.
ATOS_DEV bool ordered_key(uint32_t key, uint32_t order) {
    return order != 0u && (key >> 16) >= order;
}

// Colour windows: an assignment ORs the colours of outranking neighbours that
// fall in [val, val + 256) into a 256-bit mask (four accumulator words) and
// takes the lowest free one; when all 256 are taken it scans again with the
// next window.
constexpr int kColourWords = 4;
constexpr uint32_t kColourWindow = 64u * kColourWords;

ATOS_DEV void colour_mark(uint64_t* mask, uint32_t base, int32_t cw) {
    const uint32_t rel = (uint32_t)cw - base;
    if (cw >= 0 && rel < kColourWindow) atomicOr((unsigned long long*)&mask[rel >> 6], 1ull << (rel & 63u));
}
// lowest free colour of the window, or -1 when the window is full
ATOS_DEV int32_t colour_first_free(const uint64_t* mask, uint32_t base) {
#pragma unroll
    for (int j = 0; j < kColourWords; ++j)
        if (mask[j] != ~0ull) return (int32_t)(base + 64u * j + (uint32_t)__builtin_ctzll(~mask[j]));
    return -1;
}

// Speculative greedy colouring as one uberkernel (Algorithm 6).  aux 0 =
// assign, aux 1 = conflict check (the paper's sign of the task word).
//   assign(v): clear v's queued flag, take the lowest colour no outranking
//     neighbour holds (colour windows above), store it, push check(v).
//   check(v): for every neighbour w holding v's colour, the lower-ranked
//     endpoint is sent back to assign, at most once while queued.
// Ordered class (see ordered_key): such a vertex is not coloured
// speculatively.  wait[v] counts its outranking neighbours without a colour;
// its assign is skipped while wait[v] > 0 or once it holds a colour (the
// colour is set once, by compare-and-swap from -1), and the check of a class
// vertex u decrements wait[w] of every lower-ranked class neighbour w,
// pushing assign(w) when it reaches zero.  A class vertex therefore takes its
// colour once, from final colours of all its outranking neighbours: first-fit
// in rank order within the class, with no cascade of recolouring among the
// densely connected high-degree vertices.  Its check runs in the same task,
// as a second pass over its edges right after the colour is set (its colour
// is final, so nothing is gained by queueing it), which saves a trip through
// the worklist on the class's dependency chain.  Its wake-up is safe against
// its initial task: the decrement that reaches zero happens after the colour
// stores it depends on completed, and the compare-and-swap admits one check
// per vertex.
// Of two adjacent vertices assigned concurrently, at least one check must
// observe the other's final colour (store-buffering pattern): a colour store
// completes before the check that follows it reads neighbour colours (the
// check task is published after its store completed, or, for a class
// vertex, the compare-and-swap has returned), and checks read neighbour
// colours at the coherence point, so the later of the two checks sees the
// earlier store.
struct GcApp {
    int32_t* color;
    uint32_t* queued;
    const uint32_t* key;
    uint32_t* wait;
    uint64_t* mask;  // per class vertex: colours < 256 of its outranking class neighbours
    uint32_t order;  // ordered-class degree, 0 = none
    uint32_t forbid_all;  // speculative assignments avoid every neighbour's colour (Alg 6 as printed)
    static constexpr int kAccWords = kColourWords;
    static constexpr bool kHasFinish = true;
    static constexpr bool kHasNotify = true;
    // assign and check reduce over a task's edges by OR (colour mask, recolour
    // bit), so a long neighbour list can be split over workers
    static constexpr bool kSplittable = true;

    ATOS_DEV void init_task(uint64_t i, uint32_t& v, uint32_t& aux) const {
        v = (uint32_t)i;  // assign(v) for every vertex, in ID order
        aux = 0u;
    }
    ATOS_DEV bool prepare(uint32_t v, uint32_t& aux, uint32_t, uint32_t& val, uint64_t*) const {
        if (aux == 0u) {
            if (ordered_key(key[v], order)) {
                const uint32_t wt = ld_agent(wait + v);  // both loads in flight together
                const int32_t cv = ld_agent(color + v);
                if (wt != 0u || cv >= 0) return false;  // not ready yet, or already coloured
                st_agent(queued + v, 0u);
                // Every outranking neighbour is a class vertex with its final colour,
                // and each ORed its colour (if < 256) into mask[v] before counting
                // itself off wait[v]: the first free colour needs no neighbour scan.
                uint64_t m[kColourWords];
#pragma unroll
                for (int j = 0; j < kColourWords; ++j) m[j] = ld_agent(mask + (uint64_t)v * kColourWords + j);
                const int32_t c = colour_first_free(m, 0u);
                if (c < 0) {  // 0..255 all taken: scan the neighbours from the next window
                    val = kColourWindow;
                    return true;
                }
                if (!cas_agent(color + v, -1, c)) return false;  // coloured already
                aux = 1u;  // straight to its check pass
                val = (uint32_t)c;
                return true;
            }
            st_agent(queued + v, 0u);
            val = 0u;  // colour window base
        } else {
            val = (uint32_t)ld_agent(color + v);
        }
        return true;
    }

    struct Nbr {
        int32_t colour;
        uint32_t key;
        uint32_t kv;  // key of v
    };
    ATOS_DEV Nbr gather(uint32_t v, uint32_t, uint32_t w) const {
        return Nbr{ld_agent(color + w), key[w], key[v]};
    }
    // What a check pass of v does for neighbour w with the colour v took (val):
    // 1 = w is lower-ranked with the same colour: w recolours (flagged once in
    // queued[w]); 2 = w is a lower-ranked class neighbour of the class vertex
    // v: one outranking colour less for w to wait for; 0 = nothing.
    ATOS_DEV uint32_t check_case(uint32_t v, uint32_t val, uint32_t w, const Nbr& nb) const {
        if (w == v) return 0u;
        const bool w_up = nb.key != nb.kv ? nb.key > nb.kv : w > v;
        if (w_up) return 0u;
        if (nb.colour == (int32_t)val) return 1u;
        return (ordered_key(nb.kv, order) && ordered_key(nb.key, order)) ? 2u : 0u;
    }
    // check pass of a class vertex v (colour val): record val in the mask of
    // each lower-ranked class neighbour before counting v off its wait
    ATOS_DEV void notify(uint32_t v, uint32_t aux, uint32_t val, uint32_t w, const Nbr& nb) const {
        if (aux != 0u && val < kColourWindow && check_case(v, val, w, nb) == 2u)
            or_agent(mask + (uint64_t)w * kColourWords + (val >> 6), (uint64_t)1 << (val & 63u));
    }
    // update word: the old value of the one counter the check updated (queued
    // flag: +1, the first flagger pushes; wait counter: -1, the last pushes)
    ATOS_DEV uint64_t edge(uint32_t v, uint32_t aux, uint32_t val, uint32_t, uint32_t w, const Nbr& nb,
                           uint64_t* acc) const {
        // (one exit: every path returns the one register the atomic writes)
        uint32_t old = 0u;
        uint32_t c = 0u;
        if (w != v) {
            const bool w_up = nb.key != nb.kv ? nb.key > nb.kv : w > v;  // w outranks v
            if (aux == 0u) {
                // with forbid_all a speculative vertex avoids every neighbour's
                // colour; a class vertex (coloured once, in rank order) its
                // outranking neighbours' colours, as its mask holds them
                if (w_up || (forbid_all && !ordered_key(nb.kv, order))) colour_mark(acc, val, nb.colour);
            } else if (w_up) {
                if (nb.colour == (int32_t)val)
                    atomicOr((unsigned long long*)acc, 1ull);  // v recolours (once, in finish)
            } else {
                c = check_case(v, val, w, nb);
            }
        }
        if (c != 0u) old = add_agent(c == 1u ? queued + w : wait + w, c == 1u ? 1u : ~0u);
        return old;
    }
    ATOS_DEV bool decide(uint32_t v, uint32_t aux, uint32_t val, uint32_t w, const Nbr& nb,
                         uint64_t word, uint32_t& paux, uint64_t*) const {
        paux = 0u;  // assign(w)
        if (aux == 0u) return false;
        const uint32_t c = check_case(v, val, w, nb);
        return (c == 1u && (uint32_t)word == 0u) || (c == 2u && (uint32_t)word == 1u);
    }
    ATOS_DEV uint32_t finish(uint32_t v, uint32_t& aux, uint32_t, uint32_t& val, uint64_t* acc,
                             uint32_t& pv, uint32_t& paux) const {
        if (aux == 0u) {
            const int32_t c = colour_first_free(acc, val);
            if (c < 0) {  // the whole window is taken: scan again with the next one
                val += kColourWindow;
#pragma unroll
                for (int j = 0; j < kColourWords; ++j) acc[j] = 0;
                return kFinishRepeat;
            }
            if (ordered_key(key[v], order)) {
                if (!cas_agent(color + v, -1, c)) return kFinishNone;  // coloured already
                aux = 1u;  // its check, as a second pass in this task
                val = (uint32_t)c;
#pragma unroll
                for (int j = 0; j < kColourWords; ++j) acc[j] = 0;
                return kFinishRepeat;
            }
            st_agent(color + v, c);
            pv = v;
            paux = 1u;  // check(v)
            return kFinishPush;
        }
        if ((acc[0] & 1ull) && add_agent(queued + v, 1u) == 0u) {
            pv = v;
            paux = 0u;
            return kFinishPush;
        }
        return kFinishNone;
    }
};

// Batched BFS and PageRank instances in one persistent launch.  Instances are
// disjoint vertex ranges of one union graph whose edges never leave their
// range, so tasks stay inside their instance with no lookup.  The task's aux
// word carries the application: bit 15 set = PageRank task, clear = BFS task
// with the low 15 bits of its pusher's depth.  `state` holds the BFS depth
// (u32) of BFS vertices; PageRank ranks accumulate in `rank` and are written
// to `state` as FP32 bits when the run ends.
struct BatchTables {
    const uint32_t* bfs_src;     // [n_bfs] BFS sources, in instance order
    const uint64_t* pr_prefix;   // [n_pr + 1] exclusive prefix of PageRank range sizes
    const uint32_t* pr_begin;    // [n_pr] first vertex of each PageRank range
    uint32_t n_bfs;
    uint32_t n_pr;
};

constexpr uint32_t kBatchPr = 0x8000u;

struct BatchApp {
    uint32_t* state;
    double* rank;     // FP64 rank accumulator of PageRank vertices (see PrApp)
    double* residue;  // FP64 residues of PageRank vertices (see PrApp)
    double damping;
    double eps;
    BatchTables t;
    static constexpr int kAccWords = 1;
    static constexpr bool kHasFinish = false;
    static constexpr bool kHasNotify = false;
    static constexpr bool kSplittable = true;

    // initial tasks: every BFS source, then every vertex of every PageRank range
    ATOS_DEV void init_task(uint64_t i, uint32_t& v, uint32_t& aux) const {
        if (i < t.n_bfs) {
            v = t.bfs_src[i];
            aux = 0u;
            return;
        }
        const uint64_t j = i - t.n_bfs;
        uint32_t lo = 0, hi = t.n_pr;  // range k with pr_prefix[k] <= j < pr_prefix[k+1]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (t.pr_prefix[mid] <= j) lo = mid; else hi = mid;
        }
        v = t.pr_begin[lo] + (uint32_t)(j - t.pr_prefix[lo]);
        aux = kBatchPr;
    }
    ATOS_DEV bool prepare(uint32_t v, uint32_t aux, uint32_t deg, uint32_t& val, uint64_t* acc) const {
        if (aux & kBatchPr) {
            const double r = exch_agent(residue + v, 0.0);
            if (!(r > 0.0)) return false;
            add_agent(rank + v, r);
            if (deg == 0u) return false;
            acc[0] = (uint64_t)__double_as_longlong(damping * r / (double)deg);
            return true;
        }
        const uint32_t d = ld_agent(state + v);
        val = d + 1u;
        return (d & 0x7FFFu) == aux;
    }
    using Nbr = uint32_t;  // BFS: the neighbour's depth (plain load, see BfsApp)
    ATOS_DEV Nbr gather(uint32_t, uint32_t aux, uint32_t w) const { return (aux & kBatchPr) ? 0u : state[w]; }
    ATOS_DEV uint64_t edge(uint32_t, uint32_t aux, uint32_t val, uint32_t, uint32_t w, Nbr dw,
                           uint64_t* acc) const {
        if (aux & kBatchPr) {
            const double delta = __longlong_as_double((long long)*acc);
            return (uint64_t)__double_as_longlong(add_agent(residue + w, delta));
        }
        uint32_t old = 0u;
        if (val < dw) old = min_agent(state + w, val);
        return old;
    }
    // update word: PageRank: the bits of w's old residue; BFS: w's old state
    // when the plain load let an update through
    ATOS_DEV bool decide(uint32_t, uint32_t aux, uint32_t val, uint32_t, Nbr dw, uint64_t word,
                         uint32_t& paux, uint64_t* acc) const {
        if (aux & kBatchPr) {
            const double delta = __longlong_as_double((long long)*acc);
            const double old = __longlong_as_double((long long)word);
            paux = kBatchPr;
            return old <= eps && old + delta > eps;
        }
        paux = val & 0x7FFFu;
        return val < dw && val < (uint32_t)word;
    }
    ATOS_DEV uint32_t finish(uint32_t, uint32_t&, uint32_t, uint32_t&, uint64_t*, uint32_t&,
                             uint32_t&) const {
        return kFinishNone;
    }
};

// A batch whose PageRank instances combine the residue updates of their
// highest-degree vertices (as PrCombApp).  Only PageRank instances' edges are
// tagged in the column copy, so BFS tasks read plain neighbour ids.
struct BatchCombApp : BatchApp {
    const uint32_t* comb_vertex;  // [kCombSlots] vertex of each slot
    double* comb;                 // the worker's LDS table (set by the kernel)
    static constexpr uint32_t kCombSlots = PrCombApp::kCombSlots;
    static constexpr uint32_t kCombAux = kBatchPr;

    ATOS_DEV uint64_t edge(uint32_t v, uint32_t aux, uint32_t val, uint32_t deg, uint32_t w, Nbr dw,
                           uint64_t* acc) const {
        if ((aux & kBatchPr) && (w & kCombTag)) {
            (void)atomicAdd(comb + (w & ~kCombTag), __longlong_as_double((long long)*acc));
            return 0ull;
        }
        return BatchApp::edge(v, aux, val, deg, w, dw, acc);
    }
    ATOS_DEV bool decide(uint32_t v, uint32_t aux, uint32_t val, uint32_t w, Nbr dw, uint64_t word,
                         uint32_t& paux, uint64_t* acc) const {
        if ((aux & kBatchPr) && (w & kCombTag)) {
            paux = kBatchPr;
            return false;  // decided when the slot is flushed
        }
        return BatchApp::decide(v, aux, val, w, dw, word, paux, acc);
    }
    ATOS_DEV uint64_t comb_issue(uint32_t w, double x) const {
        return (uint64_t)__double_as_longlong(add_agent(residue + w, x));
    }
    ATOS_DEV bool comb_decide(double x, uint64_t word) const {
        const double old = __longlong_as_double((long long)word);
        return old <= eps && old + x > eps;
    }
};

}  // namespace atos
