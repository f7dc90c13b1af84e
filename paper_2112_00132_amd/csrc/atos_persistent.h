// Persistent worklist kernel (paper section 3, Listing 2; section 3.4).
//
// Every workgroup of the grid is one worker (BLOCK = 64 is the wavefront
// worker, the counterpart of the paper's warp worker; BLOCK = 128..1024 are
// workgroup workers, the counterpart of its CTA worker).  A worker loops:
//
//   claim FETCH consecutive ring positions with one atomic on `head`
//   take the tasks already published in those positions (FULL slots), stage
//   them in LDS, mark the slots FREE for the next lap
//   per task: read its neighbour range, run the application's `prepare`
//   exclusive scan of the tasks' edge counts; load-balancing search maps
//   every edge of the batch to one thread (section 3.3: data parallelism
//   inside the worker on top of task parallelism across workers)
//   per edge: the application's `edge` callback, which may emit a new task
//   new tasks are gathered in LDS with ballot/mbcnt and published with one
//   atomic on `tail` per flush
//   `done += tasks taken`
//
// Positions a worker claimed but that are not yet published stay owned by
// it and are retried.  Termination: `tail` is advanced when a task is
// reserved (before the task that produced it is counted in `done`), so
// done == tail means every task ever reserved has been processed and none
// can appear again; an idle worker that observes it (reading done first)
// exits.  Every wait is bounded by a device deadline and by the status word.
#pragma once

#include "atos_device.h"

namespace atos {

template <class OffT>
struct PersistArgs {
    const OffT* offs;
    const int32_t* cols;
    int64_t n;
    WsHeader* hdr;
    RingView ring;
    int32_t fetch;         // tasks claimed per pop, 1..BLOCK
    uint32_t push_spin_limit;
    uint64_t timeout_ticks;
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
    __shared__ uint64_t s_acc[BLOCK];
    __shared__ uint64_t s_push[PUSH_CAP];
    __shared__ uint32_t s_wsum[NW + 1];
    __shared__ uint32_t s_push_n;
    __shared__ uint32_t s_k;
    __shared__ uint32_t s_claimed;
    __shared__ uint32_t s_stop;
    __shared__ uint64_t s_pop_base;
    __shared__ uint64_t s_push_base;

    const int tid = threadIdx.x;
    WsHeader* H = a.hdr;
    const RingView R = a.ring;
    const uint32_t F = (uint32_t)a.fetch;
    const uint64_t deadline = now_ticks() + a.timeout_ticks;

    // ---- publish the initial tasks (positions init_base .. init_base + n_init - 1)
    {
        const uint64_t base0 = ld_agent(&H->init_base);
        const uint64_t n_init = ld_agent(&H->n_init);
        for (uint64_t i = (uint64_t)blockIdx.x * BLOCK + tid; i < n_init;
             i += (uint64_t)gridDim.x * BLOCK) {
            uint32_t v, aux;
            app.init_task(i, v, aux);
            const uint64_t pos = base0 + i;
            if (!cas_agent(R.slot(pos), R.free_word(pos), R.full_word(pos, make_payload(v, aux)))) {
                or_agent(&H->status, (uint32_t)kStatusCorrupt);
            }
        }
    }
    if (tid == 0) {
        s_push_n = 0;
        s_k = 0;
    }

    bool my_pending = false;
    uint64_t my_pos = 0;
    uint32_t pending_cnt = 0;
    uint32_t spin = 0;
    uint64_t st_pop = 0, st_push = 0, st_edges = 0;

    // Publish the tasks gathered in s_push: reserve positions with one atomic
    // on tail, then turn each slot FREE -> FULL.  Called by all threads.
    auto flush = [&]() {
        __syncthreads();
        const uint32_t n = s_push_n;
        if (n == 0) return;
        if constexpr (App::kSeqCstPublish) {
            fence_seqcst_agent();
        } else {
            fence_release_agent();
        }
        if (tid == 0) s_push_base = add_agent(&H->tail, (uint64_t)n);
        __syncthreads();
        const uint64_t base = s_push_base;
        for (uint32_t i = tid; i < n; i += BLOCK) {
            const uint64_t pos = base + i;
            const uint64_t want = R.free_word(pos);
            const uint64_t full = R.full_word(pos, s_push[i]);
            uint32_t tries = 0;
            while (!cas_agent(R.slot(pos), want, full)) {
                // The previous lap's task in this slot has not been taken yet.
                if (ld_agent(&H->status) != 0u) break;
                if (++tries > a.push_spin_limit) {
                    or_agent(&H->status, (uint32_t)kStatusOverflow);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
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

    __syncthreads();
    for (;;) {
        // ---- pop: claim a window of F positions when the previous one is used up
        if (pending_cnt == 0) {
            if (tid == 0) {
                uint32_t got = 0;
                if (ld_agent(&H->status) != 0u) {
                    got = 2;  // another worker stopped the run
                } else if (now_ticks() > deadline) {
                    or_agent(&H->status, (uint32_t)kStatusTimeout);
                    got = 2;
                } else {
                    const uint64_t h = ld_agent(&H->head);
                    const uint64_t t = ld_agent(&H->tail);
                    if (h < t) {
                        s_pop_base = add_agent(&H->head, (uint64_t)F);
                        got = 1;
                    }
                }
                s_claimed = got;
            }
            __syncthreads();
            if (s_claimed == 2) break;
            if (s_claimed == 1) {
                my_pos = s_pop_base + (uint64_t)tid;
                my_pending = (uint32_t)tid < F;
                pending_cnt = F;
            }
        }
        bool got = false;
        uint64_t word = 0;
        if (my_pending) {
            word = ld_agent(R.slot(my_pos));
            if (R.is_full_for(word, my_pos)) {
                got = true;
                my_pending = false;
                st_agent(R.slot(my_pos), R.free_word(my_pos + R.mask + 1));
            }
        }
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
        pending_cnt = (uint32_t)__syncthreads_count(my_pending);
        const uint32_t k = s_k;
        if (k == 0) {
            // ---- idle: stop on error, on termination (done == tail), or at the deadline
            if (tid == 0) {
                uint32_t stop = 0;
                if (ld_agent(&H->status) != 0u) {
                    stop = 1;
                } else {
                    const uint64_t d = __hip_atomic_load(&H->done, __ATOMIC_ACQUIRE,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t t = ld_agent(&H->tail);
                    if (d == t) {
                        stop = 1;
                    } else if (now_ticks() > deadline) {
                        or_agent(&H->status, (uint32_t)kStatusTimeout);
                        stop = 1;
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
        if constexpr (App::kSeqCstPublish) {
            fence_seqcst_agent();
        } else {
            fence_acquire_agent();
        }

        // ---- per task: neighbour range and application prepare
        if ((uint32_t)tid < k) {
            const uint32_t v = s_vert[tid];
            const OffT beg = a.offs[v];
            const OffT end = a.offs[v + 1];
            uint32_t val = 0;
            uint64_t acc = 0;
            const uint32_t deg = (uint32_t)(end - beg);
            const bool active = app.prepare(v, s_aux[tid], deg, val, acc);
            s_start[tid] = beg;
            s_deg[tid] = deg;
            s_val[tid] = val;
            s_acc[tid] = acc;
            s_active[tid] = active ? 1u : 0u;
        }
        __syncthreads();

        bool repeat;
        do {
            const uint32_t cnt = ((uint32_t)tid < k && s_active[tid]) ? s_deg[tid] : 0u;
            uint32_t total;
            const uint32_t ex = block_exclusive_scan<BLOCK>(cnt, s_wsum, total);
            if ((uint32_t)tid < k) s_scan[tid] = ex;
            if (tid == 0) s_scan[k] = total;
            __syncthreads();
            if (tid == 0) st_edges += total;

            // ---- load-balancing search over the batch's edges
            // (s_push_n is stable here: the last append was before the previous barrier)
            const bool may_overflow = s_push_n + total + BLOCK > (uint32_t)PUSH_CAP;
            for (uint32_t eb = 0; eb < total; eb += BLOCK) {
                const uint32_t e = eb + (uint32_t)tid;
                bool push = false;
                uint64_t payload = 0;
                if (e < total) {
                    const uint32_t i = lbs_search(s_scan, k, e);
                    const OffT idx = s_start[i] + (OffT)(e - s_scan[i]);
                    const uint32_t w = (uint32_t)a.cols[idx];
                    uint32_t paux = 0;
                    push = app.edge(s_vert[i], s_aux[i], s_val[i], s_deg[i], w, paux, &s_acc[i]);
                    payload = make_payload(w, paux);
                }
                append(push, payload);
                if (may_overflow && push_buffer_nearly_full()) flush();
            }

            // ---- per task: application finish (may emit one task, or ask for another pass)
            repeat = false;
            if constexpr (App::kHasFinish) {
                if (push_buffer_nearly_full()) flush();
                bool push = false;
                uint64_t payload = 0;
                bool again = false;
                if ((uint32_t)tid < k && s_active[tid]) {
                    uint32_t pv = 0, paux = 0;
                    uint32_t val = s_val[tid];
                    uint64_t acc = s_acc[tid];
                    const uint32_t r = app.finish(s_vert[tid], s_aux[tid], s_deg[tid], val, acc,
                                                  pv, paux);
                    if (r == kFinishPush) {
                        push = true;
                        payload = make_payload(pv, paux);
                    } else if (r == kFinishRepeat) {
                        again = true;
                    }
                    s_val[tid] = val;
                    s_acc[tid] = acc;
                }
                if ((uint32_t)tid < k) s_active[tid] = again ? 1u : 0u;
                append(push, payload);
                repeat = __syncthreads_or(again) != 0;
            }
        } while (repeat);

        flush();
        if (tid == 0) {
            st_pop += k;
            s_k = 0;
            __hip_atomic_fetch_add(&H->done, (uint64_t)k, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }

    if (tid == 0) {
        add_agent(&H->stat_popped, st_pop);
        add_agent(&H->stat_pushed, st_push);
        add_agent(&H->stat_edges, st_edges);
        if (ld_agent(&H->status) != 0u) st_agent(&H->cookie, (uint64_t)0);
    }
}

// ------------------------------------------------------------------ applications
// Each application supplies:
//   init_task(i, v, aux)              vertex and aux word of initial task i
//   prepare(v, aux, deg, val, acc)    per popped task; returns whether the task
//                                     is processed (its edges scanned, finish run)
//   edge(v, aux, val, deg, w, paux, acc)  per neighbour w of v (deg = deg(v));
//                                     returns whether to push w
//   finish(...)                       per processed task after its edges (optional)
//   kSeqCstPublish                    use seq_cst instead of acquire/release fences

// Speculative BFS (Algorithm 2).  A task carries the low 16 bits of the
// depth its pusher set; when the vertex has since been lowered again the
// task is a stale duplicate and is dropped (the newer push expands it).
struct BfsApp {
    uint32_t* depth;
    uint32_t source;
    static constexpr bool kHasFinish = false;
    static constexpr bool kSeqCstPublish = false;

    ATOS_DEV void init_task(uint64_t, uint32_t& v, uint32_t& aux) const {
        v = source;
        aux = 0u;
    }
    ATOS_DEV bool prepare(uint32_t v, uint32_t aux, uint32_t, uint32_t& val, uint64_t&) const {
        const uint32_t d = ld_agent(depth + v);
        val = d + 1u;
        return (d & 0xFFFFu) == aux;
    }
    ATOS_DEV bool edge(uint32_t, uint32_t, uint32_t nd, uint32_t, uint32_t w, uint32_t& paux,
                       uint64_t*) const {
        // A plain load may return an older value, and depths only decrease, so
        // it never hides an improvement: it only filters hopeless updates.
        if (nd >= depth[w]) return false;
        const uint32_t old = min_agent(depth + w, nd);
        paux = nd & 0xFFFFu;
        return nd < old;
    }
    ATOS_DEV uint32_t finish(uint32_t, uint32_t, uint32_t, uint32_t&, uint64_t&, uint32_t&,
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
struct PrApp {
    float* rank;
    float* residue;
    float damping;
    float eps;
    static constexpr bool kHasFinish = false;
    static constexpr bool kSeqCstPublish = false;

    ATOS_DEV void init_task(uint64_t i, uint32_t& v, uint32_t& aux) const {
        v = (uint32_t)i;  // every vertex, in ID order
        aux = 0u;
    }
    ATOS_DEV bool prepare(uint32_t v, uint32_t, uint32_t deg, uint32_t& val, uint64_t&) const {
        const float r = exch_agent(residue + v, 0.0f);
        if (!(r > 0.0f)) return false;
        add_agent(rank + v, r);
        if (deg == 0u) return false;
        val = __float_as_uint(damping * r / (float)deg);
        return true;
    }
    ATOS_DEV bool edge(uint32_t, uint32_t, uint32_t val, uint32_t, uint32_t w, uint32_t& paux,
                       uint64_t*) const {
        const float delta = __uint_as_float(val);
        const float old = add_agent(residue + w, delta);
        paux = 0u;
        return old <= eps && old + delta > eps;
    }
    ATOS_DEV uint32_t finish(uint32_t, uint32_t, uint32_t, uint32_t&, uint64_t&, uint32_t&,
                             uint32_t&) const {
        return kFinishNone;
    }
};

// Colouring rank.  Vertices are totally ordered by (key, id), key packing
// min(degree, 65535) in the high 16 bits and the top 16 bits of a 32-bit hash
// of (seed, id) in the low ones: higher degree outranks lower, the random
// hash breaks ties.  A vertex forbids only the colours of neighbours that
// outrank it; when it collides with a lower-ranked neighbour, that neighbour
// recolours.  The colouring therefore converges to first-fit in rank order
// whatever the timing of the workers, and the top vertex of any conflict
// never moves, so runs terminate.
ATOS_DEV uint32_t colour_key(uint64_t seed, uint32_t v, uint64_t deg) {
    const uint32_t d = deg > 0xFFFFull ? 0xFFFFu : (uint32_t)deg;
    return (d << 16) | (priority_hash(seed, v) >> 16);
}
ATOS_DEV bool outranks(const uint32_t* key, uint32_t w, uint32_t v) {
    const uint32_t kw = key[w], kv = key[v];
    return kw != kv ? kw > kv : w > v;
}

// Speculative greedy colouring as one uberkernel (Algorithm 6).  aux 0 =
// assign, aux 1 = conflict check (the paper's sign of the task word).
//   assign(v): clear v's queued flag, OR the colours of the outranking
//     neighbours that fall in the 64-colour window [val, val+64) into a mask,
//     take the lowest free colour (next window when all 64 are used), store
//     it, push check(v).
//   check(v): for every neighbour w holding v's colour, the lower-ranked
//     endpoint is sent back to assign, at most once while queued.
// Publishing uses seq_cst fences so that of two adjacent vertices assigned
// concurrently, at least one check observes the other's final colour.
struct GcApp {
    int32_t* color;
    uint32_t* queued;
    const uint32_t* key;
    static constexpr bool kHasFinish = true;
    static constexpr bool kSeqCstPublish = true;

    ATOS_DEV void init_task(uint64_t i, uint32_t& v, uint32_t& aux) const {
        v = (uint32_t)i;  // assign(v) for every vertex, in ID order
        aux = 0u;
    }
    ATOS_DEV bool prepare(uint32_t v, uint32_t aux, uint32_t, uint32_t& val, uint64_t& acc) const {
        acc = 0;
        if (aux == 0u) {
            st_agent(queued + v, 0u);
            fence_seqcst_agent();
            val = 0u;  // colour window base
        } else {
            val = (uint32_t)ld_agent(color + v);
        }
        return true;
    }
    ATOS_DEV bool edge(uint32_t v, uint32_t aux, uint32_t val, uint32_t, uint32_t w,
                       uint32_t& paux, uint64_t* acc) const {
        if (w == v) return false;
        const int32_t cw = ld_agent(color + w);
        if (aux == 0u) {
            const uint32_t rel = (uint32_t)cw - val;
            if (cw >= 0 && rel < 64u && outranks(key, w, v))
                atomicOr((unsigned long long*)acc, 1ull << rel);
            return false;
        }
        if (cw != (int32_t)val) return false;
        if (outranks(key, w, v)) {
            atomicOr((unsigned long long*)acc, 1ull);  // v recolours (once, in finish)
            return false;
        }
        if (exch_agent(queued + w, 1u) != 0u) return false;
        paux = 0u;
        return true;
    }
    ATOS_DEV uint32_t finish(uint32_t v, uint32_t aux, uint32_t, uint32_t& val, uint64_t& acc,
                             uint32_t& pv, uint32_t& paux) const {
        if (aux == 0u) {
            if (acc == ~0ull) {  // all 64 colours of this window are taken
                val += 64u;
                acc = 0;
                return kFinishRepeat;
            }
            const int32_t c = (int32_t)(val + (uint32_t)__builtin_ctzll(~acc));
            st_agent(color + v, c);
            pv = v;
            paux = 1u;  // check(v)
            return kFinishPush;
        }
        if ((acc & 1ull) && exch_agent(queued + v, 1u) == 0u) {
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
// (u32) or the PageRank rank (f32 bits) of each vertex.
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
    float* residue;
    float damping;
    float eps;
    BatchTables t;
    static constexpr bool kHasFinish = false;
    static constexpr bool kSeqCstPublish = false;

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
    ATOS_DEV bool prepare(uint32_t v, uint32_t aux, uint32_t deg, uint32_t& val, uint64_t&) const {
        if (aux & kBatchPr) {
            const float r = exch_agent(residue + v, 0.0f);
            if (!(r > 0.0f)) return false;
            add_agent((float*)state + v, r);
            if (deg == 0u) return false;
            val = __float_as_uint(damping * r / (float)deg);
            return true;
        }
        const uint32_t d = ld_agent(state + v);
        val = d + 1u;
        return (d & 0x7FFFu) == aux;
    }
    ATOS_DEV bool edge(uint32_t, uint32_t aux, uint32_t val, uint32_t, uint32_t w, uint32_t& paux,
                       uint64_t*) const {
        if (aux & kBatchPr) {
            const float delta = __uint_as_float(val);
            const float old = add_agent(residue + w, delta);
            paux = kBatchPr;
            return old <= eps && old + delta > eps;
        }
        if (val >= state[w]) return false;
        const uint32_t old = min_agent(state + w, val);
        paux = val & 0x7FFFu;
        return val < old;
    }
    ATOS_DEV uint32_t finish(uint32_t, uint32_t, uint32_t, uint32_t&, uint64_t&, uint32_t&,
                             uint32_t&) const {
        return kFinishNone;
    }
};

}  // namespace atos
