// Level-synchronous (bulk-synchronous) frontier kernels: the in-GPU baselines
// of the paper's Algorithms 1, 3 and 5 (section 5).  One launch processes one
// frontier; the host synchronises between levels (the paper's
// cudaDeviceSynchronize) to read the next frontier's size.
//
// Each workgroup takes BLOCK consecutive frontier entries, scans their
// degrees in LDS and spreads their edges over its threads with the same
// load-balancing search as the persistent worker; new frontier entries are
// gathered in LDS with ballot/mbcnt and appended with one atomic per flush.
#pragma once

#include "atos_device.h"
#include "atos_persistent.h"

namespace atos {

template <class OffT>
struct FrontierArgs {
    const OffT* offs;
    const int32_t* cols;
    const uint32_t* in;   // frontier entries (vertex ids)
    uint32_t n_in;
    uint32_t* out;        // next frontier (may be null when the app never appends)
    uint32_t* out_count;  // device counter of `out`
    uint64_t* edges;      // running count of neighbour-list entries scanned
};

template <int BLOCK, class App, class OffT>
__global__ __launch_bounds__(BLOCK) void frontier_kernel(FrontierArgs<OffT> a, App app) {
    constexpr int PUSH_CAP = (2 * BLOCK < 512) ? 512 : 2 * BLOCK;
    constexpr int NW = BLOCK / kWave;
    __shared__ uint32_t s_vert[BLOCK];
    __shared__ uint32_t s_val[BLOCK];
    __shared__ uint32_t s_deg[BLOCK];
    __shared__ uint32_t s_active[BLOCK];
    __shared__ OffT s_start[BLOCK];
    __shared__ uint32_t s_scan[BLOCK + 1];
    constexpr int W = App::kAccWords;
    __shared__ uint64_t s_acc[BLOCK * W];
    __shared__ uint32_t s_push[PUSH_CAP];
    __shared__ uint32_t s_wsum[NW + 1];
    __shared__ uint32_t s_push_n;
    __shared__ uint32_t s_push_base;

    const int tid = threadIdx.x;
    const uint64_t first = (uint64_t)blockIdx.x * BLOCK;
    if (first >= a.n_in) return;
    const uint32_t k = (uint32_t)min((uint64_t)BLOCK, (uint64_t)a.n_in - first);
    if (tid == 0) s_push_n = 0;

    auto flush = [&]() {
        __syncthreads();
        const uint32_t n = s_push_n;
        if (n == 0) return;
        if (tid == 0) s_push_base = atomicAdd(a.out_count, n);
        __syncthreads();
        const uint32_t base = s_push_base;
        for (uint32_t i = tid; i < n; i += BLOCK) a.out[base + i] = s_push[i];
        __syncthreads();
        if (tid == 0) s_push_n = 0;
        __syncthreads();
    };
    auto nearly_full = [&]() -> bool {
        __syncthreads();
        return __syncthreads_or(tid == 0 && s_push_n + BLOCK > (uint32_t)PUSH_CAP) != 0;
    };
    auto append = [&](bool push, uint32_t v) {
        const uint64_t m = ballot(push);
        if (m) {
            uint32_t wbase = 0;
            if (lane_id() == (uint32_t)__builtin_ctzll(m))
                wbase = atomicAdd(&s_push_n, (uint32_t)__popcll(m));
            wbase = __shfl(wbase, __builtin_ctzll(m), kWave);
            if (push) s_push[wbase + mbcnt(m)] = v;
        }
    };

    if ((uint32_t)tid < k) {
        const uint32_t v = a.in[first + tid];
        const OffT beg = a.offs[v];
        const OffT end = a.offs[v + 1];
        const uint32_t deg = (uint32_t)(end - beg);
        uint32_t val = 0;
        uint64_t* acc = &s_acc[tid * W];
#pragma unroll
        for (int j = 0; j < W; ++j) acc[j] = 0;
        const bool active = app.prepare(v, deg, val, acc);
        s_vert[tid] = v;
        s_start[tid] = beg;
        s_deg[tid] = deg;
        s_val[tid] = val;
        s_active[tid] = active ? 1u : 0u;
    }
    __syncthreads();

    bool repeat;
    do {
        const uint32_t cnt = ((uint32_t)tid < k && s_active[tid]) ? s_deg[tid] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<BLOCK>(cnt, s_wsum, total);
        if ((uint32_t)tid < k) s_scan[tid] = ex;
        if (tid == 0) {
            s_scan[k] = total;
            if (total) add_agent(a.edges, (uint64_t)total);
        }
        __syncthreads();
        const bool may_overflow = s_push_n + total + BLOCK > (uint32_t)PUSH_CAP;
        for (uint32_t eb = 0; eb < total; eb += BLOCK) {
            const uint32_t e = eb + (uint32_t)tid;
            bool push = false;
            uint32_t w = 0;
            if (e < total) {
                const uint32_t i = lbs_search(s_scan, k, e);
                w = (uint32_t)a.cols[s_start[i] + (OffT)(e - s_scan[i])];
                push = app.edge(s_vert[i], s_val[i], s_deg[i], w, &s_acc[i * W]);
            }
            append(push, w);
            if (may_overflow && nearly_full()) flush();
        }
        repeat = false;
        if constexpr (App::kHasFinish) {
            if (nearly_full()) flush();
            bool push = false, again = false;
            uint32_t pv = 0;
            if ((uint32_t)tid < k && s_active[tid]) {
                uint32_t val = s_val[tid];
                const uint32_t r = app.finish(s_vert[tid], s_deg[tid], val, &s_acc[tid * W]);
                if (r == kFinishPush) {
                    push = true;
                    pv = s_vert[tid];
                } else if (r == kFinishRepeat) {
                    again = true;
                }
                s_val[tid] = val;
            }
            if ((uint32_t)tid < k) s_active[tid] = again ? 1u : 0u;
            append(push, pv);
            repeat = __syncthreads_or(again) != 0;
        }
    } while (repeat);
    flush();
}

// Algorithm 1: expand the frontier; a neighbour joins the next frontier when
// this level's atomic minimum lowered its depth.
struct BspBfs {
    uint32_t* depth;
    static constexpr int kAccWords = 1;
    static constexpr bool kHasFinish = false;
    ATOS_DEV bool prepare(uint32_t v, uint32_t deg, uint32_t& val, uint64_t*) const {
        val = depth[v] + 1u;
        return deg > 0;
    }
    ATOS_DEV bool edge(uint32_t, uint32_t nd, uint32_t, uint32_t w, uint64_t*) const {
        if (nd >= depth[w]) return false;
        return nd < min_agent(depth + w, nd);
    }
    ATOS_DEV uint32_t finish(uint32_t, uint32_t, uint32_t&, uint64_t*) const { return kFinishNone; }
};

// Algorithm 3, first kernel: move every frontier vertex's residue into its
// rank and push damping*res/deg to its neighbours.  The next frontier is
// built by the separate filter kernel (residue > eps).
struct BspPrPush {
    double* rank;     // FP64 accumulator, as in the persistent PageRank
    double* residue;  // FP64, as in the persistent PageRank
    double damping;
    static constexpr int kAccWords = 1;
    static constexpr bool kHasFinish = false;
    ATOS_DEV bool prepare(uint32_t v, uint32_t deg, uint32_t&, uint64_t* acc) const {
        const double r = exch_agent(residue + v, 0.0);
        if (!(r > 0.0)) return false;
        rank[v] += r;  // one frontier entry per vertex in a round: no concurrent update
        if (deg == 0u) return false;
        acc[0] = (uint64_t)__double_as_longlong(damping * r / (double)deg);
        return true;
    }
    ATOS_DEV bool edge(uint32_t, uint32_t, uint32_t, uint32_t w, uint64_t* acc) const {
        add_agent(residue + w, __longlong_as_double((long long)*acc));
        return false;
    }
    ATOS_DEV uint32_t finish(uint32_t, uint32_t, uint32_t&, uint64_t*) const { return kFinishNone; }
};

// Algorithm 5, first kernel: every frontier vertex takes the lowest colour
// not held by an outranking neighbour (256-colour windows; ranks and the
// ordered class as in the persistent colouring, see GcApp).
struct BspGcAssign {
    int32_t* color;
    const uint32_t* key;
    uint32_t* queued;
    const uint32_t* wait;
    uint32_t order;
    uint32_t forbid_all;  // speculative vertices avoid every neighbour's colour (Alg 5 as
                          // printed); ordered-class vertices, coloured once in rank
                          // order, avoid their outranking neighbours' colours either way
    static constexpr int kAccWords = kColourWords;
    static constexpr bool kHasFinish = true;
    ATOS_DEV bool prepare(uint32_t v, uint32_t, uint32_t& val, uint64_t*) const {
        if (ordered_key(key[v], order) && (wait[v] != 0u || color[v] >= 0)) return false;
        queued[v] = 0u;  // this round's check may send v back again
        val = 0u;
        return true;
    }
    ATOS_DEV bool edge(uint32_t v, uint32_t base, uint32_t, uint32_t w, uint64_t* acc) const {
        if (w == v) return false;
        if (outranks(key, w, v) || (forbid_all && !ordered_key(key[v], order)))
            colour_mark(acc, base, ld_agent(color + w));
        return false;
    }
    ATOS_DEV uint32_t finish(uint32_t v, uint32_t, uint32_t& val, uint64_t* acc) const {
        const int32_t c = colour_first_free(acc, val);
        if (c < 0) {
            val += kColourWindow;
#pragma unroll
            for (int j = 0; j < kColourWords; ++j) acc[j] = 0;
            return kFinishRepeat;
        }
        st_agent(color + v, c);
        return kFinishNone;
    }
};

// Algorithm 5, second kernel: a vertex that shares its colour with a
// neighbour joins the next frontier when that neighbour outranks it; a
// collision with a lower-ranked neighbour sends the neighbour instead (it
// may have settled in an earlier round, since assignments ignore
// lower-ranked neighbours).  `queued` keeps each vertex in the next
// frontier once.  A class vertex coloured this round releases its
// lower-ranked class neighbours (wait, as in GcApp); a frontier vertex
// without a colour (a class vertex still waiting) checks nothing.
struct BspGcCheck {
    const int32_t* color;
    const uint32_t* key;
    uint32_t* queued;
    uint32_t* wait;
    uint32_t order;
    static constexpr int kAccWords = 1;
    static constexpr bool kHasFinish = true;
    ATOS_DEV bool prepare(uint32_t v, uint32_t, uint32_t& val, uint64_t*) const {
        if (color[v] < 0) return false;
        val = (uint32_t)color[v];
        return true;
    }
    ATOS_DEV bool edge(uint32_t v, uint32_t cv, uint32_t, uint32_t w, uint64_t* acc) const {
        if (w == v) return false;
        if (color[w] == (int32_t)cv) {
            if (outranks(key, w, v)) {
                atomicOr((unsigned long long*)acc, 1ull);
                return false;
            }
            return exch_agent(queued + w, 1u) == 0u;  // w recolours next round
        }
        if (ordered_key(key[v], order) && ordered_key(key[w], order) && !outranks(key, w, v))
            return add_agent(wait + w, ~0u) == 1u;  // w's last outranking neighbour: next round
        return false;
    }
    ATOS_DEV uint32_t finish(uint32_t v, uint32_t, uint32_t&, uint64_t* acc) const {
        return ((acc[0] & 1ull) && exch_agent(queued + v, 1u) == 0u) ? kFinishPush : kFinishNone;
    }
};

// Algorithm 3, second kernel: the next frontier is every vertex whose
// residue exceeds eps, in ID order within each wavefront.
__global__ void pr_filter_kernel(const double* residue, int64_t n, double eps, uint32_t* out,
                                 uint32_t* out_count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const int64_t v = base + threadIdx.x;
        const bool take = v < n && residue[v] > eps;
        const uint64_t m = ballot(take);
        if (m) {
            uint32_t wbase = 0;
            if (lane_id() == (uint32_t)__builtin_ctzll(m)) wbase = atomicAdd(out_count, (uint32_t)__popcll(m));
            wbase = __shfl(wbase, __builtin_ctzll(m), kWave);
            if (take) out[wbase + mbcnt(m)] = (uint32_t)v;
        }
    }
}

}  // namespace atos
