/*
 * CPU oracle for the three graph applications of the Atos paper
 * (arXiv 2112.00132, section 5 "Three Case Studies").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file: only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header or constant with the HIP
 * library; it is plain C, sequential unless a thread count is passed, and
 * computes in FP64 where floating point is involved.
 *
 * Graph convention: undirected graph in CSR form, offsets int64 [n+1],
 * cols int32 [offsets[n]], both directions of every edge present.
 *
 * What each routine computes and which passage of the paper it follows is
 * stated above the routine.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ BFS
 * Breadth-first search depths (section 5.1, Algorithm 1).  Algorithm 1 is
 * level-synchronous BFS, which the paper identifies with Dijkstra's
 * algorithm on unit weights: every vertex ends with its minimum hop count
 * from the source.  The speculative variant (Algorithm 2) converges to the
 * same values.  Written out as the textbook FIFO BFS.
 * Unreached vertices keep the initial value MAX_UINT32 (Algorithm 1's
 * initialisation), whose bit pattern is -1 as int32.
 * Returns the number of reached vertices, or -1 on a bad argument. */
int64_t oracle_bfs(int64_t n, const int64_t *offsets, const int32_t *cols,
                   int64_t source, int32_t *depth)
{
    if (n < 0 || source < 0 || source >= n) return -1;
    for (int64_t v = 0; v < n; ++v) depth[v] = -1;
    int32_t *fifo = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!fifo) return -1;
    int64_t head = 0, tail = 0;
    depth[source] = 0;
    fifo[tail++] = (int32_t)source;
    while (head < tail) {
        int32_t u = fifo[head++];
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
            int32_t w = cols[e];
            if (depth[w] == -1) {
                depth[w] = depth[u] + 1;
                fifo[tail++] = w;
            }
        }
    }
    free(fifo);
    return tail;
}

/* Level-synchronous BFS (section 5.1, Algorithm 1) over `threads` OpenMP
 * threads, for the CPU timing only: level by level, every vertex of the
 * current frontier claims each unvisited neighbour with a compare-and-swap
 * from -1 to level + 1, and a claimed neighbour is appended to the next
 * frontier.  The depths equal oracle_bfs's (a vertex is claimed at the first
 * level that reaches it).  Returns the number of reached vertices, or -1. */
int64_t oracle_bfs_levelsync(int64_t n, const int64_t *offsets, const int32_t *cols,
                             int64_t source, int threads, int32_t *depth)
{
    if (n < 0 || source < 0 || source >= n) return -1;
    int32_t *cur = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *next = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!cur || !next) { free(cur); free(next); return -1; }
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    for (int64_t v = 0; v < n; ++v) depth[v] = -1;
    depth[source] = 0;
    cur[0] = (int32_t)source;
    int64_t ncur = 1, reached = 1;
    int32_t level = 0;
    while (ncur > 0) {
        int64_t nnext = 0;
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < ncur; ++i) {
            int32_t u = cur[i];
            for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
                int32_t w = cols[e];
                int32_t expect = -1;
                if (__atomic_load_n(&depth[w], __ATOMIC_RELAXED) == -1 &&
                    __atomic_compare_exchange_n(&depth[w], &expect, level + 1, 0,
                                                __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
                    int64_t slot = __atomic_fetch_add(&nnext, 1, __ATOMIC_RELAXED);
                    next[slot] = w;
                }
            }
        }
        int32_t *t = cur;
        cur = next;
        next = t;
        ncur = nnext;
        reached += nnext;
        ++level;
    }
    free(cur);
    free(next);
    return reached;
}

/* ------------------------------------------------------------------ PageRank
 * PageRank on the undirected graph with damping lambda (section 5.2,
 * Algorithms 3-4).  The paper initialises every rank to 1 - lambda and
 * pushes lambda * residue / degree along each edge, i.e. it computes the
 * unnormalised fixed point
 *       x = (1 - lambda) * 1 + lambda * A * D^-1 * x
 * (A adjacency, D degrees); a vertex of degree 0 keeps x = 1 - lambda.
 * This routine is that definition solved by Jacobi iteration in FP64:
 *       x_{k+1}(v) = (1 - lambda) * t(v) + lambda * sum_{u in adj(v)} x_k(u) / deg(u)
 * where t = 1 for global PageRank, or t = e_source for personalized
 * PageRank (source >= 0).  Iteration starts from x_0 = t and stops when
 * max_v |x_{k+1}(v) - x_k(v)| < tol or after max_iter sweeps.  Each x_{k+1}(v)
 * is an independent sum in CSR order, so the thread count does not change
 * the result.
 * Outputs: x [n]; *out_delta = last max |x_{k+1} - x_k|;
 * *out_wdelta = last max_v |x_{k+1}(v) - x_k(v)| / max(deg(v), 1), from which
 * the caller can bound the error: |x_k(v) - x*(v)| <= deg(v) * lambda/(1-lambda)
 * * wdelta (the map contracts by lambda in the D^-1-weighted max norm).
 * Returns the number of sweeps, or -1 on a bad argument. */
static int pagerank_jacobi(int64_t n, const int64_t *offsets, const int32_t *cols,
                           double lambda, int64_t source, double tol, int max_iter,
                           int threads, double *x, double *out_delta, double *out_wdelta)
{
    if (n < 0 || !(lambda > 0.0 && lambda < 1.0) || source >= n) return -1;
    double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *inv_deg = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!y || !inv_deg) { free(y); free(inv_deg); return -1; }
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = offsets[v + 1] - offsets[v];
        inv_deg[v] = d > 0 ? 1.0 / (double)d : 0.0;
        x[v] = (source < 0) ? 1.0 : (v == source ? 1.0 : 0.0);
    }
    int it = 0;
    double delta = INFINITY, wdelta = INFINITY;
    while (it < max_iter) {
        double dmax = 0.0, wmax = 0.0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(max : dmax, wmax)
        for (int64_t v = 0; v < n; ++v) {
            double acc = 0.0;
            for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) acc += x[cols[e]] * inv_deg[cols[e]];
            double teleport = (source < 0) ? 1.0 : (v == source ? 1.0 : 0.0);
            double nv = (1.0 - lambda) * teleport + lambda * acc;
            double d = fabs(nv - x[v]);
            int64_t deg = offsets[v + 1] - offsets[v];
            double w = d / (double)(deg > 0 ? deg : 1);
            if (d > dmax) dmax = d;
            if (w > wmax) wmax = w;
            y[v] = nv;
        }
        memcpy(x, y, (size_t)n * sizeof(double));
        ++it;
        delta = dmax;
        wdelta = wmax;
        if (delta < tol) break;
    }
    if (out_delta) *out_delta = delta;
    if (out_wdelta) *out_wdelta = wdelta;
    free(y);
    free(inv_deg);
    return it;
}

int oracle_pagerank(int64_t n, const int64_t *offsets, const int32_t *cols, double lambda,
                    double tol, int max_iter, int threads, double *x, double *out_delta,
                    double *out_wdelta)
{
    return pagerank_jacobi(n, offsets, cols, lambda, -1, tol, max_iter, threads, x, out_delta,
                           out_wdelta);
}

int oracle_ppr(int64_t n, const int64_t *offsets, const int32_t *cols, int64_t source,
               double lambda, double tol, int max_iter, int threads, double *x,
               double *out_delta, double *out_wdelta)
{
    if (source < 0) return -1;
    return pagerank_jacobi(n, offsets, cols, lambda, source, tol, max_iter, threads, x,
                           out_delta, out_wdelta);
}

/* ------------------------------------------------------------------ push PageRank
 * The paper's bulk-synchronous push PageRank (Algorithm 3) run sequentially
 * in FP64, used for work counts and as the like-for-like CPU baseline.
 *   rank(v) = 1 - lambda, residue(v) = 0 for every v; then the initial
 *   residue is scattered along edges so that the pair (rank, residue)
 *   represents the fixed point above exactly (the printed initialisation
 *   line is garbled; this is the reading that keeps the invariant
 *   x = rank + (I - lambda A D^-1)^-1 residue): every vertex u adds
 *   (1 - lambda) * lambda / deg(u) to the residue of each neighbour.
 *   The first frontier is every vertex (Algorithm 3's initialisation).
 *   Each round: for each frontier vertex v in order, take res = residue(v)
 *   and zero it, add res to rank(v), and add lambda * res / deg(v) to the
 *   residue of each neighbour; then the next frontier is every vertex with
 *   residue > epsilon, in ID order.  Stops when the frontier is empty.
 * A degree-0 vertex never receives residue, so the division is never by 0.
 * Outputs rank and residue; *out_edge_pushes = number of neighbour updates;
 * *out_pops = frontier entries processed.  Returns rounds, -1 on bad args. */
int oracle_pagerank_push_bsp(int64_t n, const int64_t *offsets, const int32_t *cols,
                             double lambda, double epsilon, int max_rounds, double *rank,
                             double *residue, int64_t *out_edge_pushes, int64_t *out_pops)
{
    if (n < 0 || !(lambda > 0.0 && lambda < 1.0) || !(epsilon > 0.0)) return -1;
    int32_t *frontier = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!frontier) return -1;
    for (int64_t v = 0; v < n; ++v) { rank[v] = 1.0 - lambda; residue[v] = 0.0; }
    for (int64_t u = 0; u < n; ++u) {
        int64_t d = offsets[u + 1] - offsets[u];
        for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e)
            residue[cols[e]] += (1.0 - lambda) * lambda / (double)d;
    }
    int64_t fsize = 0;
    for (int64_t v = 0; v < n; ++v) frontier[fsize++] = (int32_t)v;
    int64_t pushes = 0, pops = 0;
    int rounds = 0;
    while (fsize > 0 && rounds < max_rounds) {
        for (int64_t i = 0; i < fsize; ++i) {
            int32_t v = frontier[i];
            double res = residue[v];
            residue[v] = 0.0;
            rank[v] += res;
            ++pops;
            int64_t d = offsets[v + 1] - offsets[v];
            if (d == 0) continue;
            double share = res * lambda / (double)d;
            for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) residue[cols[e]] += share;
            pushes += d;
        }
        fsize = 0;
        for (int64_t v = 0; v < n; ++v)
            if (residue[v] > epsilon) frontier[fsize++] = (int32_t)v;
        ++rounds;
    }
    free(frontier);
    if (out_edge_pushes) *out_edge_pushes = pushes;
    if (out_pops) *out_pops = pops;
    return rounds;
}

/* ------------------------------------------------------------------ colouring
 * Sequential greedy (first-fit) colouring in vertex-ID order: every vertex,
 * in increasing ID, takes the smallest colour not used by an already
 * coloured neighbour (section 5.3; Algorithms 5-6 are the speculative
 * parallel form of this greedy rule, whose sequential execution with
 * initial queue in ID order is exactly this loop).  Colours are 0-based.
 * Returns the number of colours used (max colour + 1), or -1 on bad args. */
int64_t oracle_greedy_color(int64_t n, const int64_t *offsets, const int32_t *cols,
                            int32_t *color)
{
    if (n < 0) return -1;
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = offsets[v + 1] - offsets[v];
        if (d > maxdeg) maxdeg = d;
    }
    /* mark[c] == v + 1 means colour c is used by a neighbour of v */
    int64_t *mark = (int64_t *)calloc((size_t)(maxdeg + 2), sizeof(int64_t));
    if (!mark) return -1;
    for (int64_t v = 0; v < n; ++v) color[v] = -1;
    int64_t ncolors = 0;
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
            int32_t c = color[cols[e]];
            if (c >= 0 && c <= maxdeg) mark[c] = v + 1;
        }
        int32_t c = 0;
        while (mark[c] == v + 1) ++c;
        color[v] = c;
        if (c + 1 > ncolors) ncolors = c + 1;
    }
    free(mark);
    return ncolors;
}

/* ------------------------------------------------------------------ speculative colouring
 * Rank of a vertex for the speculative colouring: a 32-bit key whose high
 * 16 bits are min(degree, 65535) and whose low 16 bits are the top half of
 * a 32-bit pseudo-random priority of (seed, id); ties on the key go to the
 * larger id.  The priority is MurmurHash3's 64-bit finaliser (fmix64)
 * applied to seed XOR (0x9E3779B97F4A7C15 * (id + 1)), low 32 bits. */
static uint32_t rank_priority(uint64_t seed, uint32_t id)
{
    uint64_t k = seed ^ (0x9E3779B97F4A7C15ull * ((uint64_t)id + 1ull));
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return (uint32_t)k;
}

void oracle_color_rank_keys(int64_t n, const int64_t *offsets, uint64_t seed, uint32_t *key)
{
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = offsets[v + 1] - offsets[v];
        uint32_t dk = d > 0xFFFF ? 0xFFFFu : (uint32_t)d;
        key[v] = (dk << 16) | (rank_priority(seed, (uint32_t)v) >> 16);
    }
}

static int outranks(const uint32_t *key, int64_t w, int64_t v)
{
    return key[w] != key[v] ? key[w] > key[v] : w > v;
}

/* Algorithm 6 (asynchronous speculative greedy colouring) executed by one
 * worker that takes one task at a time from a FIFO worklist: the worklist
 * starts with assign(v) for every vertex in ID order.
 *   assign(v): v is no longer queued; v takes the smallest colour not held by
 *     a neighbour that outranks it; check(v) is appended.
 *   check(v): for each neighbour w in CSR order holding v's colour: if w
 *     outranks v, v must recolour; otherwise w must recolour and assign(w) is
 *     appended unless w is already queued.  After the scan, assign(v) is
 *     appended if v must recolour and is not queued.
 * Ordered class (order_degree > 0): a vertex of degree >= order_degree is
 * not coloured speculatively.  Its outranking neighbours all have at least
 * its degree, so they are in the class too; it waits for all of them to hold
 * colours, and each is coloured exactly once:
 *   wait(v) = number of outranking neighbours (at the start);
 *   assign(v) of a class vertex is skipped (the task is still counted) while
 *     wait(v) > 0 or once v holds a colour;
 *   the check of a class vertex runs in its assign task, right after the
 *     colour is set, instead of as a task of its own;
 *   check(u) of a class vertex u also, for each lower-ranked class neighbour w
 *     in CSR order, decrements wait(w) and appends assign(w) when it reaches 0.
 * (The forbidden set restricted to outranking neighbours, the rule that the
 * lower-ranked endpoint recolours, and the ordered class are this project's
 * reading of the conflict step, see the colouring rank above.)
 * Status: this routine replays those readings with one FIFO worker; it is
 * not a result the paper defines (a speculative colouring is not unique).
 * Its pins are a hand-traced run with the ordered class off, closed forms
 * (K_n, star) and, with every vertex ordered, first-fit in rank order; the
 * concurrent colourings are checked only by validity, the rank bound and
 * the colour-count band.
 * Outputs colours and *out_tasks = tasks processed.  Returns the number of
 * colours, or -1 on bad arguments. */
int64_t oracle_color_fifo(int64_t n, const int64_t *offsets, const int32_t *cols, uint64_t seed,
                          int64_t order_degree, int32_t *color, int64_t *out_tasks)
{
    if (n < 0 || order_degree < 0 || order_degree > 0xFFFF) return -1;
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v)
        if (offsets[v + 1] - offsets[v] > maxdeg) maxdeg = offsets[v + 1] - offsets[v];
    uint32_t *key = (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
    int64_t *wait = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    unsigned char *queued = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
    int64_t *mark = (int64_t *)calloc((size_t)(maxdeg + 2), sizeof(int64_t));
    /* at most: n initial assigns, one wake-up assign and one check per vertex */
    int64_t cap = 3 * (n > 0 ? n : 1) + 2;
    int64_t *fifo = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    if (!key || !wait || !queued || !mark || !fifo) {
        free(key); free(wait); free(queued); free(mark); free(fifo);
        return -1;
    }
    oracle_color_rank_keys(n, offsets, seed, key);
#define ORDERED(v) (order_degree > 0 && (int64_t)(key[v] >> 16) >= order_degree)
    for (int64_t v = 0; v < n; ++v) {
        if (!ORDERED(v)) continue;
        for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e)
            if (cols[e] != v && outranks(key, cols[e], v)) ++wait[v];
    }
    int64_t head = 0, count = 0, tasks = 0, stamp = 0;
#define PUSH(task) do { fifo[(head + count) % cap] = (task); ++count; } while (0)
    for (int64_t v = 0; v < n; ++v) {
        color[v] = -1;
        queued[v] = 1;
        PUSH(2 * v);  /* even = assign, odd = check */
    }
    while (count > 0) {
        int64_t t = fifo[head];
        head = (head + 1) % cap;
        --count;
        ++tasks;
        int64_t v = t / 2;
        if ((t & 1) == 0) {
            if (ORDERED(v) && (wait[v] > 0 || color[v] >= 0)) continue;
            queued[v] = 0;
            ++stamp;
            for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
                int64_t w = cols[e];
                if (w == v || color[w] < 0 || !outranks(key, w, v)) continue;
                if (color[w] <= maxdeg) mark[color[w]] = stamp;
            }
            int32_t c = 0;
            while (mark[c] == stamp) ++c;
            color[v] = c;
            if (!ORDERED(v)) {
                PUSH(2 * v + 1);
                continue;
            }
            /* a class vertex's check follows in the same task */
        }
        {
            int lost = 0;
            for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) {
                int64_t w = cols[e];
                if (w == v) continue;
                if (color[w] == color[v]) {
                    if (outranks(key, w, v)) {
                        lost = 1;
                    } else if (!queued[w]) {
                        queued[w] = 1;
                        PUSH(2 * w);
                    }
                } else if (ORDERED(v) && ORDERED(w) && !outranks(key, w, v)) {
                    if (--wait[w] == 0) PUSH(2 * w);
                }
            }
            if (lost && !queued[v]) {
                queued[v] = 1;
                PUSH(2 * v);
            }
        }
    }
#undef ORDERED
#undef PUSH
    int64_t ncolors = 0;
    for (int64_t v = 0; v < n; ++v)
        if (color[v] + 1 > ncolors) ncolors = color[v] + 1;
    free(key); free(wait); free(queued); free(mark); free(fifo);
    if (out_tasks) *out_tasks = tasks;
    return ncolors;
}
