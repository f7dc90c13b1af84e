/*
 * atos.h -- C ABI of libatos, a persistent-worklist graph engine for AMD
 * Instinct MI355X (gfx950), after "Atos: A Task-Parallel GPU Dynamic
 * Scheduling Framework for Dynamic Irregular Computations" (Chen et al.,
 * PPoPP'22, arXiv 2112.00132).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers named d_* are device pointers on the current HIP device; all of
 *    them are owned by the caller and must stay valid until the work queued
 *    on `stream` has finished.  The library never allocates device memory on
 *    the query path: scratch state lives in a caller-provided workspace
 *    (d_ws, ws_bytes) sized by atos_workspace_bytes().
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call is stream-ordered.  With st == NULL a call only enqueues work
 *    and returns; with st != NULL it also waits for that work and fills *st
 *    (status of the device run, counters, device time).
 *  - Argument errors are reported synchronously by the return value and
 *    nothing is enqueued.  Outcomes only known on the device (worklist
 *    overflow, deadline expiry) are reported in st->status, or later by
 *    atos_workspace_stats() on the same workspace.
 *  - A workspace may be reused by any number of calls of the application it
 *    was sized for, on one stream at a time.  Calls on different streams
 *    need different workspaces.  A graph handle is immutable after load and
 *    may be shared by concurrent calls.
 *  - No C++ exception crosses this interface.
 *
 * Graph: an undirected graph in CSR form -- offsets[n+1] (int32 or int64),
 * cols[m] (int32), both directions of every edge stored, no self-loops
 * needed for correctness (a self-loop is harmless for BFS and colouring
 * skips it; PageRank treats it as an ordinary edge).
 */
#ifndef ATOS_H
#define ATOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ATOS_OK = 0,
    ATOS_EINVAL = 1,         /* bad argument; nothing was enqueued */
    ATOS_ENOMEM = 2,         /* workspace smaller than atos_workspace_bytes() */
    ATOS_EOVERFLOW = 3,      /* device worklist ring overflowed; rerun with a larger
                                queue_capacity (results are incomplete) */
    ATOS_ETIMEOUT = 4,       /* the run passed its deadline and stopped (results incomplete) */
    ATOS_EABORTED = 5,       /* the run was stopped from the host (atos_config.abort_flag) */
    ATOS_EHIP = 6,           /* a HIP runtime call failed, or the worklist held a word this
                                library did not write (workspace memory reused elsewhere) */
    ATOS_ENOTSYMMETRIC = 7,  /* PageRank/colouring need a graph loaded with ATOS_GRAPH_SYMMETRIC */
    ATOS_EUNSUPPORTED = 8,   /* configuration the library does not implement */
    ATOS_EAGAIN = 9          /* serving: no free query slot, state memory or worklist
                                capacity right now; submit again after a release */
} atos_status;

typedef struct atos_graph *atos_graph_t;

/* atos_graph_load() flags */
#define ATOS_GRAPH_SYMMETRIC 1u /* caller asserts every edge u->v has its v->u */
#define ATOS_GRAPH_VALIDATE 2u  /* check offsets/cols (and symmetry when SYMMETRIC) on the device */

/* applications (atos_workspace_bytes) */
#define ATOS_APP_BFS 1
#define ATOS_APP_PAGERANK 2
#define ATOS_APP_COLOR 3

/* atos_config.strategy -- kernel strategy (paper section 3.4) */
#define ATOS_PERSISTENT 0 /* one persistent kernel, workers loop on the worklist */
#define ATOS_BSP 1        /* level-synchronous frontier kernels, one host round per level
                             (the bulk-synchronous baselines, Algorithms 1, 3 and 5) */
#define ATOS_DISCRETE 2   /* the persistent kernel's workers and worklist, one launch per
                             round: a round takes the tasks published before it started and
                             pushes the next round's; the host reads the worklist counters
                             after each round (stats.rounds counts them) and stops when every
                             task is done.  Not for batches or the server (EUNSUPPORTED). */
#define ATOS_ROUNDS 3     /* the discrete strategy's rounds inside one persistent launch: a
                             worker takes only tasks published before the current round
                             began, and once every task of the round has been taken the
                             workers advance it to all tasks published by then, so no
                             launch, host round trip or drain separates the rounds (the
                             old round's last batches push into the round after the next);
                             stats.rounds counts the rounds.  Not for batches or the
                             server (EUNSUPPORTED). */

/* atos_config.queue_layout */
#define ATOS_QUEUE_AUTO 0
#define ATOS_QUEUE_GLOBAL 1  /* one shared ring (the paper's single shared task queue) */
#define ATOS_QUEUE_PER_XCD 2 /* one ring per XCD; workers push locally and steal when
                                their ring is empty (default) */
#define ATOS_QUEUE_SEGMENTED 3 /* batches only: one ring per XCD, and the union graph's
                                vertices cut into 8 segments of whole instances (about
                                n/8 vertices each); every task goes to the ring of its
                                vertex's segment, so an instance's tasks stay in one FIFO
                                order; workers take from their own XCD's ring first and
                                steal as with PER_XCD.  EUNSUPPORTED for single runs. */

/*
 * Launch configuration (paper section 4, the launch arguments of the Queues
 * API: persistent or not, numBlock, numThread and FETCH_SIZE).  Zero in any
 * field selects the library default.
 */
typedef struct {
    int32_t strategy;       /* ATOS_PERSISTENT (default), ATOS_DISCRETE, ATOS_ROUNDS or ATOS_BSP */
    int32_t worker;         /* threads per worker: 64 = one wavefront worker,
                               128/256/512/1024 = one workgroup worker (paper section 3.2);
                               default 1024 (colouring on a graph whose largest
                               degree exceeds 32 times its average: 512) */
    int32_t fetch;          /* tasks claimed per pop, 1..256 and <= worker (FETCH_SIZE);
                               default min(worker, 256) */
    int32_t queue_layout;   /* ATOS_QUEUE_* */
    int32_t grid;           /* workgroups launched; 0 = as many as can be co-resident
                               (the paper's default, section 4), except colouring with
                               512- or 1024-thread workers: one per CU */
    int32_t pr_check_size;  /* PageRank enqueue rule: 0 = enqueue a vertex when its residue
                               crosses epsilon; 1..65536 = Algorithm 4's rule (Check_Size):
                               edge updates enqueue nothing, and after every task its
                               worker sweeps this many positions of a round-robin cursor
                               over all vertices and enqueues those with residue >
                               epsilon; when a launch's worklist drains, a clean sweep of
                               every vertex seeds the next launch with what it finds, and
                               the run ends when it finds nothing (stats.rounds =
                               launches).  Whole-graph ATOS_PERSISTENT PageRank only
                               (EUNSUPPORTED for personalized PageRank, other strategies
                               and batches) */
    int64_t queue_capacity; /* entries per ring (rounded up to a power of two); 0 = default */
    uint32_t timeout_ms;    /* device deadline per call; 0 = 60000 ms */
    int32_t split_degree;   /* persistent runs: a task with more neighbours than this is
                               posted to the hub board and its neighbour list is processed
                               in chunks by all workers (colouring: the chunk that completes
                               a pass runs its finish step on the OR of the chunks'
                               colour masks); 0 = default (BFS: max(8 * worker, 4096);
                               PageRank: max(2 * worker, 2048); colouring: max(4 * worker,
                               1024)), -1 = never split */
    int32_t color_order_degree; /* colouring: vertices with at least this many neighbours
                               (<= 65535) are coloured in rank order instead of
                               speculatively (see atos_color); 0 = default (8; none with
                               color_forbid_all), -1 = every vertex speculative, -2 = about
                               sqrt(n) of the highest-degree vertices (those of degree >= 64
                               from the lowest degree class where at most ceil(sqrt(n))
                               remain; none when no vertex has degree 64) */
    int32_t fetch_policy;   /* ATOS_FETCH_FIXED: a pop takes up to `fetch` tasks (the
                               paper's rule); ATOS_FETCH_ADAPTIVE: only its share of what
                               the ring holds, ceil(queued / workers per ring), at most
                               `fetch`, so a shallow worklist of heavy tasks is spread over
                               many workers; ATOS_FETCH_AUTO (0): adaptive for colouring,
                               fixed for BFS and PageRank */
    int32_t push_policy;    /* ATOS_PUSH_OWN: a worker publishes into its own XCD's ring;
                               ATOS_PUSH_SHALLOWEST: into the ring that held the fewest
                               tasks at its last probe, which keeps the rings equally deep
                               (and so one FIFO order across them); ATOS_PUSH_AUTO (0):
                               shallowest for colouring and for persistent PageRank over
                               the whole graph (batches included), own for BFS, for
                               personalized PageRank and for PageRank as discrete
                               launches or rounds */
    uint32_t discrete_tail; /* ATOS_DISCRETE: once a round leaves at most this many tasks
                               queued, the rest of the run is one persistent launch of the
                               same workers, so the many short rounds at the end cost no
                               launch and host round trip each (stats.rounds counts that
                               launch as one round); 0 = never (every round discrete) */
    int32_t color_forbid_all; /* colouring: 0 = an assignment avoids the colours of the
                               neighbours that outrank the vertex (default); 1 = it avoids
                               the colour of every neighbour, as Algorithms 5 and 6 print
                               it (the lower-ranked endpoint of a conflict still
                               recolours, so runs terminate); no ordered class unless
                               color_order_degree is given */
    int32_t pr_combine;     /* whole-graph PageRank (threshold-crossing rule, not ATOS_BSP):
                               the residue updates of the (at most 12288) highest-degree
                               vertices of degree >= 64 are summed in a per-worker table
                               in LDS and applied with one device atomic per vertex and
                               flush, the crossing test taken on the sum; a worker flushes
                               after every N edges and whenever it finds no task.  N > 0
                               = on with that window; -1 = off (every update is one
                               device atomic); 0 = default: on with N = 131072 (batches:
                               32768) for 1024-thread workers, off for smaller ones (the table takes
                               the LDS of further co-resident workgroups).  The set-up
                               (degree classes, slots, a tagged copy of the column array
                               in the workspace) runs on every call.  Batches combine
                               their PageRank instances' vertices the same way (BFS
                               instances are untouched), and so does Algorithm 4's rule
                               (pr_check_size > 0: a flush only adds the sums, the
                               sweeps enqueue).  N > 0 gives EUNSUPPORTED for ATOS_BSP
                               and atos_ppr */
    const uint32_t *abort_flag; /* NULL, or a word in pinned host memory (hipHostMalloc,
                               atos_host_alloc) that the host may set non-zero while the
                               run is on the GPU: the workers poll it (every 32 loop
                               iterations of a worker) and stop, the level-synchronous
                               loop reads it before every level, and the run ends with
                               status ATOS_EABORTED (results incomplete; the workspace
                               stays valid for the next call).  The flag must stay
                               allocated until the call's work has finished. */
} atos_config;

#define ATOS_PUSH_AUTO 0
#define ATOS_PUSH_OWN 1
#define ATOS_PUSH_SHALLOWEST 2
#define ATOS_PUSH_QUERY 3 /* server only: every task into the ring of its query's slot */

#define ATOS_FETCH_AUTO 0
#define ATOS_FETCH_FIXED 1
#define ATOS_FETCH_ADAPTIVE 2

/* Per-call outcome and counters. */
typedef struct {
    int32_t status;         /* atos_status of the device run */
    int32_t reserved0;
    uint64_t tasks_popped;  /* tasks taken from the worklist (BSP: frontier entries) */
    uint64_t tasks_pushed;  /* tasks appended to the worklist (BSP: frontier appends) */
    uint64_t edges_scanned; /* neighbour-list entries visited by the workers */
    uint64_t rounds;        /* BSP levels/rounds; discrete: launches; ATOS_ROUNDS: rounds
                               inside the launch; 1 for a persistent run */
    float device_ms;        /* wall time of all the work the call enqueued, from HIP events */
    float kernel_ms;        /* persistent: the worker kernel alone; discrete: its rounds with
                               the host reads between them; BSP: same as device_ms */
    uint64_t push_retries;  /* pushes that found their slot still held by the previous lap */
    uint64_t idle_iterations; /* worker loop iterations that found no task */
    uint64_t steals;        /* task windows a worker claimed from another XCD's ring */
    uint64_t hub_posts;     /* high-degree tasks split into chunks over all workers */
    uint64_t combined_updates; /* PageRank with pr_combine: edge updates summed in LDS tables
                               (the rest of edges_scanned were device atomics) */
    uint64_t combine_atomics;  /* PageRank with pr_combine: device atomics that applied them */
} atos_stats;

/*
 * Load a CSR graph (the graph of paper section 5, where a vertex's neighbour
 * list vertex.neighbors and its length neighborLen are what every callback
 * reads; here they are cols[offsets[v] .. offsets[v+1])).  The handle borrows
 * d_offsets and d_cols (they must outlive it) and keeps only host metadata:
 * n, m, the offset width, the
 * maximum degree (computed on the device during the call) and launch
 * occupancy.  Synchronizes `stream` before returning.
 *   d_offsets: n_vertices+1 entries, int64 if offsets_are_int64 else int32,
 *              non-decreasing, offsets[0] = 0, offsets[n] = n_edges.
 *   d_cols:    n_edges int32 vertex ids in [0, n_vertices).
 *   n_vertices < 2^31 - 1.  n_edges < 2^31 unless offsets are int64.
 * Errors: EINVAL for null/negative/oversized arguments, or (with
 * ATOS_GRAPH_VALIDATE) malformed CSR; ENOTSYMMETRIC when VALIDATE finds an
 * edge without its reverse; EHIP on runtime failure.
 */
atos_status atos_graph_load(const void *d_offsets, int32_t offsets_are_int64,
                            const int32_t *d_cols, int64_t n_vertices, int64_t n_edges,
                            uint32_t flags, void *stream, atos_graph_t *out);
atos_status atos_graph_free(atos_graph_t g);
atos_status atos_graph_info(atos_graph_t g, int64_t *n_vertices, int64_t *n_edges,
                            int64_t *max_degree);

/*
 * Bytes of workspace that application `app` (ATOS_APP_*) needs on graph g
 * under configuration cfg (NULL = defaults).  The workspace must be 256-byte
 * aligned.  Before its first use, and whenever its memory has been used for
 * anything else since, the caller zeroes its first ATOS_WORKSPACE_HEADER_BYTES
 * bytes (e.g. hipMemsetAsync); the library prepares everything else itself
 * and keeps the worklist ring consistent from one call to the next.
 */
#define ATOS_WORKSPACE_HEADER_BYTES 4096
atos_status atos_workspace_bytes(atos_graph_t g, int32_t app, const atos_config *cfg,
                                 size_t *bytes);

/*
 * Counters and status of the last run recorded in a workspace.  Synchronizes
 * `stream`.
 */
atos_status atos_workspace_stats(const void *d_ws, void *stream, atos_stats *st);

/*
 * Breadth-first search (paper section 5.1).  d_depth[v] receives the hop
 * distance from `source` (int32; -1, the bit pattern of the paper's
 * MAX_UINT32, for unreached vertices).
 *   ATOS_PERSISTENT runs the speculative BFS of Algorithm 2: workers pop a
 *   vertex, lower each neighbour's depth with an atomic minimum and push the
 *   neighbours they improved.  ATOS_BSP runs Algorithm 1 (one frontier
 *   expansion per level, host synchronisation between levels).  Both end
 *   with the exact hop distances.
 * Errors: EINVAL (null pointers, source outside [0, n)), ENOMEM.
 */
atos_status atos_bfs(atos_graph_t g, int64_t source, int32_t *d_depth, void *d_ws,
                     size_t ws_bytes, const atos_config *cfg, void *stream, atos_stats *st);

/*
 * atos_bfs without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  The workspace is a fixed library-owned device
 * array of ATOS_NOALLOC_SCRATCH_BYTES, one per GPU, taken the first time the
 * call runs on that GPU and held until the process ends; the call allocates
 * nothing (no hipMalloc/hipFree, no event).  Same graph, source, depth,
 * configuration and errors as atos_bfs, plus:
 *   ENOMEM  when atos_workspace_bytes(g, ATOS_APP_BFS, cfg) exceeds
 *           ATOS_NOALLOC_SCRATCH_BYTES (with the default configuration this
 *           admits graphs of up to 2^21 vertices); nothing is enqueued.
 *   st      when given, waits for the run and carries its status and
 *           counters; device_ms and kernel_ms are 0 (no timing events).
 * Every call on one GPU shares that GPU's array and leaves its worklist in
 * the state the next call expects; calls that overlap on one GPU (different
 * streams or host threads without ordering between them) race and must not
 * be issued.  The graph must live on the current device (EINVAL otherwise).
 */
#define ATOS_NOALLOC_SCRATCH_BYTES ((size_t)64 * 1024 * 1024 + (size_t)64 * 1024)
atos_status atos_bfs_noalloc(atos_graph_t g, int64_t source, int32_t *d_depth,
                             const atos_config *cfg, void *stream, atos_stats *st);

/*
 * PageRank by residual pushing (paper section 5.2).  Computes ranks p that
 * approximate the unnormalised fixed point x = (1-d) + d * A * D^-1 * x
 * (damping d): every vertex starts with rank 1-d and the residue that makes
 * (rank, residue) represent x exactly; a worker that takes vertex v moves
 * its residue r into its rank and adds d*r/deg(v) to each neighbour's
 * residue.  The run ends when no residue exceeds epsilon, which bounds the
 * error per vertex by 0 <= x(v) - p(v) <= deg(v)*epsilon/(1-d) (plus FP32
 * rounding of the output).  Ranks and residues are held in FP64 in the
 * workspace (a hub collects many tiny residue increments, which FP32 would
 * round away) and rounded to FP32 once at the end.
 *   ATOS_PERSISTENT = asynchronous PageRank (Algorithm 4); ATOS_BSP =
 *   Algorithm 3 (push round, then a filter round that rebuilds the
 *   frontier from residue > epsilon).
 *   With residue combining (atos_config.pr_combine, on by default for
 *   1024-thread workers) the updates to the highest-degree vertices are
 *   summed per worker before they reach the device residue; the sums and
 *   the bound are the same, only the order of the FP64 additions differs.
 *   d_rank[n] (FP32) receives p; d_residual[n] (FP32, may be NULL) receives
 *   the final residues, rounded to FP32.
 * Errors: EINVAL (null d_rank, damping outside (0,1), epsilon <= 0),
 * ENOTSYMMETRIC, ENOMEM.
 */
atos_status atos_pagerank(atos_graph_t g, float damping, float epsilon, float *d_rank,
                          float *d_residual, void *d_ws, size_t ws_bytes, const atos_config *cfg,
                          void *stream, atos_stats *st);

/*
 * Personalized PageRank from one source vertex, by the same residual pushing:
 * approximates x = (1-d) e_source + d * A * D^-1 * x, starting from rank 0
 * everywhere and residue 1-d at the source (one initial task).  Same bound,
 * arguments, workspace (ATOS_APP_PAGERANK) and errors as atos_pagerank, plus
 * EINVAL for a source outside [0, n).
 */
atos_status atos_ppr(atos_graph_t g, int64_t source, float damping, float epsilon, float *d_rank,
                     float *d_residual, void *d_ws, size_t ws_bytes, const atos_config *cfg,
                     void *stream, atos_stats *st);

/*
 * Speculative greedy colouring (paper section 5.3, the Gebremedhin-Manne
 * scheme).  Every vertex takes the smallest colour not held by a neighbour,
 * reading neighbour colours that may be out of date; a conflict check after
 * each assignment sends one endpoint of every monochromatic edge back for
 * recolouring.  Vertices are ranked by (degree, priority, id), priority
 * being a 32-bit hash of (priority_seed, id): a vertex avoids the colours of
 * the neighbours that outrank it, and of two colliding neighbours the
 * lower-ranked one recolours.  The top vertex of any conflict keeps its
 * colour, so the run terminates.  Vertices with at least
 * cfg->color_order_degree neighbours (the densely connected high-degree
 * vertices, where speculation would cascade) are not coloured
 * speculatively: each waits until all its outranking neighbours (which have
 * at least its degree) hold colours, then takes its colour once; they end
 * up exactly first-fit in rank order among themselves.  The result is a
 * proper colouring, every colour at most the vertex's number of outranking
 * neighbours; it is not unique (with color_order_degree = 1 it is:
 * first-fit in rank order).  With cfg->color_forbid_all = 1 an assignment
 * avoids the colour of every neighbour, as the paper's Algorithms 5 and 6
 * print it, with no ordered class unless color_order_degree gives one (its
 * vertices, coloured once in rank order, still avoid only their outranking
 * neighbours' colours; with -2 the class is the ~sqrt(n) highest-degree
 * vertices: on R-MAT graphs of scale 16 to
 * 23 0.84-0.94 times the colours of sequential first-fit, 1.5 times as fast
 * as the default rule); the result is then a proper colouring with every
 * colour at most the vertex's degree.
 *   ATOS_PERSISTENT = Algorithm 6 (one kernel, assignment and check tasks on
 *   one worklist); ATOS_BSP = Algorithm 5 (assign kernel, then conflict
 *   kernel, per round).
 *   d_color[n] (int32) receives colours; d_n_colors (device int32, may be
 *   NULL) receives max colour + 1.
 * Errors: EINVAL, ENOTSYMMETRIC, ENOMEM.
 */
atos_status atos_color(atos_graph_t g, uint64_t priority_seed, int32_t *d_color,
                       int32_t *d_n_colors, void *d_ws, size_t ws_bytes, const atos_config *cfg,
                       void *stream, atos_stats *st);

/* ------------------------------------------------------------------ batching
 * Many BFS and PageRank instances in one persistent launch.  The instances'
 * graphs are concatenated into one union graph (load it with int64 offsets;
 * column ids are global), and instance i owns the vertex range
 * [vertex_begin, vertex_end): its edges must stay inside that range.  One
 * worklist serves all instances; a task's application travels in its task
 * word, so no instance lookup happens on the hot path.  Every PageRank
 * instance of a batch shares one damping and epsilon.
 */
typedef struct {
    int32_t app;          /* ATOS_APP_BFS or ATOS_APP_PAGERANK */
    int32_t reserved;     /* must be zero */
    int64_t vertex_begin; /* first vertex of the instance in the union graph */
    int64_t vertex_end;   /* one past its last vertex */
    int64_t source;       /* BFS: source vertex (global id, inside the range); else ignored */
} atos_batch_instance;

typedef struct atos_batch *atos_batch_t;
typedef struct atos_exec *atos_exec_t;

/*
 * Validate and plan a batch.  `instances` (host array, sorted by
 * vertex_begin, non-overlapping) is copied.  The plan owns a small device
 * table (allocated here, freed by atos_batch_free) and borrows the graph.
 * Synchronizes `stream`.
 * Errors: EINVAL (bad ranges or sources, an edge leaving its instance,
 * damping/epsilon out of range when PageRank instances exist),
 * ENOTSYMMETRIC (PageRank on a graph not loaded as symmetric),
 * EUNSUPPORTED (strategy other than ATOS_PERSISTENT), EHIP.
 */
atos_status atos_batch_plan(atos_graph_t g, const atos_batch_instance *instances,
                            int32_t n_instances, float damping, float epsilon,
                            const atos_config *cfg, void *stream, atos_batch_t *out);
atos_status atos_batch_free(atos_batch_t b);
/* Workspace bytes of a planned batch.  With PageRank instances it includes
 * the residue-combining arrays (a tag per vertex and a copy of the column
 * array, 4 bytes each), whatever the configuration, so that
 * atos_batch_set_config may turn combining on or off. */
atos_status atos_batch_workspace_bytes(atos_batch_t b, size_t *bytes);

/*
 * Run a planned batch.  d_state[n] (n = union vertices) receives, for the
 * vertices of BFS instances, the hop depth as uint32 (0xFFFFFFFF =
 * unreached) and, for vertices of PageRank instances, the FP32 rank bits;
 * other vertices are left untouched.  d_residual[n] (FP32, may be NULL)
 * receives PageRank residues.  Same workspace rules as single runs.
 */
atos_status atos_batch_run(atos_batch_t b, uint32_t *d_state, float *d_residual, void *d_ws,
                           size_t ws_bytes, void *stream, atos_stats *st);

/*
 * Capture one atos_batch_run (without stats) into an instantiated hipGraph.
 * `stream` must be a non-null stream; the graph replays on any stream with
 * atos_exec_launch, reusing the same output and workspace buffers.  The
 * captured work contains kernels only (no memset or copy nodes).
 */
atos_status atos_batch_capture(atos_batch_t b, uint32_t *d_state, float *d_residual, void *d_ws,
                               size_t ws_bytes, void *stream, atos_exec_t *out);
atos_status atos_exec_launch(atos_exec_t e, void *stream);
atos_status atos_exec_free(atos_exec_t e);

/* ------------------------------------------------------------------ autotuning
 * The best launch shape and kernel strategy depend on the application and
 * the input (paper section 6.6: worker size vs FETCH_SIZE, where only
 * FETCH_SIZE <= worker size is meaningful, and persistent vs discrete
 * kernels).  The tuner first times every persistent configuration of worker
 * size in {64, 128, 256, 512, 1024} x fetch in {1, 2, 4, ..., min(worker,
 * 256)} x queue layout in {PER_XCD, GLOBAL} (84 points); then, at the
 * winner's worker size, fetch and layout, the strategies ATOS_PERSISTENT,
 * ATOS_DISCRETE and ATOS_ROUNDS each with ATOS_PUSH_OWN and
 * ATOS_PUSH_SHALLOWEST (6 points; a batch runs persistent only, 2 points).
 * Each point runs `reps` times after one warm-up run; the one with the
 * lowest median device time wins.  Fields of `base` other than
 * strategy/worker/fetch/queue_layout/push_policy (capacity, timeout, grid,
 * split degree, ...) are kept.
 */
typedef struct {
    atos_config cfg;
    float median_ms;   /* -1 when the configuration failed */
    int32_t status;    /* atos_status of the failing run, or ATOS_OK */
    int32_t reserved;
} atos_tune_result;

/*
 * Tune one application on graph g.  The arguments of the runs are those of
 * atos_bfs (source, d_out = int32 depths), atos_pagerank (damping, epsilon,
 * d_out = FP32 ranks, d_residual may be NULL) or atos_color (seed, d_out =
 * int32 colours).  The workspace must be sized with atos_workspace_bytes for
 * `base` (the size does not depend on worker or fetch).  results[] (host,
 * may be NULL when max_results is 0) receives up to max_results timed
 * points; *best the winner.  Synchronous.  Errors: EINVAL; EUNSUPPORTED when
 * no configuration ran.
 */
atos_status atos_autotune(atos_graph_t g, int32_t app, int64_t source, float damping,
                          float epsilon, uint64_t seed, void *d_out, float *d_residual,
                          void *d_ws, size_t ws_bytes, const atos_config *base, int32_t reps,
                          void *stream, atos_tune_result *results, int32_t max_results,
                          int32_t *n_results, atos_config *best);

/* Once a point has run, every later point's runs are cut at five times the
 * best median so far (at least 1 s, at most its own timeout_ms): a point that
 * slow cannot win, and it is recorded with status ETIMEOUT.
 *
 * Progress: with a callback set, the tuner calls fn(points done, points
 * planned so far, that point's result, user) after every point, on the
 * calling thread.  The callback is process-wide (the last one set wins;
 * fn = NULL removes it). */
typedef void (*atos_tune_progress_fn)(int32_t done, int32_t planned, const atos_tune_result *point,
                                      void *user);
atos_status atos_tune_set_progress(atos_tune_progress_fn fn, void *user);

/* Change the worker size / fetch / layout of a planned batch (the ring
 * capacity chosen at plan time is kept). */
atos_status atos_batch_set_config(atos_batch_t b, const atos_config *cfg);

/* Tune a planned batch the same way; the batch keeps its configuration. */
atos_status atos_batch_autotune(atos_batch_t b, uint32_t *d_state, float *d_residual, void *d_ws,
                                size_t ws_bytes, int32_t reps, void *stream,
                                atos_tune_result *results, int32_t max_results,
                                int32_t *n_results, atos_config *best);

/* ------------------------------------------------------------------ microbenchmarks
 * Measured ceilings for the primitives the kernels use.  d_buf is caller
 * device memory of `bytes` (>= 4096) bytes whose contents are overwritten;
 * the kernel runs with `grid` x `block` threads (block a multiple of 64, at
 * most 1024) on `stream`, and *ms receives its duration from HIP events.
 *   COPY               bytes/2 read + bytes/2 written (16-byte words)
 *   ATOMIC_ADD_F32     `iters` agent-scope FP32 adds at pseudo-random
 *                      addresses of a bytes/4-entry array
 *   ATOMIC_MIN_U32     `iters` agent-scope u32 minimums, same pattern
 *   SAME_ADDRESS       every wavefront adds to one 64-bit counter `iters` times
 *   FENCES             every thread stores, then release + acquire agent fences,
 *                      `iters` times (needs grid*block + 64 <= bytes/4)
 *   GATHER_PLAIN       `iters` pseudo-random 4-byte loads (plain)
 *   GATHER_COHERENT    `iters` pseudo-random 4-byte agent-scope atomic loads
 *   LITMUS_MP          message passing between grid/2 writer/reader pairs on
 *                      different XCDs for `iters` rounds with agent-scope loads and
 *                      stores only; words [0] stale reads, [1] bounded-spin
 *                      give-ups, [2] rounds completed are left in d_buf
 */
#define ATOS_MB_COPY 0
#define ATOS_MB_ATOMIC_ADD_F32 1
#define ATOS_MB_ATOMIC_MIN_U32 2
#define ATOS_MB_SAME_ADDRESS 3
#define ATOS_MB_FENCES 4
#define ATOS_MB_GATHER_PLAIN 5
#define ATOS_MB_GATHER_COHERENT 6
#define ATOS_MB_LITMUS_MP 7
#define ATOS_MB_ATOMIC_ADD_F64 8 /* random agent-scope FP64 adds returning the old value */
#define ATOS_MB_ATOMIC_ADD_F64_NORET 10 /* the same adds, old value unused (no-return form) */
#define ATOS_MB_ATOMIC_ADD_F64_XCD 11 /* FP64 adds returning the old value, workgroup scope, each
                                         XCD into its own eighth of the array (L2-local) */
#define ATOS_MB_CLOCK 9 /* one thread spins until the device clock advanced `iters` ticks;
                           words [0..2] of d_buf: start, end readings, reads (uint64) */
atos_status atos_microbench(int32_t kind, void *d_buf, size_t bytes, int64_t iters, int32_t grid,
                            int32_t block, void *stream, float *ms);

/*
 * ---------------------------------------------------------------- tracing
 * Per-batch event trace of the persistent worker kernel, for profiling the
 * schedule (when each worker took which batch, for how long).  While a
 * buffer is attached, every persistent launch made afterwards on the
 * buffer's device (BFS, PageRank, personalized PageRank, colouring, batched
 * runs, and graphs captured while attached) appends one record per batch a
 * worker processes; records beyond the buffer's capacity are counted but
 * not stored.  A level-synchronous run (ATOS_BSP) made while attached
 * appends one record as each level starts and one after its last level:
 * worker = level number, tasks = frontier size | ATOS_TRACE_BSP_LEVEL, edges =
 * edges scanned by the run's earlier levels (low 32 bits), t_begin = device
 * clock, t_end = 0, vertex = 0xFFFFFFFF; a level lasts from its record to the
 * next (each record costs one one-thread launch, so a traced BSP run is a few
 * microseconds per level slower than an untraced one).  The serving daemon
 * does not record.
 *
 * Buffer layout (device memory, >= 256-byte aligned, owned by the caller):
 *   uint64 count         records appended since attach (may exceed capacity)
 *   uint64 capacity      (bytes - 64) / 32, written by atos_trace_attach
 *   uint64 clock_khz     rate of the records' clock, written by atos_trace_attach
 *   40 bytes             reserved
 *   atos_trace_record[capacity]
 * Attaching zeroes the count (a synchronous copy: call it while no Atos
 * kernel runs).  Tracing adds one device atomic per batch.  Attaching a new
 * buffer replaces the old one; d_buf = NULL detaches.  EINVAL: bytes < 96
 * or a misaligned buffer.
 */
typedef struct {
    uint64_t t_begin; /* device wall clock (hipDeviceAttributeWallClockRate kHz) when the batch
                         was taken */
    uint64_t t_end;   /* when its new tasks were published and it was counted done */
    uint32_t worker;  /* workgroup index */
    uint32_t tasks;   /* tasks in the batch; bit 31 set = a chunk of a hub task (tasks = 1) */
    uint32_t edges;   /* edges scanned, over every pass of the batch */
    uint32_t vertex;  /* vertex of the batch's highest-degree task */
} atos_trace_record;

#define ATOS_TRACE_HUB_CHUNK 0x80000000u
#define ATOS_TRACE_BSP_LEVEL 0x40000000u

atos_status atos_trace_attach(void *d_buf, size_t bytes);

/*
 * ---------------------------------------------------------------- serving
 * A resident daemon for a stream of queries (continuous batching; the
 * serving workload built on the worklist of paper section 3): one persistent
 * worker kernel stays on the GPU and runs BFS and personalized PageRank
 * queries on a fixed set of resident graphs.  Queries are submitted from the
 * host at any time through a ring in pinned host memory; an idle worker
 * admits each into a free query slot, initialises its state with tasks of
 * its own and starts it in the same worklist that carries every running
 * query, so queries that arrive while others run overlap with them on the
 * device.  Completions come back through a second host-memory ring.
 *
 * Memory: the caller passes one device arena (>= 256-byte aligned) that
 * holds the daemon's control block, query slots and worklist rings
 * (atos_server_arena_bytes) followed by the state heap; per-query state is
 * carved from the heap at submit time and returned at release, so admission
 * is bounded by free memory, by free slots and by worklist capacity (a query
 * reserves 2 ring entries per vertex of its graph while it runs, in the ring
 * of its slot by default, where each ring holds 4 entries per resident vertex;
 * with one shared ring or own-ring pushes, the rings together hold 16 per
 * resident vertex).  The server
 * allocates its two host rings with hipHostMalloc at creation; nothing is
 * allocated per query.
 *
 * Result state of a completed query, at arena + state_offset:
 *   BFS:       uint32 depth[n] (0xFFFFFFFF = unreached)
 *   PageRank:  double rank[n], then double residue[n]; the personalized rank
 *              x = (1-d) e_source + d A D^-1 x is approximated with every
 *              residue <= epsilon (same method and bound as atos_pagerank).
 * The state stays valid until atos_server_release.  Calls on one server are
 * serialised by the library (any host thread may call).
 */
typedef struct atos_server *atos_server_t;

typedef struct {
    int32_t worker;         /* threads per worker, 64..1024 (default 1024) */
    int32_t fetch;          /* tasks per pop, 1..worker (default: worker) */
    int32_t grid;           /* daemon workgroups; 0 = co-resident maximum less one per CU */
    int32_t max_queries;    /* query slots, 1..2048 (default 256) */
    int64_t queue_capacity; /* worklist entries per ring (power of two); 0 = default */
    uint32_t timeout_ms;    /* the daemon ends at this deadline even if never stopped
                               (default 600000) */
    int32_t queue_layout;   /* ATOS_QUEUE_PER_XCD (AUTO, default) or ATOS_QUEUE_GLOBAL
                               (one shared ring) */
    int32_t push_policy;    /* with a ring per XCD: ATOS_PUSH_QUERY (AUTO, default): every
                               task goes to the ring of its query's slot, so each query
                               keeps one FIFO order, and a worker takes from another ring
                               only what that ring's own workers could not take at once;
                               ATOS_PUSH_OWN or ATOS_PUSH_SHALLOWEST (see atos_config).
                               With ATOS_PUSH_QUERY admission budgets each ring apart and
                               the default rings hold 4 entries per resident vertex each. */
    uint32_t reserved[3];   /* must be zero */
} atos_server_config;

typedef struct {
    int32_t graph;   /* index into the server's graph list */
    int32_t app;     /* ATOS_APP_BFS, or ATOS_APP_PAGERANK (personalized from source) */
    int64_t source;
    float damping;   /* PageRank only, in (0, 1) */
    float epsilon;   /* PageRank only, > 0 */
    uint64_t tag;    /* returned unchanged with the completion */
    void *out;       /* NULL, or device-accessible memory (pinned host memory from
                        atos_host_alloc, or device memory) where the daemon writes
                        the result before it posts the completion: n int32 depths
                        (-1 = unreached) for BFS; n FP32 ranks then n FP32 residues
                        for PageRank.  The host reads it with no GPU call of its own. */
} atos_query;

typedef struct {
    uint64_t query_id;
    uint64_t tag;
    int32_t status;         /* atos_status of the query */
    int32_t app;
    int32_t graph;
    int32_t reserved;
    uint64_t state_offset;  /* byte offset of the result state in the arena */
    uint64_t tasks;         /* tasks processed, including state initialisation */
    uint64_t edges;         /* neighbour-list entries scanned */
    double device_us;       /* admission to completion on the device clock */
} atos_completion;

/* Arena bytes the server needs before its state heap. */
atos_status atos_server_arena_bytes(const atos_graph_t *graphs, int32_t n_graphs,
                                    const atos_server_config *cfg, size_t *bytes);
/* Create a server over n_graphs loaded graphs (borrowed; every graph must have
 * fewer than 2^25 vertices).  EINVAL for bad arguments, ENOMEM when the arena
 * has no room for a heap. */
atos_status atos_server_create(const atos_graph_t *graphs, int32_t n_graphs,
                               const atos_server_config *cfg, void *d_arena, size_t arena_bytes,
                               atos_server_t *out);
/* Initialise the control block and rings and launch the daemon on `stream`
 * (which it then occupies until stopped); returns without waiting. */
atos_status atos_server_start(atos_server_t s, void *stream);
/* Submit a query; *query_id identifies it in completions.  EAGAIN when no
 * slot, heap memory or worklist capacity is free (nothing was submitted);
 * EINVAL for a bad query or a server not running. */
atos_status atos_server_submit(atos_server_t s, const atos_query *q, uint64_t *query_id);
/* Collect up to max completions (non-blocking); *n_out = number written.
 * When none is ready and the daemon has ended on an error, returns that error
 * (ETIMEOUT, EOVERFLOW or EHIP). */
atos_status atos_server_poll(atos_server_t s, atos_completion *out, int32_t max, int32_t *n_out);
/* Return a completed query's slot and state to the server. */
atos_status atos_server_release(atos_server_t s, uint64_t query_id);
/* Ask the daemon to end once every admitted query is complete, wait for it,
 * and report its counters (device_ms = daemon lifetime, rounds = queries
 * completed).  Returns the daemon's status (OK, ETIMEOUT, EOVERFLOW, EHIP).
 * No submit is accepted after stop; completions can still be polled. */
atos_status atos_server_stop(atos_server_t s, atos_stats *st);
/* Free the server (stopping it first if it runs). */
atos_status atos_server_destroy(atos_server_t s);

/* Pinned host memory the GPU can read and write (hipHostMalloc, mapped and
 * coherent), for query outputs.  Allocate it before the daemon starts and
 * free it after it stops: freeing pinned memory may wait for the device. */
atos_status atos_host_alloc(size_t bytes, void **out);
atos_status atos_host_free(void *p);

/* The daemon's state for inspection while it runs: a worker of the daemon
 * copies it into host memory on request (consistent per word, not across
 * words; waits up to 5 s for a worker, EINVAL when the daemon is not
 * running, ETIMEOUT when no worker answered).
 * Writes, as uint64 words: [0] status, [1] submit_head, [2] comp_tail,
 * [3] active, [4] admitted, [5] completed, [6] worklist rings, [7] ring
 * capacity, [8] query slots, [9] device clock at the daemon's start, [10]
 * device clock when it found its deadline passed (0 if not), [11] device
 * clock rate in kHz, [12] this server's launch number, [13] and [14] the
 * launch numbers that wrote [9] and [10]; then per ring (head, tail, done);
 * then per slot
 * (query_id, pending, init_left, app << 32 | graph); then the first
 * `ring_words` (<= 8) slot words of every ring from its head.  *n_words =
 * words written (EINVAL when max_words is too small). */
atos_status atos_server_snapshot(atos_server_t s, int32_t ring_words, uint64_t *out,
                                 int64_t max_words, int64_t *n_words);

/* Human-readable name of a status code (static string). */
const char *atos_strerror(atos_status s);

/* Library version, "major.minor.patch". */
const char *atos_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ATOS_H */
