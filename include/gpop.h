/*
 * gpop.h -- C ABI of the MI355X partition-centric scatter/gather engine.
 *
 * The engine runs the iteration of "GPOP: A scalable cache- and
 * memory-efficient framework for Graph Processing Over Partitions"
 * (Lakhotia, Pati, Kannan, Prasanna): vertices are split into index-range
 * partitions of q vertices (Sec. 3.1.1); each iteration scatters the active
 * partitions' messages into per-(source, destination)-partition bins, in
 * source-centric or partition-centric mode chosen per partition (Sec. 3.1.2,
 * Algorithms 2 and 3, Sec. 3.2), then gathers each destination partition's
 * bins into its vertex state and builds the next frontier (Algorithm 2).
 *
 * Conventions for every call:
 *   - Return value is a gpop_status; 0 (GPOP_OK) means success. On failure
 *     gpop_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread). No C++ exception crosses this boundary.
 *   - "device" pointers are HIP device allocations owned by the caller. The
 *     library never allocates device memory: every device buffer it uses is
 *     carved from the caller's workspace, whose size gpop_plan() reports.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Calls enqueue work on it and return without synchronising unless the
 *     call says otherwise.
 *   - A gpop_graph handle is not thread-safe; one handle serves one stream
 *     at a time. It borrows the CSR, the workspace and the state array, which
 *     must outlive it.
 */
#ifndef GPOP_H
#define GPOP_H

#include <stddef.h>
#include <stdint.h>

#include "gpop_mlp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GPOP_ABI_VERSION 1

typedef enum gpop_status {
    GPOP_OK = 0,
    GPOP_EINVAL = 1,    /* malformed argument or graph                      */
    GPOP_ENOMEM = 2,    /* workspace smaller than gpop_plan() asked for     */
    GPOP_EDEVICE = 3,   /* a HIP runtime call failed                        */
    GPOP_ESTATE = 4,    /* call out of order (e.g. iterate before init)     */
    GPOP_ENOTSUP = 5    /* valid request this library does not support      */
} gpop_status;

/* Programs: the user functions of the programming-interface section
 * (scatterFunc, initFunc, gatherFunc, filterFunc, applyWeight) compiled in.
 * Gather combines messages with a commutative, associative reduce (min for
 * the integer programs, sum for the PageRank family), which is what lets one
 * workgroup combine a partition's messages in parallel. */
typedef enum gpop_program {
    GPOP_PROG_BFS_LEVEL = 0,     /* u32 hop level; unreached 0xFFFFFFFF (BFS app)     */
    GPOP_PROG_CC_MINLABEL = 1,   /* u32 min vertex id of the component (CC app)       */
    GPOP_PROG_SSSP_U32 = 2,      /* u32 distance, u8 weights, saturating (SSSP app)   */
    GPOP_PROG_PAGERANK_F32 = 3,  /* f32 PageRank, dangling mass spread uniformly       */
    GPOP_PROG_PPR_F32 = 4,       /* f32 personalised PageRank, restart to one seed     */
    GPOP_PROG_CARRY_BFS = 5,     /* BFS levels where initFunc keeps a reached vertex
                                    active for `persist` iterations (selective
                                    continuity of the active set)                      */
    GPOP_PROG_BFS_PARENT = 6,    /* u32 parent in the BFS tree of the root (Algorithm 5):
                                    scatterFunc sends the vertex id, gatherFunc sets
                                    the parent of an unvisited vertex; of the messages
                                    one iteration brings, the least source id wins
                                    (the first in the paper's gather order); the
                                    root's parent is the root, unreached 0xFFFFFFFF  */
    GPOP_PROG_NIBBLE_F32 = 7     /* f32 Parallel Nibble (the paper's Nibble application):
                                    scatterFunc sends PR/(2 deg), initFunc halves PR
                                    and keeps the vertex iff PR >= eps * deg,
                                    gatherFunc adds, filterFunc keeps iff
                                    PR >= eps * deg; a vertex without out-edges is
                                    never kept. Seed PR = 1, others 0              */
} gpop_program;

typedef enum gpop_selector {
    GPOP_SEL_ANALYTICAL = 0,  /* Eq. 1 of the performance-modelling section      */
    GPOP_SEL_FORCE_SC = 1,    /* every scattered partition source-centric        */
    GPOP_SEL_FORCE_PC = 2,    /* every scattered partition partition-centric     */
    GPOP_SEL_LEARNED = 3      /* MLP on per-partition features; falls back to    */
                              /* the analytical model if no valid weights        */
} gpop_selector;

/* Per-partition mode of one iteration. */
#define GPOP_MODE_NONE 0u  /* no active vertex: not scattered */
#define GPOP_MODE_SC 1u
#define GPOP_MODE_PC 2u

/* CSR input (the graph format of the challenges section): offsets has V + 1
 * non-decreasing entries with offsets[0] = 0 and offsets[V] = E; cols has E
 * entries < V, each row sorted ascending (duplicates and self-loops allowed);
 * weights is NULL or E bytes. All three are device pointers. */
typedef struct gpop_graph_desc {
    uint32_t num_vertices;        /* V >= 1                                   */
    uint32_t reserved0;
    uint64_t num_edges;           /* E < 2^32                                 */
    const uint32_t* offsets;
    const uint32_t* cols;
    const uint8_t* weights;
} gpop_graph_desc;

/* How gather combines a partition's messages in the workgroup's on-chip copy
 * of its state (neither uses global atomics or locks; both give the same
 * bits):
 *   GPOP_COMBINE_LDS    one LDS min / 64-bit integer add per message (default)
 *   GPOP_COMBINE_ROUNDS atomic-free: write-then-verify rounds (min) and
 *                       per-destination tag rounds (sum), barriers between
 *                       rounds */
#define GPOP_COMBINE_LDS 0u
#define GPOP_COMBINE_ROUNDS 1u

/* Where gather reads the static ids of partition-centric bins (Sec. 3.1.2;
 * the results are the same bits either way):
 *   GPOP_PCSTREAM_AUTO  column streams in iterations where partition-centric
 *                       partitions hold at least half of the graph's edges,
 *                       the per-bin layout otherwise (default)
 *   GPOP_PCSTREAM_OFF   always the per-bin layout; the column streams are
 *                       not built (smaller workspace, faster preprocessing)
 *   GPOP_PCSTREAM_ON    column streams whenever a partition is scattered
 *                       partition-centric
 * A column stream holds every static id of one destination partition, bins
 * in source order, cut into 256-id chunks; per chunk a bitmap of bin starts
 * and a short table ({message offset, source partition}) of the bins that
 * start in it let a wave decode a whole chunk that spans several bins. */
#define GPOP_PCSTREAM_AUTO 0u
#define GPOP_PCSTREAM_OFF 1u
#define GPOP_PCSTREAM_ON 2u

/* How a source-centric task reserves the slots of its messages in the bins
 * (gpop_options.sc_reserve):
 *   GPOP_SCRES_AUTO   per bin when the iteration's tasks hold at least 2k
 *                     work units, else per message piece
 *   GPOP_SCRES_PIECE  one device-wide atomic per message piece (one pass)
 *   GPOP_SCRES_BIN    two passes: the wave counts its pieces per bin in LDS,
 *                     reserves each bin's share with one atomic, then writes
 * The result is the same in every mode; only the order of messages inside a
 * bin differs, and no combine depends on it. */
#define GPOP_SCRES_AUTO 0u
#define GPOP_SCRES_PIECE 1u
#define GPOP_SCRES_BIN 2u

typedef struct gpop_options {
    uint32_t log2_part;   /* q = 2^log2_part vertices per partition, 8..15;
                             0 picks 14 (16384 vertices)                        */
    uint32_t sc_task_log2;     /* log2 of the largest source-centric task, in
                                  work units (an active vertex and each of its
                                  out-edges count one each), 6..24; 0 picks
                                  max(1024, 4k). Iterations with little
                                  source-centric work use smaller tasks       */
    uint32_t gather_task_ids;  /* ids per gather task (>= 256); 0 picks
                                  max(2^16, E / n), n = 2^20 / k clamped to
                                  [256, 512]. A partition whose bins hold more
                                  ids is gathered by several tasks (at most
                                  64) and merged                               */
    uint32_t combine;          /* GPOP_COMBINE_LDS (0) or GPOP_COMBINE_ROUNDS   */
    uint32_t pc_stream;        /* GPOP_PCSTREAM_AUTO (0), _OFF or _ON: how
                                  gather reads partition-centric bins       */
    uint32_t sc_reserve;       /* GPOP_SCRES_AUTO (0), _PIECE or _BIN        */
    uint32_t reserved[2];      /* must be zero                                  */
} gpop_options;

typedef struct gpop_plan_info {
    uint32_t q;                 /* vertices per partition                     */
    uint32_t k;                 /* number of partitions, ceil(V / q)          */
    uint64_t workspace_bytes;   /* device workspace gpop_graph_create needs   */
    uint64_t reserved[6];
} gpop_plan_info;

typedef struct gpop_params {
    uint32_t root;       /* BFS / SSSP / CARRY root, PPR seed                 */
    uint32_t persist;    /* CARRY_BFS: iterations a vertex stays active (>=1) */
    float damping;       /* PAGERANK damping d (0.85 in the paper's runs)    */
    float alpha;         /* PPR restart probability                           */
    float epsilon;       /* NIBBLE threshold eps (> 0, finite)                */
    uint32_t reserved[3];
} gpop_params;

/* Static per-graph statistics after preprocessing. */
typedef struct gpop_graph_info {
    uint32_t q, k;
    uint64_t num_vertices, num_edges;
    uint64_t num_messages;      /* M = sum_p r^p E^p: PNG messages (Sec. 3.1.2) */
    uint64_t nonempty_bins;     /* (p, q) pairs with at least one edge          */
    uint64_t reserved[6];
} gpop_graph_info;

/* One record per completed iteration (written on the device). */
typedef struct gpop_iter_stats {
    uint64_t active_vertices;   /* sum_p V_a^p at the start of the iteration  */
    uint64_t active_edges;      /* sum_p E_a^p                                 */
    uint32_t sc_parts, pc_parts;
    uint64_t sc_msgs, sc_ids;   /* messages / ids written in SC mode           */
    uint64_t pc_msgs, pc_ids;   /* messages / static ids of PC partitions      */
    uint64_t gathered_ids;      /* non-identity ids combined by gather         */
    uint32_t gather_parts;      /* whole-partition gather tasks that ran       */
    uint32_t split_tasks;       /* partial gather tasks that wrote a result    */
    uint64_t sc_active_vertices; /* V_a summed over SC partitions              */
    uint64_t sc_active_edges;    /* E_a summed over SC partitions              */
    uint64_t pc_vertices;        /* vertices of PC partitions                  */
    uint64_t merged_parts;       /* split partitions merged                    */
    uint32_t learned_fallbacks;  /* partitions the learned selector left to Eq. 1 */
    uint32_t gathered_bins;      /* bins listed by the active list and read by gather */
} gpop_iter_stats;

/* ------------------------------------------------------------------ setup */

/* Partition count and workspace size for a graph (host-side arithmetic from
 * V, E and the options; the device pointers are not read). Partitioning is
 * the paper's index-range scheme with q a power of two (Sec. 3.1.1).
 * Errors: GPOP_EINVAL for V = 0, E >= 2^32, bad log2_part or nonzero
 * reserved fields. */
int gpop_plan(const gpop_graph_desc* desc, const gpop_options* opts, gpop_plan_info* out);

/* Validates the CSR on the device and builds the partition-node bipartite
 * layout (PNG, Sec. 3.1.2 and Algorithm 3): for every partition pair (p, q)
 * the sources N_i^p(q) and their destination ids, written once and reused by
 * every partition-centric scatter. Runs on `stream` and synchronises it.
 * d_workspace must be 256-byte aligned with ws_bytes >= workspace_bytes.
 * Errors: GPOP_EINVAL (malformed CSR: non-monotone offsets, col >= V, unsorted
 * row), GPOP_ENOMEM (workspace too small), GPOP_EDEVICE. */
int gpop_graph_create(const gpop_graph_desc* desc, const gpop_options* opts,
                      void* d_workspace, size_t ws_bytes, void* stream, struct gpop_graph** out);

/* Releases the host-side handle (device memory stays the caller's). NULL ok. */
int gpop_graph_destroy(struct gpop_graph* g);

int gpop_graph_get_info(const struct gpop_graph* g, gpop_graph_info* out);

/* ---------------------------------------------------------------- program */

/* Binds `prog` and the caller's state array (V x 4 bytes: u32 for the integer
 * programs, f32 for the PageRank family and Nibble) and writes its initial
 * values (initial val[] of each application in the applications section;
 * PageRank 1/V, PPR e_seed, Nibble e_seed, CC v, BFS/SSSP/CARRY infinity
 * except root = 0, BFS_PARENT 0xFFFFFFFF except root = root). Clears the
 * frontier and the iteration counter. Errors: GPOP_EINVAL for a bad program,
 * root >= V, persist = 0, a weighted program on an unweighted graph, damping
 * or alpha outside [0, 1], or a Nibble epsilon that is not finite and > 0. */
int gpop_state_init(struct gpop_graph* g, gpop_program prog, const gpop_params* prm,
                    void* d_state, void* stream);

/* loadFrontier (applications section): makes the n device-resident vertex
 * ids the active set. Order and duplicates do not matter. Ids >= V make the
 * next gpop_check() report GPOP_EINVAL and are ignored. */
int gpop_set_frontier(struct gpop_graph* g, const uint32_t* d_vertices, uint32_t n, void* stream);

/* Makes every vertex active. */
int gpop_set_frontier_all(struct gpop_graph* g, void* stream);

/* Mode selection per partition (performance-modelling section). bw_ratio is
 * BW_PC / BW_SC. The paper's figure for its CPU is 2; a new graph starts with
 * the analytical model at 16, the ratio that is fastest on MI355X across the
 * BFS/CC and SSSP workloads (source-centric bins are written in partial cache
 * lines, partition-centric values in full ones). s_i / s_v are the index and value
 * sizes in bytes used by the model (the paper uses 4 and 4). For
 * GPOP_SEL_LEARNED, d_mlp is a device gpop_mlp_model (gpop_mlp.h); the call
 * copies it into the graph's workspace (synchronously), so the caller may
 * free or retrain it afterwards. A model whose header is wrong or whose
 * values are not finite is rejected with GPOP_EINVAL and the previous
 * selector stays active; NULL with GPOP_SEL_LEARNED selects the analytical
 * model. bw_ratio, s_i and s_v also feed the learned model's last feature
 * and its analytical fallback. */
int gpop_set_selector(struct gpop_graph* g, gpop_selector kind, float bw_ratio,
                      uint32_t s_i, uint32_t s_v, const void* d_mlp);

/* Interleaved scatter-gather (Sec. 3.3): when a partition is scattered it
 * should already carry the updates its in-neighbours sent earlier in the same
 * iteration. Here the partitions are cut into `classes` contiguous index
 * ranges (colour classes); engine iteration t scatters only the active
 * partitions of class t mod classes and gathers every column, and the other
 * active partitions keep their frontier, so they scatter in a later
 * iteration with values those gathers already improved. Every wait stays at
 * a kernel boundary. classes = 0 or 1 turns it off (the default); 2..16 turn
 * it on. Each engine iteration (one class scattered) counts as an iteration
 * of gpop_run and of the statistics records. Only the programs whose gather
 * keeps a minimum, whose result is the unique fixed point whatever the order
 * of updates, take it: BFS_LEVEL, CC_MINLABEL and SSSP_U32 (the paper
 * enables it for connected components and SSSP). Errors: GPOP_EINVAL for
 * classes > 16; GPOP_ENOTSUP if the bound program is another one (and
 * gpop_state_init of another program fails with GPOP_ENOTSUP while it is
 * on). */
int gpop_set_isg(struct gpop_graph* g, uint32_t classes);

/* Per-partition features of the learned selector (gpop_mlp.h) for the
 * current frontier and iteration: writes k x GPOP_MLP_IN floats (row p =
 * partition p) to d_out. Partitions without active vertices get their
 * features too (V_a = E_a = 0). */
int gpop_features(struct gpop_graph* g, float* d_out, void* stream);

/* Measures what scattering the current frontier costs in one mode, without
 * changing the run: plans every active partition in mode `kind`
 * (GPOP_SEL_FORCE_SC or GPOP_SEL_FORCE_PC), runs that mode's scatter kernels
 * with per-task timers, and splits the measured kernel time over the
 * partitions in proportion to the wave time their tasks took. Writes k
 * floats (microseconds; 0 for partitions without active vertices) to h_us
 * and the whole scatter time to *h_total_us (either may be NULL).
 * Synchronises `stream`. The bins it writes are overwritten by the next
 * gpop_scatter, and the iteration records are unaffected. Errors:
 * GPOP_EINVAL for another kind, GPOP_ESTATE before gpop_state_init. */
int gpop_probe_scatter(struct gpop_graph* g, gpop_selector kind, float* h_us, float* h_total_us,
                       void* stream);

/* -------------------------------------------------------------- iteration */

/* Scatter half of one iteration (Algorithm 2, scatter phase, with
 * Algorithm 3 for partition-centric partitions): picks the mode of each
 * partition with active vertices and writes its bins. */
int gpop_scatter(struct gpop_graph* g, void* stream);

/* Gather half (Algorithm 2: reInit, gather, filter): each partition that
 * received messages or has active vertices combines its bins into its
 * state in on-chip memory, then builds the next frontier. */
int gpop_gather(struct gpop_graph* g, void* stream);

/* scatter_and_gather: one full iteration. */
int gpop_iterate(struct gpop_graph* g, void* stream);

/* Iterates while the frontier is non-empty and fewer than max_iter
 * iterations have run (the driver loop of the applications section).
 * Iterations are recorded once per program as a HIP graph of four
 * iterations and replayed; the device stops a run when its frontier is
 * empty or the limit is reached (later kernels of a replay return at once).
 * Synchronises `stream` before returning and reports the iterations run in
 * *h_iters (may be NULL). Reaching max_iter with a non-empty frontier is not
 * an error: gpop_frontier_size() then reports the remaining frontier, and a
 * later gpop_run or gpop_iterate continues from there. */
int gpop_run(struct gpop_graph* g, uint32_t max_iter, uint32_t* h_iters, void* stream);

/* G.frontierSize: number of active vertices. Synchronises `stream`. */
int gpop_frontier_size(struct gpop_graph* g, uint64_t* h_out, void* stream);

/* Iterations completed since gpop_state_init (host-side counter). */
int gpop_iterations(const struct gpop_graph* g, uint32_t* h_out);

/* Copies up to max_records per-iteration records (oldest first) into h_out
 * and reports how many were copied. Synchronises `stream`. */
int gpop_iter_stats_read(struct gpop_graph* g, gpop_iter_stats* h_out, uint32_t max_records,
                         uint32_t* h_count, void* stream);

/* Copies the per-partition modes chosen in the most recent scatter (k bytes,
 * GPOP_MODE_*) into h_modes. Synchronises `stream`. */
int gpop_modes_read(struct gpop_graph* g, uint8_t* h_modes, void* stream);

/* Reads the device error word (ids >= V passed to gpop_set_frontier).
 * Synchronises `stream`. Returns GPOP_EINVAL if an error was recorded. */
int gpop_check(struct gpop_graph* g, void* stream);

/* ---------------------------------------------------------------- batches */

/* A batch runs one program many times at once: several seeds on one graph
 * (graphs[i] may repeat) or independent graphs of any size. Each run has
 * its own state, frontier and bins; the graphs' preprocessed layouts are
 * shared. Every kernel of an iteration is launched once for all runs (each
 * run owns a slice of the grid), and a fixed number of iterations is
 * recorded once as a HIP graph and replayed until every run has finished, so
 * the host neither launches per run nor synchronises per iteration. The
 * graph handles must outlive the batch and must not be iterated while the
 * batch runs. Each run uses its graph's selector (gpop_set_selector). */
struct gpop_batch;

#define GPOP_BATCH_EAGER 1u  /* gpop_batch_run flag: launch directly, no HIP graph */

/* Device workspace bytes for a batch of n runs on graphs[0..n-1]. */
int gpop_batch_plan(struct gpop_graph* const* graphs, uint32_t n, uint64_t* ws_bytes);

/* Creates the batch over a caller-owned, 256-byte aligned workspace of at
 * least gpop_batch_plan bytes. Synchronises `stream`. Errors: GPOP_EINVAL
 * (NULL graphs, n = 0, misaligned workspace), GPOP_ENOMEM (workspace too
 * small). */
int gpop_batch_create(struct gpop_graph* const* graphs, uint32_t n, void* d_ws, size_t ws_bytes,
                      void* stream, struct gpop_batch** out);

/* Releases the host-side handle and its recorded graph. NULL ok. */
int gpop_batch_destroy(struct gpop_batch* b);

/* Binds `prog` to every run: prm[i] and the state array d_states[i] (V_i x
 * 4 bytes) of run i, and writes the initial values as gpop_state_init does.
 * Synchronises `stream`. Errors as gpop_state_init, for any run. */
int gpop_batch_state_init(struct gpop_batch* b, gpop_program prog, const gpop_params* prm,
                          void* const* d_states, void* stream);

/* Frontier of run `run` (after gpop_batch_state_init, before
 * gpop_batch_run), as gpop_set_frontier / gpop_set_frontier_all. */
int gpop_batch_set_frontier(struct gpop_batch* b, uint32_t run, const uint32_t* d_vertices, uint32_t n,
                            void* stream);
int gpop_batch_set_frontier_all(struct gpop_batch* b, uint32_t run, void* stream);

/* Runs every run until its frontier is empty or it has done max_iter more
 * iterations. flags: 0 or GPOP_BATCH_EAGER. Synchronises `stream`; h_iters
 * (n entries, may be NULL) receives each run's iteration count. */
int gpop_batch_run(struct gpop_batch* b, uint32_t max_iter, uint32_t flags, uint32_t* h_iters,
                   void* stream);

/* gpop_check for every run. Synchronises `stream`. */
int gpop_batch_check(struct gpop_batch* b, void* stream);

/* -------------------------------------------------------------- autotuner */

/* Tuning space: partition size 2^log2_part (the paper's partition-size
 * parameter, sized here to the workgroup's on-chip memory) and the "bin tile
 * shape": ids per gather task (gather_task_ids) and active edges per
 * source-centric task (2^sc_task_log2). */
#define GPOP_TUNE_MAX 64

typedef struct gpop_tune_result {
    gpop_options best;             /* fastest candidate                          */
    float best_ms;                 /* its run time                               */
    uint32_t n_tried;              /* candidates that could run                  */
    float run_ms[GPOP_TUNE_MAX];   /* per candidate (in the order given): fastest of the
                                      repetitions, or a negative value if it could not
                                      run (plan, workspace or on-chip memory)     */
    float prep_ms[GPOP_TUNE_MAX];  /* preprocessing time of each candidate       */
} gpop_tune_result;

/* Fills out[0..*n) with the default candidates for `prog` on a graph of V
 * vertices and E edges: every partition size from 2^12 to 2^15 whose gather
 * fits on chip (one size at least V, at most), crossed with gather tasks of
 * the default size or 2^16 ids and source-centric tasks of the default size
 * or 2^12 edges. */
int gpop_autotune_candidates(gpop_program prog, uint32_t num_vertices, uint64_t num_edges,
                             gpop_options* out, uint32_t cap, uint32_t* n);

/* Times `prog` on the graph for each candidate: builds the layout in the
 * caller's workspace (at least the largest gpop_plan size of the
 * candidates), binds d_state, sets the frontier (d_frontier[0..n_frontier),
 * or every vertex when d_frontier is NULL), runs at most max_iter
 * iterations `reps` times, keeps the fastest. The graph layout built last is
 * released; build the chosen one with gpop_graph_create. Synchronises
 * `stream`. Errors: GPOP_EINVAL (bad arguments, n_cand = 0 or >
 * GPOP_TUNE_MAX), GPOP_ENOTSUP if no candidate could run. */
int gpop_autotune(const gpop_graph_desc* desc, gpop_program prog, const gpop_params* prm,
                  const uint32_t* d_frontier, uint32_t n_frontier, uint32_t max_iter, uint32_t reps,
                  const gpop_options* cands, uint32_t n_cand, void* d_ws, size_t ws_bytes,
                  void* d_state, void* stream, gpop_tune_result* out);

/* ------------------------------------------------------------- profiling */

/* Kernel identifiers for gpop_profile_read. */
#define GPOP_KERNEL_PLAN 0
#define GPOP_KERNEL_SCATTER_SC 1
#define GPOP_KERNEL_SCATTER_PC 2
#define GPOP_KERNEL_GATHER 3
#define GPOP_KERNEL_MERGE 4  /* combine of partitions gathered by several tasks */
#define GPOP_KERNEL_COUNT 5

/* When enabled, every kernel launch is bracketed by HIP events on its
 * stream. gpop_profile_read synchronises the stream and returns, per kernel
 * id, the summed milliseconds and the number of launches since profiling
 * was enabled (arrays of GPOP_KERNEL_COUNT entries). While profiling,
 * gpop_run launches its iterations directly instead of replaying the
 * recorded HIP graph (the kernels are the same). */
int gpop_profile_enable(struct gpop_graph* g, int enable);
int gpop_profile_read(struct gpop_graph* g, double* h_ms, uint64_t* h_launches, void* stream);

/* Reference streams for the roofline of the kernels above: one launch on
 * `stream` of a plain kernel that moves `bytes` bytes of device memory in
 * the access mix `mix`, so that a caller timing it gets the bandwidth that
 * mix reaches on this GPU. GPOP_STREAM_READ reads `bytes` bytes of d_src
 * (d_dst: at least 4 bytes, written at most once); GPOP_STREAM_COPY copies
 * `bytes` bytes of d_src to d_dst (the reads and writes of the merge, and
 * the copy ceiling); GPOP_STREAM_WIDEN reads `bytes` bytes of 16-bit words
 * from d_src and writes them widened to 32 bits, 2 * bytes bytes, to d_dst
 * (the mix of the partition-centric scatter's stream: a 2-byte source index
 * read and a 4-byte value written per message slot). The gather reads far
 * more than it writes: its reference is GPOP_STREAM_READ.
 * GPOP_STREAM_SEGMENTS reads `bytes` bytes of d_src as 512-byte segments in a
 * scattered order (segment j at j times an odd constant, modulo their
 * count; d_dst as for GPOP_STREAM_READ): the pattern of the gather's message
 * values, short runs spread over the message array; `bytes` / 512 must be
 * a power of two. Both pointers
 * are 16-byte aligned, `bytes` is a nonzero multiple of 16 (of 8 for
 * GPOP_STREAM_WIDEN) and below 2^40; d_src and d_dst are the caller's and
 * do not overlap. Errors: GPOP_EINVAL for another mix, a NULL or misaligned
 * pointer or a bad size; GPOP_EDEVICE if the launch fails. */
#define GPOP_STREAM_READ 0
#define GPOP_STREAM_COPY 1
#define GPOP_STREAM_WIDEN 2
#define GPOP_STREAM_SEGMENTS 3
int gpop_stream_ceiling(int mix, const void* d_src, void* d_dst, uint64_t bytes, void* stream);

/* --------------------------------------------------------------- errors */

const char* gpop_last_error(void);
int gpop_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GPOP_H */
