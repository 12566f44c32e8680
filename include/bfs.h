/*
 * bfs.h - C ABI of libbfs.so: level-synchronous breadth-first search and the
 * local sparse-matrix x sparse-vector product (SpMSpV) of the 2D algorithm,
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method (Bulu\c{c} and Madduri, "Parallel Breadth-First Search on
 * Distributed Memory Systems"):
 *   - BFS explores the graph one level at a time (section 2.1, Algorithm 1;
 *     one synchronisation per level as in the PRAM formulation of section
 *     2.2).
 *   - Each level is the product x_{k+1} = A^T (x) x_k masked by the
 *     complement of the visited set (section 3.2): a sparse-matrix x
 *     sparse-vector product over a (select, min) semiring, with a dense
 *     parents array standing in for the union of past frontiers.
 *   - One process's share of the 2D decomposition (section 3.2, Eq. of the
 *     2D partitioning; Algorithm 3) is a hypersparse block stored as DCSC
 *     (section 4.1: IR row ids, CP column pointers, JC non-empty column
 *     ids); its local product is bfs_spmspv (Algorithm 3, the SpMSV step;
 *     section 4.2).
 *
 * Output convention (Algorithm 3): parent[v] is the predecessor of v on a
 * shortest path from the root, -1 when unreachable; parent[root] = root.
 * level[v] is the hop distance d(root, v) (Algorithm 1's d), -1 when
 * unreachable. The semiring's "min" makes parent[v] the smallest vertex id
 * among the neighbours of v one level closer to the root, so results are
 * unique and deterministic.
 *
 * Conventions of every call:
 *   - Returns a bfs_status code (0 = BFS_OK); never throws or aborts across
 *     the ABI. bfs_last_error() gives a thread-local message for the last
 *     failing call on the calling thread.
 *   - Vertex ids and DCSC indices are int32 (ids < 2^31). CSR row offsets
 *     are int32 or int64 at the caller's choice (stored as int64 on the
 *     device).
 *   - Input arrays are copied at create time: the library owns its device
 *     copy, and the caller may free its arrays as soon as create returns.
 *   - Output arrays are caller-owned. They are device pointers (e.g. a
 *     PyTorch tensor's data_ptr()) unless stated otherwise; bfs_run also
 *     accepts host pointers (filled by a copy on the same stream).
 *   - Streams are hipStream_t passed as void* (NULL = the default stream).
 *   - All calls on one graph handle must come from one host thread at a
 *     time; a handle's device workspace is shared by its runs, so two runs on
 *     one handle must not overlap on different streams.
 */
#ifndef BFS_MI355X_BFS_H
#define BFS_MI355X_BFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfs_graph bfs_graph_t;
typedef struct bfs_server bfs_server_t;

typedef enum bfs_status {
  BFS_OK = 0,
  BFS_ERR_ARG = -1,         /* bad argument (null handle, root out of range, ...) */
  BFS_ERR_FORMAT = -2,      /* malformed CSR/DCSC rejected at create */
  BFS_ERR_OOM = -3,         /* device or host allocation failed */
  BFS_ERR_CAPACITY = -4,    /* output too small; required size reported */
  BFS_ERR_DEVICE = -5,      /* HIP runtime or kernel error */
  BFS_ERR_BUSY = -6,        /* handle has work in flight */
  BFS_ERR_TIMEOUT = -7,     /* wait or server ticket timed out */
  BFS_ERR_UNSUPPORTED = -8  /* size or mode outside what this build handles */
} bfs_status_t;

/* Flags for the create calls. */
#define BFS_DEVICE_PTRS 0x1u  /* input arrays are device pointers */
#define BFS_TRUSTED 0x2u      /* skip validation of the input arrays */
#define BFS_SYMMETRIC 0x4u    /* CSR: caller asserts an undirected graph (every edge in both
                                 rows) with ascending adjacency lists; without this flag and
                                 without BFS_TRUSTED the library checks it at create */
#define BFS_NO_RELABEL 0x8u   /* CSR: do not build the degree-ordered copy that graphs with
                                 n >= 2^20 otherwise get for the single-query level kernels
                                 (results are identical either way; the copy costs nnz * 4 +
                                 n * 16 device bytes) */
#define BFS_UPPER 0x10u       /* CSR: symmetric storage (the paper's closing section): the
                                 arrays hold each undirected edge once, in the row of its
                                 smaller endpoint (every adjacency v of row u has v > u, rows
                                 strictly ascending; checked unless BFS_TRUSTED, else
                                 BFS_ERR_FORMAT). bfs_run searches the symmetric closure with
                                 the same results as the full CSR, storing half the
                                 adjacencies and no degree-ordered copy: each level pushes the
                                 frontier's stored (larger) neighbours and every unvisited
                                 vertex not reached that way scans its own row for a frontier
                                 vertex, so levels read the rows of all unvisited vertices.
                                 Such graphs run through bfs_run / bfs_run_async / bfs_tune
                                 and the server's whole-GPU lane; bfs_run_batch rejects them
                                 (BFS_ERR_UNSUPPORTED). */

/*
 * Sparse vector with device storage, indices strictly ascending (the 2D
 * algorithm's frontier is a sorted sparse vector, section 4.1).
 *   nnz       number of entries (host value; set by bfs_spmspv on output)
 *   capacity  entries that idx/val can hold (output vectors only)
 *   idx       device int32[capacity], ascending
 *   val       device int32[capacity]; for an input frontier it may be NULL,
 *             meaning val(k) = k (the frontier vertex's own id is selected)
 */
typedef struct bfs_svec {
  int64_t nnz;
  int64_t capacity;
  int32_t* idx;
  int32_t* val;
} bfs_svec_t;

/* Statistics of the last completed run on a graph handle. */
typedef struct bfs_run_stats {
  int32_t depth;             /* largest level assigned (0 for an isolated root) */
  int32_t levels;            /* levels expanded (levels with a non-empty input frontier) */
  int64_t edges_traversed;   /* sum of the degrees of the reached vertices (twice the
                                undirected edges of the searched component, the TEPS
                                numerator); pull levels examine fewer (pull_edges) */
  int64_t reached;           /* vertices with level >= 0 */
  int64_t frontier_total;    /* sum of frontier sizes over all levels */
  int32_t expand_launches;   /* launch groups enqueued (each: the device level loop for small
                                frontiers, then one level's kernels), including empty
                                speculative ones */
  int32_t mark_levels;       /* levels resolved by mark-and-resolve instead of atomicMin */
  double expand_ms;          /* summed device time of the levels' expand launches, claim,
                                mark and pull kernels (options.profile = 1) */
  double mark_ms;            /* the mark-and-resolve expand kernel's share of expand_ms */
  double total_ms;           /* device time of the whole run (options.profile = 1) */
  int32_t pull_levels;       /* mark levels whose product was computed by rows (pull) */
  int32_t reserved;
  double pull_ms;            /* the pull kernel's share of expand_ms */
  int64_t pull_edges;        /* adjacencies examined by the pull levels */
  int32_t small_levels;      /* levels run by the device level loop for small frontiers */
  int32_t reserved2;
  double small_ms;           /* device time of the device level loop's launches (profile = 1) */
  double finish_ms;          /* device time of the levels' finish launches (profile = 1) */
} bfs_run_stats_t;

/* Run-time tuning knobs of a graph handle (0 = keep the current value). */
typedef struct bfs_options {
  int32_t mode;         /* 1 = the level kernels enqueued level by level (batch_levels
                           between host reads of the frontier size); 2 = graph mode: 16
                           levels captured once in a hipGraph and replayed, 1, 2, 4 then
                           8 replays between host reads (high-diameter graphs); profiling
                           then records the whole-run time only */
  int32_t batch_levels; /* levels enqueued between host checks in mode 1 */
  int32_t grid_blocks;  /* blocks of the expand kernel */
  int32_t lds_bitmap;   /* 1 = stage the visited bitmap in LDS when it fits */
  int32_t profile;      /* 1 = time each level's expand and finish with HIP events (-1 = off) */
  int32_t claim;        /* how a level resolves its new vertices' parents:
                           3 = by frontier size (default), 1 = atomicMin claims always,
                           2 = mark-and-resolve whenever the graph is symmetric */
  int32_t claim_threshold; /* frontier edges from which a level uses mark-and-resolve
                              (0 = keep; default max(n / 64, 4096)) */
  int32_t claim_min_frontier; /* frontier vertices from which a level uses mark-and-resolve
                                 (0 = keep; default n / 1024 clamped to [1024, 4096]); a
                                 frontier whose adjacencies times pull_alpha reach nnz
                                 pulls whatever its vertex count */
  int32_t cold_probe;   /* mark-and-resolve expands, targets beyond the LDS-resident hot
                           prefix of the visited bitmap: 1 = read the touch-mark byte;
                           2 = read the visited word first, the byte only when unvisited;
                           3 = 2 once a quarter of the vertices is reached, else 1
                           (0 = keep; default 3) */
  int32_t spmspv_sort_max; /* bfs_spmspv: frontiers of up to this many entries (at most
                              8192) take the single-workgroup sort path when their product
                              fits it, larger ones the sparse accumulator; -1 = never
                              (0 = keep; default 512; bfs_tune measures it) */
  int32_t pull_alpha;   /* a mark level computes its product by rows (every unvisited vertex
                           searches its ascending adjacency list for the first vertex of the
                           frontier) instead of pushing the frontier's adjacencies when
                           pull_alpha * (frontier adjacencies) >= adjacencies of the
                           vertices not yet visited; -1 = never (0 = keep; default 14) */
  int32_t small_frontier; /* device level loop: claim levels whose frontier holds at most
                             this many vertices (and at most 16384 adjacencies) run inside one
                             workgroup, level after level, without host checks or per-level
                             launches (high-diameter graphs, first and last levels of every
                             search); at most 8192; -1 = off (0 = keep; default 8192). Not
                             used for BFS_UPPER graphs */
} bfs_options_t;

/* ---------------------------------------------------------------- graphs */

/*
 * CSR graph with n vertices and nnz adjacencies (section 4.1, "Graph
 * Representation": the adjacencies of vertex i are contiguous and sorted,
 * row_offsets has n + 1 entries). offset_bytes is 4 or 8. For an undirected
 * graph each edge appears in both rows; a directed CSR is traversed along
 * its stored (outgoing) adjacencies.
 * Validation (unless BFS_TRUSTED): row_offsets[0] = 0, non-decreasing,
 * row_offsets[n] = nnz, every col_idx in [0, n). Adjacency order is not
 * required for correctness. Fails with BFS_ERR_FORMAT when violated.
 * 1 <= n < 2^31; nnz < 2^(64 - ceil(log2(n + 1))).
 */
int bfs_graph_create_csr(int64_t n, int64_t nnz, const void* row_offsets, int offset_bytes,
                         const int32_t* col_idx, uint32_t flags, bfs_graph_t** out);

/*
 * Hypersparse block in DCSC (section 4.1): nzc non-empty columns with ids
 * jc[0..nzc) strictly ascending, column pointers cp[0..nzc] (cp[0] = 0,
 * strictly increasing, cp[nzc] = nnz) and row ids ir[0..nnz), each in
 * [0, nrows). The entry A(r, k) != 0 means an edge from vertex k (column,
 * the frontier side) to vertex r (row, the output side).
 */
int bfs_graph_create_dcsc(int32_t nrows, int32_t ncols, int32_t nzc, int64_t nnz,
                          const int32_t* jc, const int32_t* cp, const int32_t* ir,
                          uint32_t flags, bfs_graph_t** out);

/* Releases a graph. BFS_ERR_BUSY while a server or batch still uses it. */
int bfs_graph_destroy(bfs_graph_t* g);

/* n (rows for a DCSC block), nnz and device bytes held by the handle. */
int bfs_graph_info(const bfs_graph_t* g, int64_t* n, int64_t* nnz, int64_t* device_bytes);

int bfs_graph_set_options(bfs_graph_t* g, const bfs_options_t* opt);
int bfs_graph_get_options(const bfs_graph_t* g, bfs_options_t* opt);

/* ---------------------------------------------------------------- BFS */

/*
 * BFS from `root` on a CSR graph (Algorithms 1 and 3). parent is required,
 * level may be NULL; both hold n int32 and may be device or host memory.
 * Synchronous: returns when the outputs are complete. The calling thread
 * waits for the device by polling the stream (for the lowest latency), so
 * it keeps one host core busy for the duration of the call; the same holds
 * for the host reads of the frontier size between batches of levels.
 */
int bfs_run(bfs_graph_t* g, int32_t root, int32_t* parent, int32_t* level);

/*
 * Same as bfs_run on `hip_stream`. The host still reads the frontier size
 * between batches of levels (so the call returns once the last level is
 * enqueued); with device outputs it does not wait for the final copies.
 * Device errors are reported by the next synchronising call on the handle.
 */
int bfs_run_async(bfs_graph_t* g, int32_t root, int32_t* parent, int32_t* level,
                  void* hip_stream);

/* Statistics of the last completed run (synchronises the handle's stream). */
int bfs_last_stats(bfs_graph_t* g, bfs_run_stats_t* st);

/* One level of the last profiled run. */
typedef struct bfs_level_info {
  int32_t level;        /* k: the level whose vertices this step discovered */
  int32_t mark;         /* 1 = mark-and-resolve, 2 = pull (by rows), 0 = atomicMin claims,
                           3 = atomicMin claims collected afterwards in vertex order (large
                               claim level),
                           4 = atomicMin claims inside the device level loop */
  int64_t frontier;     /* vertices of frontier k-1 that were expanded */
  int64_t edges;        /* their adjacencies */
  double expand_ms;     /* device time of the level's expand launches (claim, mark, pull) */
  double mark_ms;       /* the mark expand kernel's share of expand_ms (it also resolves the
                           previous push level's parents) */
  double finish_ms;     /* device time of its finish launch */
  double pull_ms;       /* the pull kernel's share of expand_ms */
  int64_t pull_candidates; /* pull levels: unvisited vertices of positive degree (searchers);
                              push mark levels: vertices whose parent was searched */
  int64_t pull_edges;   /* the adjacencies those searches examined */
  double small_ms;      /* on the first level of a run of the device level loop: that
                           launch's device time (its levels carry no time of their own) */
} bfs_level_info_t;

/*
 * Per-level record of the last run, for levels 1 .. min(capacity, 4095, the
 * level that found the frontier empty); *count receives the number written.
 * Frontier sizes and kinds are recorded always, device times only when the
 * run had options.profile = 1 (mode 1).
 */
int bfs_last_level_info(bfs_graph_t* g, bfs_level_info_t* out, int32_t capacity,
                        int32_t* count);

/*
 * Local product of one 2D share (Algorithm 3's SpMSV step, section 4.2):
 *   out[r] = min{ val(k) : k in frontier, A(r, k) != 0 },
 * emitted for every r whose set is non-empty, rows ascending. Entries of the
 * frontier on empty columns contribute nothing. No visited mask is applied
 * (the owner applies it, Algorithm 3). frontier->idx must be strictly
 * ascending and in [0, ncols) (BFS_ERR_ARG otherwise, checked on device;
 * out->idx/val are then left untouched). An empty frontier gives an empty
 * product without device work. When out->capacity is too small, returns
 * BFS_ERR_CAPACITY with the required size in out->nnz; out->idx/val then
 * hold unspecified values in their first capacity entries and nothing is
 * written past them. The block's accumulator (row bins, pair buffer of nnz
 * entries, sized at create) is reused by every call on the handle, so calls
 * on one handle must not overlap. Synchronous on `hip_stream` (reads the
 * output count back).
 */
int bfs_spmspv(bfs_graph_t* block, const bfs_svec_t* frontier, bfs_svec_t* out,
               void* hip_stream);

/*
 * BFS over a p_r x p_c grid of DCSC shares on one GPU: the 2D-partitioned
 * algorithm (Algorithm 3, section 3.2) with every share resident on the
 * device and its collectives replaced by device gathers. Per level the
 * sorted frontier is split by column block, bfs_spmspv runs on each share
 * (the frontier entries carry their global ids as values), the products of
 * a row block are folded with min into the rows not yet reached, and those
 * rows become the next frontier in ascending order.
 * shares[i * pc + j] is block (i, j) of the n x n adjacency matrix with
 * A(v, u) = 1 for each adjacency u -> v, in local ids: row block i covers
 * global rows [i*R, min((i+1)*R, n)) with R = ceil(n / pr), column block j
 * global columns
 * [j*C, min((j+1)*C, n)), C = ceil(n / pc). Every share must have that
 * shape (at least one row and column) and the handles must be distinct
 * (BFS_ERR_ARG otherwise). parent and level (nullable) are device arrays of
 * n entries, caller-owned, with bfs_run's meaning: parent = minimum-id
 * neighbour one level up. The shares' run locks are held for the call;
 * their workspace (the SpMSpV accumulators) is used. Synchronous on
 * `hip_stream` (the frontier size is read back every level); the call
 * allocates its own per-run workspace (about 24 n bytes) and frees it
 * before returning.
 */
int bfs_run_2d(bfs_graph_t* const* shares, int32_t pr, int32_t pc, int64_t n, int32_t root,
               int32_t* parent, int32_t* level, void* hip_stream);

/*
 * bfs_run_2d for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search and results as bfs_run_2d, with its per-run workspace taken from a
 * fixed device array inside the library (26 MiB per GPU, held until the
 * process ends) instead of hipMalloc, and its host read-backs into stack
 * memory instead of pinned buffers. It calls no allocator. Limits: n <=
 * 2^20, pc <= 256, pr * pc <= 1024 (BFS_ERR_CAPACITY / BFS_ERR_UNSUPPORTED
 * beyond them). Every call on one GPU uses that GPU's one array: calls that
 * overlap on the same GPU (other threads or streams) race and must be
 * serialised by the caller. The shares' own accumulators are used as in
 * bfs_run_2d. Synchronous on `hip_stream`.
 */
int bfs_run_2d_noalloc(bfs_graph_t* const* shares, int32_t pr, int32_t pc, int64_t n,
                       int32_t root, int32_t* parent, int32_t* level, void* hip_stream);

/* ---------------------------------------------------------------- batches */

/*
 * Runs `count` independent BFS queries (graphs[i], roots[i]): one persistent
 * launch of a multi-query kernel (one workgroup runs a query to completion,
 * per-query frontiers and level counters, largest estimated cost first)
 * takes the queries on graphs below 2^23 adjacencies or of average degree
 * below 8; queries on larger few-level graphs run one at a time through the
 * whole-GPU level kernels on a library-owned stream while that launch runs.
 * parents[i] (required) and levels[i] (may be NULL) are device arrays of
 * graphs[i]'s n and must not alias. Results equal those of bfs_run for each
 * query. BFS_UPPER graphs are rejected (BFS_ERR_UNSUPPORTED). Synchronous on
 * `hip_stream`.
 */
int bfs_run_batch(int32_t count, bfs_graph_t* const* graphs, const int32_t* roots,
                  int32_t* const* parents, int32_t* const* levels, void* hip_stream);

/* ---------------------------------------------------------------- server */

typedef struct bfs_server_config {
  int32_t slots;            /* queries in flight at most, in [1, 4096] */
  int64_t memory_budget;    /* device bytes for per-query frontier queues and bitmaps;
                               0 = min(25% of free memory, 16 GiB) */
  int32_t step_budget_us;   /* a device step stops advancing a query at the first level
                               boundary after this many microseconds (0 = 400) */
  int64_t large_query_nnz;  /* queries on graphs with at least this many adjacencies and an
                               average degree >= 8 (few levels) run one at a time across the
                               whole GPU on a second stream instead of in the multi-query
                               steps, where one workgroup per query would take far longer
                               (0 = 2^16, -1 = never) */
} bfs_server_config_t;

typedef struct bfs_result {
  int32_t status;         /* BFS_OK when done; BFS_ERR_BUSY while pending */
  int32_t depth;
  int64_t edges_traversed;
  double t_arrive;        /* seconds, host monotonic clock */
  double t_admit;
  double t_done;
} bfs_result_t;

/*
 * Continuous-batching server: queries are admitted while others run, as
 * slots and device memory free up, and every active query advances inside
 * the same device steps. parent/level are device arrays of the graph's n
 * and must stay valid until the ticket completes.
 */
int bfs_server_create(const bfs_server_config_t* cfg, bfs_server_t** out);
int bfs_server_submit(bfs_server_t* s, bfs_graph_t* g, int32_t root, int32_t* parent,
                      int32_t* level, uint64_t* ticket);
/* Non-blocking: fills *out; status BFS_ERR_BUSY while pending. */
int bfs_server_poll(bfs_server_t* s, uint64_t ticket, bfs_result_t* out);
/* Blocks until the ticket completes or timeout_s elapses (BFS_ERR_TIMEOUT). */
int bfs_server_wait(bfs_server_t* s, uint64_t ticket, double timeout_s, bfs_result_t* out);
/* Drives the server until every submitted query is done. */
int bfs_server_drain(bfs_server_t* s);
int bfs_server_destroy(bfs_server_t* s);

/* ---------------------------------------------------------------- tuning */

/*
 * Autotuner. CSR graph: times BFS from eight seeded roots of positive degree
 * (each root's fastest of five runs, summed) and tunes, by coordinate descent from the
 * defaults (two sweeps, a knob at a time), the expand grid (2, 4 workgroups
 * per CU), levels per host check (4, 8), the two mark-level floors together
 * (claim_min_frontier, claim_threshold: (4096, default), (1024, default),
 * (16384, default), (32, n / 512), (1024, n / 512), (4096, nnz / 16)),
 * pull_alpha (14, 4, 40) and the device level loop's frontier limit
 * (small_frontier: 8192, 1024, off); a value replaces the
 * current one only when it is more than 8% faster, and again against a fresh
 * timing of the current one, so repeated tuning keeps the same choice. The result is kept in the handle's options. DCSC share:
 * times both branches of the SpMSpV polyalgorithm (section 4.2: the binned
 * accumulator, or the sort-based merge) on sorted random frontiers of 64 to
 * 8192 entries and sets spmspv_sort_max to the largest size where the sort
 * was faster by the same margin (-1 if never). When cache_path is not NULL the choice is read from / appended to
 * that text file, one line per device name and graph shape. Results of later
 * runs do not depend on the choice, only their speed. Holds the handle's run
 * lock while timing.
 */
int bfs_tune(bfs_graph_t* g, const char* cache_path);

/* ---------------------------------------------------------------- misc */

const char* bfs_last_error(void);
/* Library version string. */
const char* bfs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BFS_MI355X_BFS_H */
