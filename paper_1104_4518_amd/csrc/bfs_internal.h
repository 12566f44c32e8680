// Internal declarations shared by the library's translation units: the
// graph handle, the per-run device state, wave64 helpers and the host-side
// launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bfs.h"

namespace bfsi {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// Waits for `s` by polling it (no blocking wait: a thread put to sleep by
// the runtime wakes tens of microseconds after the work ends, which would
// dominate calls that take microseconds). Returns the stream's error.
hipError_t wait_stream(hipStream_t s);

#define BFS_HIP(call)                                      \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return ::bfsi::hip_fail(e_, #call); \
  } while (0)

// ------------------------------------------------------------------ shapes
// Expand kernel: 256 threads (4 waves of 64) own a tile of kTile
// consecutive edges of the level's edge space.
constexpr int kBlock = 256;
constexpr int kItems = 4;
constexpr int kTile = kBlock * kItems;

enum GraphKind { kCsr = 1, kDcsc = 2 };

// Per-run device state of the CSR path. ctr[k % 3] packs the frontier
// produced by level k: (edge total << cbits) | vertex count.
struct LevelState {
  unsigned long long ctr[3];
  int32_t k_expand;   // level the next expand launch processes
  int32_t k_fold;     // level the next finish launch closes
  int32_t depth;      // largest level assigned
  int32_t levels;     // expand launches that found a non-empty frontier
  unsigned long long edges;    // sum of frontier edge totals
  unsigned long long reached;  // owners over the run (+1 for the root)
  unsigned long long frontier_total;  // sum of frontier sizes
  // vertices reached at level k with no outgoing adjacency (directed graphs):
  // not expanded, but still marked visited by fold(k)
  unsigned int zcnt[3];
  int32_t error;
  int32_t mark_levels;   // levels resolved by mark-and-resolve
  int32_t pull;          // the current level computes its product by rows (pull)
  int32_t pull_levels;   // levels computed by rows
  int32_t pad;
  unsigned long long pull_edges;   // adjacencies examined by the pull levels
  // current pull level: vertices found and their adjacencies (the next
  // level's input counter, known before finish)
  unsigned long long pull_found, pull_found_edges;
  int32_t qskip;   // the last finish built no queue (its successor pulls)
  // kind of the current and of the previous level: 0 claim (or empty),
  // 1 push mark level (its resolve runs in the next level's mark kernel),
  // 2 pull
  int32_t kind_cur, kind_prev;
  // launch groups of this run (each: the device level loop, then one level's
  // kernels), and the levels the device loop ran
  int32_t groups;
  int32_t small_levels;
  int32_t pad2;
  // input frontier counter of each level (profiling; levels < kLevelHist)
  unsigned long long hist[4096];
  int32_t hist_mark[4096];   // 0 claim, 1 mark-and-resolve, 2 pull
  // pull levels: vertices that searched, adjacencies they examined
  unsigned long long hist_pc[4096];
  unsigned long long hist_pe[4096];
  // per launch group t (< kLevelHist): the level its level kernels processed
  // (0 = none), and the first and last level its device loop ran
  int32_t grp_level[4096];
  int32_t grp_first[4096];
  int32_t grp_last[4096];
  // targets of the device level loop's atomics that must not change a word
  // (one per thread of its workgroup), so that every claim of a round is
  // issued unconditionally and the round waits once
  unsigned long long sink[1024];
};
constexpr int kLevelHist = 4096;

// What a captured level graph depends on besides the handle's own buffers.
struct GraphKey {
  long long mp_edges, mp_vertices;
  int mp_sym, probe;
  int grids[4];
  int mp_alpha, pad;
};

struct CsrDev {
  int64_t n = 0, nnz = 0;
  int cbits = 0;                 // bits of the packed counter holding the count
  int64_t* off = nullptr;        // n + 1
  int32_t* col = nullptr;        // nnz
  // workspace
  uint32_t* vis = nullptr;       // visited bitmap, ceil(n / 32) words
  unsigned long long* rpl = nullptr;   // n: (level << 32) | parent per level-kernel id
  int4* head = nullptr;          // symmetric: first 3 adjacencies and degree per vertex
  int64_t nwords = 0;
  int32_t* qv[2] = {nullptr, nullptr};   // frontier vertex ids
  int64_t* qo[2] = {nullptr, nullptr};   // row start off[v] of each entry
  int64_t* qe[2] = {nullptr, nullptr};   // exclusive edge prefix of each entry
  int32_t* zq = nullptr;         // reached vertices of out-degree 0 (per level)
  uint8_t* mark = nullptr;       // per-vertex touch marks (nwords * 32 bytes)
  int symmetric = 0;             // undirected with ascending adjacency (checked or asserted)
  // upper-triangle storage: each undirected edge once, in the row of its
  // smaller endpoint; the searched graph is its symmetric closure
  int upper = 0;
  uint32_t* fbits = nullptr;     // upper: frontier bitmaps of the two level parities
  // mark levels: hot prefix of the visited bitmap (words) and one slice of
  // newly touched hot bits per mark-path workgroup
  int hot_words = 0;
  int hot_slices = 0;
  uint32_t* hot_new = nullptr;
  uint32_t* prev_bits = nullptr;  // hot prefix's vertices one level up (resolve)

  int32_t* jstart = nullptr;     // first queue entry of each expand tile
  int64_t njstart = 0;
  LevelState* state = nullptr;
  // host staging for host-pointer outputs
  int32_t* tmp_parent = nullptr;
  int32_t* tmp_level = nullptr;
  // degree-ordered copy used by the level kernels (large graphs): new id =
  // rank of the vertex by descending degree; each row keeps its adjacencies
  // in ascending original id, mapped to new ids
  int relabeled = 0;
  int grid_expand = 0, grid_finish = 0;   // default grids on the handle's device
  int64_t n_active = 0;          // symmetric relabelled graphs: every vertex of positive
                                 // degree has a level-kernel id below this (else n)
  int64_t* roff = nullptr;       // n + 1, rows in new order
  int32_t* rcol = nullptr;       // nnz, new ids
  int32_t* rank = nullptr;       // original id -> new id
  int32_t* inv = nullptr;        // new id -> original id
  // graph mode (options.mode = 2): the captured level graph and its key
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;
  GraphKey gkey{};
};

struct DcscDev {
  int32_t nrows = 0, ncols = 0, nzc = 0;
  int64_t nnz = 0;
  int32_t* jc = nullptr;
  int32_t* cp = nullptr;
  int32_t* ir = nullptr;
  int aux_shift = 0;             // column bucket width = 2^aux_shift
  int64_t naux = 0;
  int32_t* aux = nullptr;        // aux[b] = first p with jc[p] >= b << aux_shift
  uint32_t* recs = nullptr;      // 16 words per bucket (see k_build_recs), or null
  // binned product: rows in bins of 2^18, bin b's products in
  // pairs[bin_start[b] .. bin_start[b + 1]) ((row in bin) << 32 | value)
  int32_t nbins = 0;
  int64_t* bin_start = nullptr;  // nbins + 1: stored entries in the bins before b
  int32_t* cursor = nullptr;     // products appended to each bin (zero between calls)
  unsigned long long* pairs = nullptr;   // nnz
  unsigned long long* chain = nullptr;   // chained-scan flag word per bin
  uint32_t* ticket = nullptr;    // bin tickets taken by all reductions so far (wraps)
  uint32_t ticket_base = 0;      // its value before the next reduction
  uint32_t* spa_val = nullptr;   // nrows, all 0xFFFFFFFF between calls (bins too large for LDS)
  uint32_t epoch = 0;            // calls of the binned path (flags carry it)
  int grid_bin = 0;              // workgroups of the binning kernel
  // [0] sort path's out count, [1] frontier error (the binned path writes
  // its epoch there), [2] sort path: product too large
  unsigned long long* counters = nullptr;
  // pinned host words: the sort path copies counters [0..2] there; the
  // binned path's reduction writes [0] count, [1] and [3] the error epochs,
  // [2] the epoch of the call it completed (device address h_counters_dev)
  unsigned long long* h_counters = nullptr;
  unsigned long long* h_counters_dev = nullptr;
};

}  // namespace bfsi

struct bfs_graph {
  int kind = 0;
  int device = 0;
  int64_t device_bytes = 0;
  bfs_options_t opt{};
  std::atomic<int> users{0};   // batch/server references
  bfsi::CsrDev csr;
  bfsi::DcscDev dcsc;
  hipStream_t last_stream = nullptr;
  unsigned long long* h_ctr = nullptr;   // pinned readback of one counter
  bfs_run_stats_t last{};
  int stats_valid = 0;
  // profiling (options.profile = 1): one event pair per expand launch
  std::vector<hipEvent_t> ev;
  int expand_launches = 0;
  int profiled = 0;
  // cost hints for ordering queries in batches (from earlier runs)
  int32_t hint_depth = 0;
  int64_t hint_edges = 0;
  // serialises runs that use the handle's own workspace (bfs_run, the
  // server's whole-GPU lane, bfs_tune)
  std::mutex run_mu;
};

namespace bfsi {

// ------------------------------------------------------------------ launchers
// bfs_csr.hip
int csr_alloc_workspace(bfs_graph* g);
int csr_widen(const int32_t* d_src32, int64_t n1, int64_t* d_dst, hipStream_t s);
void csr_free(bfs_graph* g);
int csr_validate(bfs_graph* g, hipStream_t s);
int csr_check_symmetric(bfs_graph* g, hipStream_t s, int* symmetric);
// Every adjacency v of row u has v > u, rows strictly ascending.
int csr_check_upper(bfs_graph* g, hipStream_t s, int* upper);
// Builds the degree-ordered copy from the host row offsets.
int csr_relabel(bfs_graph* g, const int64_t* host_off, hipStream_t s);
int csr_run(bfs_graph* g, int32_t root, int32_t* parent, int32_t* level, hipStream_t s,
            bool sync);
int csr_read_stats(bfs_graph* g, bfs_run_stats_t* st);
int csr_level_info(bfs_graph* g, bfs_level_info_t* out, int32_t capacity, int32_t* count);

// bfs_dcsc.hip
int dcsc_setup(bfs_graph* g, hipStream_t s, bool validate);
void dcsc_free(bfs_graph* g);
int dcsc_spmspv(bfs_graph* g, const bfs_svec_t* f, bfs_svec_t* out, hipStream_t s);

// ------------------------------------------------------------------ device helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __ballot(p); }

// number of set bits of `mask` below this lane
__device__ __forceinline__ int lanes_below(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ long long shfl_ll(long long v, int src) {
  const int lo = __shfl((int)(v & 0xFFFFFFFF), src, 64);
  const int hi = __shfl((int)(v >> 32), src, 64);
  return ((long long)hi << 32) | (unsigned int)lo;
}

__device__ __forceinline__ long long shfl_up_ll(long long v, int d) {
  const int lo = __shfl_up((int)(v & 0xFFFFFFFF), d, 64);
  const int hi = __shfl_up((int)(v >> 32), d, 64);
  return ((long long)hi << 32) | (unsigned int)lo;
}

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ long long wave_incl_scan(long long v) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const long long t = shfl_up_ll(v, d);
    if (l >= d) v += t;
  }
  return v;
}

}  // namespace bfsi
