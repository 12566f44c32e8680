// bfs_run_batch: many independent BFS queries in one launch of the
// multi-query kernel, and bfs_tune: picks launch shapes and level thresholds
// for a graph (or the SpMSpV branch switch for a DCSC share) by timing them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <numeric>
#include <sstream>
#include <unordered_set>
#include <string>
#include <utility>
#include <vector>

#include "bfs_multi.h"

namespace bfsi {
namespace {

// Device workspace shared by batch calls (grown on demand, kept until exit).
struct BatchPool {
  std::mutex mu;
  int device = -1;
  char* ws = nullptr;
  int64_t ws_bytes = 0;
  MQuery* d_qs = nullptr;
  int32_t* d_order = nullptr;
  int64_t q_cap = 0;
  int32_t* d_counter = nullptr;
  MQuery* h_qs = nullptr;
  int32_t* h_order = nullptr;
  hipStream_t lane = nullptr;   // queries run through the level kernels
  int lane_device = -1;
};

// Queries on graphs this large with an average degree of 8 or more (a few
// levels) run one at a time through the whole-GPU level kernels, beside the
// multi-query launch: one workgroup would take hundreds of times longer on
// them (R-MAT scale 22: ~0.4 ms across the GPU, ~400 ms in one workgroup).
constexpr int64_t kBatchLaneNnz = (int64_t)1 << 23;

bool batch_lane(const bfs_graph* g) {
  return g->csr.nnz >= kBatchLaneNnz && g->csr.nnz >= 8 * g->csr.n;
}

BatchPool& pool() {
  static BatchPool p;
  return p;
}

int grow(BatchPool& p, int64_t nq, int64_t ws_need) {
  if (nq > p.q_cap) {
    (void)hipFree(p.d_qs);
    (void)hipFree(p.d_order);
    if (p.h_qs) (void)hipHostFree(p.h_qs);
    if (p.h_order) (void)hipHostFree(p.h_order);
    p.d_qs = nullptr;
    p.d_order = nullptr;
    p.h_qs = nullptr;
    p.h_order = nullptr;
    p.q_cap = 0;
    const int64_t cap = std::max<int64_t>(nq, 1024);
    BFS_HIP(hipMalloc(&p.d_qs, (size_t)cap * sizeof(MQuery)));
    BFS_HIP(hipMalloc(&p.d_order, (size_t)cap * 4));
    BFS_HIP(hipHostMalloc(&p.h_qs, (size_t)cap * sizeof(MQuery), hipHostMallocDefault));
    BFS_HIP(hipHostMalloc(&p.h_order, (size_t)cap * 4, hipHostMallocDefault));
    p.q_cap = cap;
  }
  if (!p.d_counter) BFS_HIP(hipMalloc(&p.d_counter, 4));
  if (ws_need > p.ws_bytes) {
    (void)hipFree(p.ws);
    p.ws = nullptr;
    p.ws_bytes = 0;
    BFS_HIP(hipMalloc(&p.ws, (size_t)ws_need));
    p.ws_bytes = ws_need;
  }
  return BFS_OK;
}

bool device_ptr(const void* ptr) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Estimated cost of one query in ns: adjacency scans plus per-level latency.
double query_cost(const bfs_graph* g) {
  const double n = (double)g->csr.n, m = (double)g->csr.nnz;
  const double edges = g->hint_edges > 0 ? (double)g->hint_edges : m;
  double depth = (double)g->hint_depth;
  if (depth <= 0) depth = (m / std::max(n, 1.0) < 6.0) ? 2.0 * std::sqrt(n) : 16.0;
  return edges * 0.5 + depth * 4000.0;
}

// Launch shapes and level floors of a CSR graph, chosen by timing BFS from
// eight seeded roots of positive degree. Coordinate descent from the
// defaults: each knob in turn tries its values with the others fixed, each
// setting timed as the sum over the roots of each root's fastest of five
// runs, and a value replaces the current one only when it is faster by more
// than kTuneMargin, twice (the second time against a fresh timing of the
// current setting), so settings within timing noise of each other keep the
// earlier one and repeated tuning gives the same choice. Two sweeps over the
// knobs.
constexpr double kTuneMargin = 0.08;
constexpr int kTunePasses = 5;

int tune_csr(bfs_graph* g, const hipDeviceProp_t& prop, std::string* result) {
  const int64_t n = g->csr.n;
  int32_t *parent = nullptr, *level = nullptr;
  BFS_HIP(hipMalloc(&parent, (size_t)n * 4));
  BFS_HIP(hipMalloc(&level, (size_t)n * 4));
  std::vector<int64_t> off((size_t)std::min<int64_t>(n + 1, 1 << 22));
  const int64_t probe = (int64_t)off.size() - 1;
  BFS_HIP(hipMemcpy(off.data(), g->csr.off, off.size() * 8, hipMemcpyDeviceToHost));
  // roots like a user's: vertices of positive degree at seeded positions
  // (SplitMix64 of the attempt number), not the hubs, whose first levels
  // are unlike a typical root's
  std::vector<int32_t> cand;
  for (uint64_t i = 1; cand.size() < 8 && i <= 4096 && probe > 0; ++i) {
    uint64_t z = i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const int64_t v = (int64_t)(z % (uint64_t)probe);
    if (off[(size_t)v + 1] > off[(size_t)v]) cand.push_back((int32_t)v);
  }
  if (cand.empty()) cand.push_back(0);
  std::lock_guard<std::mutex> run_lk(g->run_mu);
  const bfs_options_t saved = g->opt;
  const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  // mark-level edge floor: the default (n / 64), or a sixteenth of the
  // adjacencies (graphs without hubs, where a push level's resolve scans far
  // for a small frontier's vertices)
  const int ct16 = (int)std::min<int64_t>(g->csr.nnz / 16, INT32_MAX);
  // or n / 512: a frontier of a few hubs (R-MAT's second level) pushed
  // without a claim per edge
  const int ct_low = (int)std::max<int64_t>(g->csr.n / 512, 4096);
  // a knob is a list of settings (values[0] the default); a setting gives
  // one or more options their values together
  using Field = int32_t bfs_options_t::*;
  using Setting = std::vector<std::pair<Field, int32_t>>;
  struct Knob {
    std::vector<Setting> values;
  };
  auto one = [](Field f, std::initializer_list<int32_t> vs) {
    Knob kb;
    for (int32_t v : vs) kb.values.push_back(Setting{{f, v}});
    return kb;
  };
  const Field cmf = &bfs_options_t::claim_min_frontier, cth = &bfs_options_t::claim_threshold;
  const std::vector<Knob> knobs = {
      one(&bfs_options_t::grid_blocks, {cus * 2, cus * 4}),
      one(&bfs_options_t::batch_levels, {4, 8}),
      // the two floors of mark-and-resolve act together (a frontier must
      // pass both), so they are tried in pairs
      Knob{{Setting{{cmf, 4096}, {cth, 0}}, Setting{{cmf, 1024}, {cth, 0}},
            Setting{{cmf, 16384}, {cth, 0}}, Setting{{cmf, 32}, {cth, ct_low}},
            Setting{{cmf, 1024}, {cth, ct_low}}, Setting{{cmf, 4096}, {cth, ct16}}}},
      one(&bfs_options_t::pull_alpha, {14, 4, 40}),
      one(&bfs_options_t::small_frontier, {8192, 1024, -1}),
  };
  auto apply = [](bfs_options_t& o, const Setting& st) {
    for (const auto& fv : st) o.*(fv.first) = fv.second;
  };
  auto holds = [](const bfs_options_t& o, const Setting& st) {
    for (const auto& fv : st)
      if (o.*(fv.first) != fv.second) return false;
    return true;
  };
  bfs_options_t cur = saved;
  for (const Knob& kb : knobs) apply(cur, kb.values[0]);
  int rc = BFS_OK;
  auto measure = [&](const bfs_options_t& o, double* out) -> int {
    g->opt = o;
    int r = csr_run(g, cand[0], parent, level, nullptr, true);   // warm
    if (r != BFS_OK) return r;
    // per root the fastest of the passes (timing noise only adds), summed
    std::vector<double> best_root(cand.size(), 1e30);
    for (int pass = 0; pass < kTunePasses; ++pass) {
      for (size_t i = 0; i < cand.size(); ++i) {
        const auto t0 = std::chrono::steady_clock::now();
        r = csr_run(g, cand[i], parent, level, nullptr, true);
        if (r != BFS_OK) return r;
        const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        best_root[i] = std::min(best_root[i], dt);
      }
    }
    *out = std::accumulate(best_root.begin(), best_root.end(), 0.0);
    return BFS_OK;
  };
  double best = 0.0;
  rc = measure(cur, &best);
  for (int sweep = 0; sweep < 2 && rc == BFS_OK; ++sweep) {
    for (const Knob& kb : knobs) {
      for (const Setting& v : kb.values) {
        if (holds(cur, v)) continue;
        bfs_options_t o = cur;
        apply(o, v);
        double t = 0.0;
        rc = measure(o, &t);
        if (rc != BFS_OK) break;
        if (t < best * (1.0 - kTuneMargin)) {
          // confirm against a fresh timing of the current setting, so one
          // slow measurement of it does not decide the choice
          double tc = 0.0, to = 0.0;
          rc = measure(cur, &tc);
          if (rc == BFS_OK) rc = measure(o, &to);
          if (rc != BFS_OK) break;
          if (to < tc * (1.0 - kTuneMargin)) {
            best = to;
            cur = o;
          } else {
            best = tc;
          }
        }
      }
      if (rc != BFS_OK) break;
    }
  }
  (void)hipFree(parent);
  (void)hipFree(level);
  g->opt = saved;
  if (rc != BFS_OK) return rc;
  for (const Knob& kb : knobs) apply(g->opt, [&] {
      Setting st = kb.values[0];
      for (auto& fv : st) fv.second = cur.*(fv.first);
      return st;
    }());
  std::ostringstream o;
  o << "grid=" << cur.grid_blocks << " batch=" << cur.batch_levels
    << " min_frontier=" << cur.claim_min_frontier << " pull_alpha=" << cur.pull_alpha
    << " claim_threshold=" << cur.claim_threshold << " small_frontier=" << cur.small_frontier;
  *result = o.str();
  return BFS_OK;
}

// The SpMSpV polyalgorithm's switch for a DCSC share: for frontiers of 64 to
// 8192 sorted random column ids, time the sort path and the accumulator; the
// sort path is kept up to the largest size where it was faster (-1 = never).
int tune_dcsc(bfs_graph* g, std::string* result) {
  const DcscDev& d = g->dcsc;
  const int sizes[] = {64, 512, 2048, 8192};
  const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(d.nrows, d.nnz));
  int32_t *f = nullptr, *oi = nullptr, *ov = nullptr;
  BFS_HIP(hipMalloc(&f, 8192 * 4));
  BFS_HIP(hipMalloc(&oi, (size_t)cap * 4));
  BFS_HIP(hipMalloc(&ov, (size_t)cap * 4));
  std::lock_guard<std::mutex> run_lk(g->run_mu);
  const bfs_options_t saved = g->opt;
  uint64_t x = 0x9E3779B97F4A7C15ull;   // fixed seed: a repeatable choice
  int chosen = -1;
  int rc = BFS_OK;
  for (int sz : sizes) {
    const int k = (int)std::min<int64_t>(sz, d.ncols);
    if (k <= 0) break;
    std::vector<int32_t> h;
    std::unordered_set<int32_t> seen;
    while ((int)h.size() < k) {
      x ^= x << 13;   // xorshift64
      x ^= x >> 7;
      x ^= x << 17;
      const int32_t c = (int32_t)(x % (uint64_t)d.ncols);
      if (seen.insert(c).second) h.push_back(c);
    }
    std::sort(h.begin(), h.end());
    BFS_HIP(hipMemcpy(f, h.data(), h.size() * 4, hipMemcpyHostToDevice));
    double t[2] = {0, 0};
    for (int path = 0; path < 2 && rc == BFS_OK; ++path) {
      g->opt.spmspv_sort_max = path ? 8192 : -1;
      bfs_svec_t fv{k, k, f, nullptr}, out{0, cap, oi, ov};
      rc = dcsc_spmspv(g, &fv, &out, nullptr);   // warm
      const auto t0 = std::chrono::steady_clock::now();
      for (int rep = 0; rep < 5 && rc == BFS_OK; ++rep) {
        out.nnz = 0;
        rc = dcsc_spmspv(g, &fv, &out, nullptr);
      }
      t[path] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (rc != BFS_OK) break;
    if (t[1] < t[0] * (1.0 - kTuneMargin)) chosen = k;
  }
  (void)hipFree(f);
  (void)hipFree(oi);
  (void)hipFree(ov);
  g->opt = saved;
  if (rc != BFS_OK) return rc;
  g->opt.spmspv_sort_max = chosen;
  *result = "sort_max=" + std::to_string(chosen);
  return BFS_OK;
}

}  // namespace
}  // namespace bfsi

using namespace bfsi;

extern "C" {

int bfs_run_batch(int32_t count, bfs_graph_t* const* graphs, const int32_t* roots,
                  int32_t* const* parents, int32_t* const* levels, void* hip_stream) {
  try {
    if (count < 0) return fail(BFS_ERR_ARG, "count must be >= 0");
    if (count == 0) return BFS_OK;
    if (!graphs || !roots || !parents) return fail(BFS_ERR_ARG, "NULL argument array");
    std::unordered_set<const void*> outs;
    for (int32_t i = 0; i < count; ++i) {
      const bfs_graph* g = graphs[i];
      if (!g || g->kind != kCsr) return fail(BFS_ERR_ARG, "batch query needs a CSR graph");
      if (g->csr.upper)
        return fail(BFS_ERR_UNSUPPORTED, "batch queries need full CSR graphs (not BFS_UPPER)");
      if (roots[i] < 0 || (int64_t)roots[i] >= g->csr.n)
        return fail(BFS_ERR_ARG, "root out of range in batch");
      if (!parents[i] || !device_ptr(parents[i]))
        return fail(BFS_ERR_ARG, "batch parents must be device arrays");
      if (!outs.insert(parents[i]).second) return fail(BFS_ERR_ARG, "batch outputs must not alias");
      if (levels && levels[i]) {
        if (!device_ptr(levels[i])) return fail(BFS_ERR_ARG, "batch levels must be device arrays");
        if (!outs.insert(levels[i]).second)
          return fail(BFS_ERR_ARG, "batch outputs must not alias");
      }
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    BatchPool& p = pool();
    std::lock_guard<std::mutex> lk(p.mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::vector<int32_t> multi, lane;
    int64_t nmax = 1;
    for (int32_t i = 0; i < count; ++i) {
      if (batch_lane(graphs[i])) {
        lane.push_back(i);
      } else {
        multi.push_back(i);
        nmax = std::max<int64_t>(nmax, graphs[i]->csr.n);
      }
    }
    const int32_t nm = (int32_t)multi.size();
    int rc = BFS_OK;
    if (nm > 0) {
      // workgroups: co-resident capacity, bounded by the queries and by a
      // quarter of free memory for their workspaces
      const int64_t ws_one = multi_ws_bytes(nmax);
      size_t free_b = 0, total_b = 0;
      (void)hipMemGetInfo(&free_b, &total_b);
      int64_t grid = std::min<int64_t>(nm, multi_grid(dev));
      const int64_t mem_cap = std::max<int64_t>(1, (int64_t)(free_b + p.ws_bytes) / 4 / ws_one);
      grid = std::max<int64_t>(1, std::min(grid, mem_cap));
      rc = grow(p, nm, grid * ws_one);
      if (rc != BFS_OK) return rc;
      std::vector<std::pair<double, int32_t>> cost((size_t)nm);
      for (int32_t j = 0; j < nm; ++j) {
        const int32_t i = multi[(size_t)j];
        const bfs_graph* g = graphs[i];
        MQuery& q = p.h_qs[j];
        std::memset(&q, 0, sizeof(q));
        q.off = g->csr.off;
        q.col = g->csr.col;
        q.parent = parents[i];
        q.level = levels ? levels[i] : nullptr;
        q.n = (int32_t)g->csr.n;
        q.root = roots[i];
        q.status = kQueryPending;
        cost[(size_t)j] = {query_cost(g), j};
      }
      std::stable_sort(cost.begin(), cost.end(),
                       [](const auto& a, const auto& b) { return a.first > b.first; });
      for (int32_t j = 0; j < nm; ++j) p.h_order[j] = cost[(size_t)j].second;
      BFS_HIP(hipMemcpyAsync(p.d_qs, p.h_qs, (size_t)nm * sizeof(MQuery),
                             hipMemcpyHostToDevice, s));
      BFS_HIP(hipMemcpyAsync(p.d_order, p.h_order, (size_t)nm * 4, hipMemcpyHostToDevice, s));
      rc = multi_reset_counter(p.d_counter, s);
      if (rc != BFS_OK) return rc;
      rc = multi_launch(p.d_qs, p.d_order, nm, p.d_counter, (int)grid, true, 0ull, p.ws, ws_one,
                        multi_q_bytes(nmax), s);
      if (rc != BFS_OK) return rc;
      BFS_HIP(hipMemcpyAsync(p.h_qs, p.d_qs, (size_t)nm * sizeof(MQuery),
                             hipMemcpyDeviceToHost, s));
    }
    // the large queries, one at a time on the lane stream, while the
    // multi-query launch runs
    if (!lane.empty()) {
      if (!p.lane || p.lane_device != dev) {
        if (p.lane) (void)hipStreamDestroy(p.lane);
        p.lane = nullptr;
        BFS_HIP(hipStreamCreateWithFlags(&p.lane, hipStreamNonBlocking));
        p.lane_device = dev;
      }
      for (int32_t i : lane) {
        bfs_graph* g = graphs[i];
        std::lock_guard<std::mutex> gl(g->run_mu);
        rc = csr_run(g, roots[i], parents[i], levels ? levels[i] : nullptr, p.lane, true);
        if (rc != BFS_OK) return rc;
      }
    }
    if (nm > 0) {
      BFS_HIP(wait_stream(s));
      for (int32_t j = 0; j < nm; ++j) {
        const MQuery& q = p.h_qs[j];
        if (q.status != kQueryDone) return fail(BFS_ERR_DEVICE, "batch query did not complete");
        bfs_graph* g = graphs[multi[(size_t)j]];
        g->hint_depth = std::max(g->hint_depth, q.depth);
        g->hint_edges = std::max<int64_t>(g->hint_edges, (int64_t)q.edges);
      }
    }
    return BFS_OK;
  } catch (...) {
    return fail(BFS_ERR_DEVICE, "exception in bfs_run_batch");
  }
}

int bfs_tune(bfs_graph_t* g, const char* cache_path) {
  if (!g) return fail(BFS_ERR_ARG, "NULL graph");
  try {
    hipDeviceProp_t prop;
    int dev = 0;
    (void)hipGetDevice(&dev);
    BFS_HIP(hipGetDeviceProperties(&prop, dev));
    std::ostringstream key;
    if (g->kind == kCsr)
      key << prop.gcnArchName << " csr n=" << g->csr.n << " nnz=" << g->csr.nnz;
    else
      key << prop.gcnArchName << " dcsc " << g->dcsc.nrows << "x" << g->dcsc.ncols
          << " nnz=" << g->dcsc.nnz;
    if (cache_path) {
      std::ifstream in(cache_path);
      std::string line;
      while (std::getline(in, line)) {
        const size_t bar = line.find(" | ");
        if (bar == std::string::npos || line.substr(0, bar) != key.str()) continue;
        const char* rest = line.c_str() + bar + 3;
        int grid = 0, batch = 0, minf = 0, alpha = 0, ct = -1, small = 0, sort_max = 0;
        if (g->kind == kCsr &&
            std::sscanf(rest,
                        "grid=%d batch=%d min_frontier=%d pull_alpha=%d claim_threshold=%d "
                        "small_frontier=%d",
                        &grid, &batch, &minf, &alpha, &ct, &small) == 6 &&
            grid > 0 && batch > 0 && minf > 0 && (alpha > 0 || alpha == -1) && ct >= 0 &&
            (small > 0 || small == -1)) {
          g->opt.grid_blocks = grid;
          g->opt.batch_levels = batch;
          g->opt.claim_min_frontier = minf;
          g->opt.pull_alpha = alpha;
          g->opt.claim_threshold = ct;
          g->opt.small_frontier = small;
          return BFS_OK;
        }
        if (g->kind == kDcsc && std::sscanf(rest, "sort_max=%d", &sort_max) == 1 &&
            (sort_max == -1 || sort_max > 0)) {
          g->opt.spmspv_sort_max = sort_max;
          return BFS_OK;
        }
      }
    }
    std::string result;
    const int rc = g->kind == kCsr ? tune_csr(g, prop, &result) : tune_dcsc(g, &result);
    if (rc != BFS_OK) return rc;
    if (cache_path) {
      std::ofstream out(cache_path, std::ios::app);
      out << key.str() << " | " << result << "\n";
    }
    return BFS_OK;
  } catch (...) {
    return fail(BFS_ERR_DEVICE, "exception in bfs_tune");
  }
}

}  // extern "C"
