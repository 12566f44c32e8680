// Continuous-batching BFS server.
//
// A host worker thread owns a table of query slots on the device. Each
// iteration it (1) admits waiting queries in arrival order while a slot and
// enough device memory for the query's frontier queues and bitmap are free,
// (2) launches one step of the multi-query kernel over every active slot,
// where each workgroup advances its query level by level until the query
// finishes or a time budget expires at a level boundary, and (3) retires the
// queries that finished, freeing their slot and memory for the next
// arrivals. Queries that arrive while others run join at the next step, so
// their work overlaps on the device with the queries already in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bfs_multi.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Ticket {
  bfs_graph* g = nullptr;
  int32_t root = 0;
  int32_t* parent = nullptr;
  int32_t* level = nullptr;
  double t_arrive = 0, t_admit = 0, t_done = 0;
  int32_t status = BFS_ERR_BUSY;
  int32_t depth = 0;
  int64_t edges = 0;
  int slot = -1;
  int64_t ws_off = -1, ws_bytes = 0;
};

// First-fit allocator over one device arena (offsets, 256-byte granules).
struct Arena {
  std::map<int64_t, int64_t> free_;   // offset -> size
  void reset(int64_t bytes) {
    free_.clear();
    if (bytes > 0) free_[0] = bytes;
  }
  int64_t alloc(int64_t bytes) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct bfs_server {
  bfs_server_config_t cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_lane;
  std::thread worker;
  // whole-GPU lane for queries on large high-degree graphs
  std::thread lane;
  hipStream_t lane_stream = nullptr;
  std::deque<uint64_t> lane_q;
  int64_t large_nnz = 0;
  bool stop = false;
  int fatal = 0;
  uint64_t next_id = 1;
  std::unordered_map<uint64_t, Ticket> tickets;
  std::deque<uint64_t> waiting;
  std::vector<uint64_t> slot_ticket;
  int64_t in_flight = 0;
  // device tables
  bfsi::MQuery* d_qs = nullptr;
  bfsi::MQuery* h_qs = nullptr;
  int32_t* d_active = nullptr;
  int32_t* h_active = nullptr;
  char* d_arena = nullptr;
  int64_t arena_bytes = 0;
  Arena arena;
  unsigned long long budget_ticks = 0;

  void run();
  void run_lane();
  bool is_large(const bfs_graph* g) const {
    // upper-triangle graphs have no multi-query path: always the lane
    return g->csr.upper ||
           (large_nnz > 0 && g->csr.nnz >= large_nnz && g->csr.nnz >= 8 * g->csr.n);
  }
};

// Large queries one at a time across the whole GPU (the edge-balanced
// level kernels), on the lane's own stream, concurrently with the
// multi-query steps of the main worker.
void bfs_server::run_lane() {
  (void)hipSetDevice(device);
  for (;;) {
    std::unique_lock<std::mutex> lk(mu);
    cv_lane.wait(lk, [this] { return stop || !lane_q.empty(); });
    if (lane_q.empty()) {
      if (stop) break;
      continue;
    }
    const uint64_t id = lane_q.front();
    lane_q.pop_front();
    Ticket& t = tickets[id];
    t.t_admit = now_s();
    bfs_graph* g = t.g;
    const int32_t root = t.root;
    int32_t* parent = t.parent;
    int32_t* level = t.level;
    lk.unlock();
    bfs_run_stats_t st{};
    int rc;
    {
      std::lock_guard<std::mutex> gl(g->run_mu);
      rc = bfsi::csr_run(g, root, parent, level, lane_stream, true);
      if (rc == BFS_OK) rc = bfsi::csr_read_stats(g, &st);
    }
    const double t_done = now_s();
    lk.lock();
    t.status = rc;
    t.t_done = t_done;
    t.depth = st.depth;
    t.edges = st.edges_traversed;
    g->users.fetch_sub(1);
    --in_flight;
    cv_done.notify_all();
  }
}

void bfs_server::run() {
  (void)hipSetDevice(device);
  const int nslots = cfg.slots;
  std::vector<int> active;
  active.reserve((size_t)nslots);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      // admission: arrival order, a free slot and memory for the workspace
      while (!waiting.empty()) {
        Ticket& t = tickets[waiting.front()];
        int slot = -1;
        for (int i = 0; i < nslots; ++i)
          if (slot_ticket[(size_t)i] == 0) {
            slot = i;
            break;
          }
        if (slot < 0) break;
        const int64_t need = bfsi::multi_ws_bytes(t.g->csr.n);
        const int64_t off = arena.alloc(need);
        if (off < 0) break;
        t.slot = slot;
        t.ws_off = off;
        t.ws_bytes = need;
        t.t_admit = now_s();
        slot_ticket[(size_t)slot] = waiting.front();
        waiting.pop_front();
        bfsi::MQuery& q = h_qs[slot];
        std::memset(&q, 0, sizeof(q));
        char* w = d_arena + off;
        q.off = t.g->csr.off;
        q.col = t.g->csr.col;
        q.parent = t.parent;
        q.level = t.level;
        q.q[0] = reinterpret_cast<int32_t*>(w);
        q.q[1] = reinterpret_cast<int32_t*>(w + bfsi::multi_q_bytes(t.g->csr.n));
        q.vis = reinterpret_cast<uint32_t*>(w + 2 * bfsi::multi_q_bytes(t.g->csr.n));
        q.n = (int32_t)t.g->csr.n;
        q.root = t.root;
        q.status = bfsi::kQueryPending;
      }
      active.clear();
      for (int i = 0; i < nslots; ++i)
        if (slot_ticket[(size_t)i] != 0) active.push_back(i);
      if (active.empty()) {
        if (stop) break;
        cv_work.wait_for(lk, std::chrono::microseconds(200));
        continue;
      }
    }
    // one device step over every active slot
    const int hi = active.back() + 1;
    for (size_t i = 0; i < active.size(); ++i) h_active[i] = active[i];
    hipError_t e = hipMemcpyAsync(d_qs, h_qs, (size_t)hi * sizeof(bfsi::MQuery),
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_active, h_active, active.size() * 4, hipMemcpyHostToDevice, stream);
    int rc = BFS_OK;
    if (e == hipSuccess)
      rc = bfsi::multi_launch(d_qs, d_active, (int32_t)active.size(), nullptr,
                              (int)active.size(), false, budget_ticks, nullptr, 0, 0, stream);
    if (e == hipSuccess && rc == BFS_OK)
      e = hipMemcpyAsync(h_qs, d_qs, (size_t)hi * sizeof(bfsi::MQuery), hipMemcpyDeviceToHost,
                         stream);
    if (e == hipSuccess) e = bfsi::wait_stream(stream);
    const double t = now_s();
    std::unique_lock<std::mutex> lk(mu);
    if (e != hipSuccess || rc != BFS_OK) {
      // device failure: fail every in-flight and waiting ticket
      fatal = BFS_ERR_DEVICE;
      for (int s : active) {
        Ticket& tk = tickets[slot_ticket[(size_t)s]];
        tk.status = BFS_ERR_DEVICE;
        tk.t_done = t;
        tk.g->users.fetch_sub(1);
        --in_flight;
        slot_ticket[(size_t)s] = 0;
      }
      for (uint64_t id : waiting) {
        Ticket& tk = tickets[id];
        tk.status = BFS_ERR_DEVICE;
        tk.g->users.fetch_sub(1);
        --in_flight;
      }
      waiting.clear();
      cv_done.notify_all();
      if (stop) break;
      continue;
    }
    for (int s : active) {
      const bfsi::MQuery& q = h_qs[s];
      if (q.status != bfsi::kQueryDone) continue;
      const uint64_t id = slot_ticket[(size_t)s];
      Ticket& tk = tickets[id];
      tk.status = BFS_OK;
      tk.t_done = t;
      tk.depth = q.depth;
      tk.edges = (int64_t)q.edges;
      arena.release(tk.ws_off, tk.ws_bytes);
      tk.g->users.fetch_sub(1);
      --in_flight;
      slot_ticket[(size_t)s] = 0;
    }
    cv_done.notify_all();
  }
}

using namespace bfsi;

extern "C" {

int bfs_server_create(const bfs_server_config_t* cfg, bfs_server_t** out) {
  if (!cfg || !out) return fail(BFS_ERR_ARG, "NULL argument");
  *out = nullptr;
  if (cfg->slots < 1 || cfg->slots > 4096) return fail(BFS_ERR_ARG, "slots must be in [1, 4096]");
  if (cfg->memory_budget < 0 || cfg->step_budget_us < 0)
    return fail(BFS_ERR_ARG, "negative config value");
  try {
    bfs_server* s = new bfs_server();
    s->cfg = *cfg;
    (void)hipGetDevice(&s->device);
    auto bail = [&](int code) {
      (void)hipFree(s->d_qs);
      (void)hipFree(s->d_active);
      (void)hipFree(s->d_arena);
      if (s->h_qs) (void)hipHostFree(s->h_qs);
      if (s->h_active) (void)hipHostFree(s->h_active);
      if (s->stream) (void)hipStreamDestroy(s->stream);
      if (s->lane_stream) (void)hipStreamDestroy(s->lane_stream);
      delete s;
      return code;
    };
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->lane_stream, hipStreamNonBlocking);
    s->large_nnz = cfg->large_query_nnz == 0 ? ((int64_t)1 << 16) : cfg->large_query_nnz;
    const size_t nq = (size_t)cfg->slots;
    if (e == hipSuccess) e = hipMalloc(&s->d_qs, nq * sizeof(MQuery));
    if (e == hipSuccess) e = hipMalloc(&s->d_active, nq * 4);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_qs, nq * sizeof(MQuery), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_active, nq * 4, hipHostMallocDefault);
    if (e != hipSuccess) return bail(hip_fail(e, "server tables"));
    std::memset(s->h_qs, 0, nq * sizeof(MQuery));
    int64_t budget = cfg->memory_budget;
    if (budget == 0) {
      size_t fr = 0, tot = 0;
      (void)hipMemGetInfo(&fr, &tot);
      budget = std::min<int64_t>((int64_t)fr / 4, (int64_t)16 << 30);
    }
    budget = std::max<int64_t>(budget, 1 << 20) / 256 * 256;
    e = hipMalloc(&s->d_arena, (size_t)budget);
    if (e != hipSuccess) return bail(hip_fail(e, "server memory arena"));
    s->arena_bytes = budget;
    s->arena.reset(budget);
    s->slot_ticket.assign(nq, 0);
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, s->device) !=
            hipSuccess ||
        rate_khz <= 0)
      rate_khz = 100000;
    // time budget of one device step: step_budget_us microseconds (default 400)
    const int us = cfg->step_budget_us > 0 ? cfg->step_budget_us : 400;
    s->budget_ticks = (unsigned long long)rate_khz * (unsigned long long)us / 1000ull;
    if (!s->budget_ticks) s->budget_ticks = 1;
    s->worker = std::thread([s] { s->run(); });
    s->lane = std::thread([s] { s->run_lane(); });
    *out = s;
    return BFS_OK;
  } catch (...) {
    return fail(BFS_ERR_OOM, "exception in bfs_server_create");
  }
}

int bfs_server_submit(bfs_server_t* s, bfs_graph_t* g, int32_t root, int32_t* parent,
                      int32_t* level, uint64_t* ticket) {
  if (!s || !g || !parent || !ticket) return fail(BFS_ERR_ARG, "NULL argument");
  if (g->kind != kCsr) return fail(BFS_ERR_ARG, "server queries need a CSR graph");
  if (root < 0 || (int64_t)root >= g->csr.n) return fail(BFS_ERR_ARG, "root out of range");
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, parent) != hipSuccess ||
      !(a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged)) {
    (void)hipGetLastError();
    return fail(BFS_ERR_ARG, "server outputs must be device arrays");
  }
  if (level && (hipPointerGetAttributes(&a, level) != hipSuccess ||
                !(a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged))) {
    (void)hipGetLastError();
    return fail(BFS_ERR_ARG, "server outputs must be device arrays");
  }
  const bool large = s->is_large(g);
  if (!large && bfsi::multi_ws_bytes(g->csr.n) > s->arena_bytes)
    return fail(BFS_ERR_CAPACITY, "query workspace exceeds the server memory budget");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(BFS_ERR_BUSY, "server is shutting down");
  if (s->fatal) return fail(s->fatal, "server hit a device error");
  const uint64_t id = s->next_id++;
  Ticket& t = s->tickets[id];
  t.g = g;
  t.root = root;
  t.parent = parent;
  t.level = level;
  t.t_arrive = now_s();
  g->users.fetch_add(1);
  ++s->in_flight;
  if (large) {
    s->lane_q.push_back(id);
    s->cv_lane.notify_one();
  } else {
    s->waiting.push_back(id);
    s->cv_work.notify_one();
  }
  *ticket = id;
  return BFS_OK;
}

static void fill_result(const Ticket& t, bfs_result_t* out) {
  out->status = t.status;
  out->depth = t.depth;
  out->edges_traversed = t.edges;
  out->t_arrive = t.t_arrive;
  out->t_admit = t.t_admit;
  out->t_done = t.t_done;
}

int bfs_server_poll(bfs_server_t* s, uint64_t ticket, bfs_result_t* out) {
  if (!s || !out) return fail(BFS_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(BFS_ERR_ARG, "unknown ticket");
  fill_result(it->second, out);
  return BFS_OK;
}

int bfs_server_wait(bfs_server_t* s, uint64_t ticket, double timeout_s, bfs_result_t* out) {
  if (!s || !out) return fail(BFS_ERR_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(BFS_ERR_ARG, "unknown ticket");
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::duration<double>(std::max(timeout_s, 0.0));
  while (it->second.status == BFS_ERR_BUSY) {
    if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout &&
        it->second.status == BFS_ERR_BUSY) {
      fill_result(it->second, out);
      return fail(BFS_ERR_TIMEOUT, "ticket not done before the timeout");
    }
  }
  fill_result(it->second, out);
  return BFS_OK;
}

int bfs_server_drain(bfs_server_t* s) {
  if (!s) return fail(BFS_ERR_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_work.notify_one();
  s->cv_done.wait(lk, [s] { return s->in_flight == 0; });
  return s->fatal ? fail(s->fatal, "server hit a device error") : BFS_OK;
}

int bfs_server_destroy(bfs_server_t* s) {
  if (!s) return fail(BFS_ERR_ARG, "NULL argument");
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [s] { return s->in_flight == 0; });
    s->stop = true;
    s->cv_work.notify_all();
    s->cv_lane.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  if (s->lane.joinable()) s->lane.join();
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamSynchronize(s->lane_stream);
  (void)hipStreamDestroy(s->lane_stream);
  (void)hipFree(s->d_qs);
  (void)hipFree(s->d_active);
  (void)hipFree(s->d_arena);
  (void)hipHostFree(s->h_qs);
  (void)hipHostFree(s->h_active);
  (void)hipStreamDestroy(s->stream);
  delete s;
  return BFS_OK;
}

}  // extern "C"
