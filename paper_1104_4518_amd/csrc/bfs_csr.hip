// Level-synchronous BFS on a CSR graph (Algorithm 1's level structure with
// one synchronisation per level, section 2.2; each level is the masked
// (select, min) product of section 3.2 evaluated by pushing the frontier's
// adjacencies).
//
// One level k is two launches:
//   expand(k)  streams the adjacencies of frontier k-1 in edge-balanced
//              tiles, tests the visited bitmap (levels < k), claims
//              unvisited vertices with atomicMin on parent[] (the semiring's
//              min: the smallest frontier id wins), and appends each vertex
//              whose claim turned parent from -1 into a frontier vertex to
//              the next queue, with its row start and an exclusive prefix of
//              degrees, so the next level can split work by edges.
//   fold(k)    sets the visited bits of frontier k (the complement mask of
//              section 3.2 is the dense visited set) and maps every edge
//              tile of level k+1 to its first queue entry.
//
// Every launch reads the level number and the frontier counters from device
// memory, so consecutive launches have identical arguments and a level whose
// input frontier is empty exits at once: the host enqueues several levels
// between reads of the frontier size.
#include "bfs_internal.h"

#include <algorithm>

namespace bfsi {
namespace {

struct Queues {
  int32_t* qv[2];
  int64_t* qo[2];
  int64_t* qe[2];
};

__global__ void k_init(int64_t n, int32_t* __restrict__ parent, int32_t* __restrict__ level,
                       uint32_t* __restrict__ vis, int64_t nwords) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = i; v < n; v += stride) {
    parent[v] = -1;
    if (level) level[v] = -1;
  }
  for (int64_t w = i; w < nwords; w += stride) vis[w] = 0u;
}

__global__ void k_seed(const int64_t* __restrict__ off, int32_t root, int32_t* parent,
                       int32_t* level, Queues q, LevelState* st, int cbits) {
  parent[root] = root;
  if (level) level[root] = 0;
  const int64_t o = off[root];
  const int64_t d = off[root + 1] - o;
  q.qv[0][0] = root;
  q.qo[0][0] = o;
  q.qe[0][0] = 0;
  st->ctr[0] = d > 0 ? (((unsigned long long)d << cbits) | 1ull) : 0ull;
  st->ctr[1] = 0ull;
  st->ctr[2] = 0ull;
  st->k_expand = 1;
  st->k_fold = 0;
  st->depth = 0;
  st->levels = 0;
  st->edges = 0ull;
  st->reached = 1ull;
  st->frontier_total = 0ull;
  st->zcnt[0] = st->zcnt[1] = st->zcnt[2] = 0u;
  st->error = 0;
}

template <int TILE>
__global__ void k_fold(Queues q, LevelState* st, uint32_t* __restrict__ vis,
                       int32_t* __restrict__ jstart, const int32_t* __restrict__ zq, int cbits) {
  const int k = st->k_fold;
  const unsigned long long c = st->ctr[k % 3];
  const int64_t F = (int64_t)(c & ((1ull << cbits) - 1));
  const int64_t T = (int64_t)(c >> cbits);
  const int64_t Z = (int64_t)st->zcnt[k % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->k_expand = k + 1;
    if (F > 0) {
      st->edges += (unsigned long long)T;
      st->frontier_total += (unsigned long long)F;
    }
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < Z; j += stride) {
    const int32_t v = zq[j];
    atomicOr(&vis[v >> 5], 1u << (v & 31));
  }
  if (F == 0) return;
  const int32_t* __restrict__ qv = q.qv[k & 1];
  const int64_t* __restrict__ qe = q.qe[k & 1];
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < F; j += stride) {
    const int32_t v = qv[j];
    atomicOr(&vis[v >> 5], 1u << (v & 31));
    const int64_t lo = qe[j];
    const int64_t hi = (j + 1 < F) ? qe[j + 1] : T;
    for (int64_t w = (lo + TILE - 1) / TILE; w * TILE < hi; ++w) jstart[w] = (int32_t)j;
  }
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_expand(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const uint32_t* __restrict__ vis, int32_t* __restrict__ parent, int32_t* __restrict__ level,
    Queues q, const int32_t* __restrict__ jstart, int32_t* __restrict__ zq, LevelState* st,
    int cbits) {
  constexpr int TILE = BLOCK * ITEMS;
  constexpr int WAVES = BLOCK / 64;
  __shared__ long long s_qe[TILE + 1];
  __shared__ int32_t s_ov[TILE];
  __shared__ int32_t s_od[TILE];
  __shared__ long long s_oo[TILE];
  __shared__ long long s_wsum[WAVES];
  __shared__ unsigned long long s_base;
  __shared__ int s_cnt;

  const int k = st->k_expand;
  const int kin = k - 1;
  const unsigned long long cmask = (1ull << cbits) - 1;
  const unsigned long long cin = st->ctr[kin % 3];
  const int64_t F = (int64_t)(cin & cmask);
  const int64_t T = (int64_t)(cin >> cbits);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->ctr[(k + 1) % 3] = 0ull;   // output counters of level k + 1
    st->zcnt[(k + 1) % 3] = 0u;
    st->k_fold = k;
    if (F > 0) st->levels = k;
  }
  if (F == 0) return;

  const int64_t nitems = (T + TILE - 1) / TILE;
  const int32_t* __restrict__ qv_in = q.qv[kin & 1];
  const int64_t* __restrict__ qo_in = q.qo[kin & 1];
  const int64_t* __restrict__ qe_in = q.qe[kin & 1];
  int32_t* __restrict__ qv_out = q.qv[k & 1];
  int64_t* __restrict__ qo_out = q.qo[k & 1];
  int64_t* __restrict__ qe_out = q.qe[k & 1];
  unsigned long long* ctr_out = &st->ctr[k % 3];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;
  unsigned int my_reached = 0;

  for (int64_t w = blockIdx.x; w < nitems; w += gridDim.x) {
    const int64_t e0 = w * TILE;
    const int64_t e1 = min(e0 + (int64_t)TILE, T);
    const int32_t j0 = jstart[w];
    const int32_t j1 = (w + 1 < nitems) ? jstart[w + 1] : (int32_t)(F - 1);
    const int R = j1 - j0 + 1;
    for (int r = tid; r < R; r += BLOCK) s_qe[r] = qe_in[j0 + r];
    if (tid == 0) s_cnt = 0;
    __syncthreads();

#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int64_t e = e0 + (int64_t)i * BLOCK + tid;
      bool own = false;
      int32_t v = 0;
      if (e < e1) {
        // row of edge e: last r with s_qe[r] <= e (rows are non-empty)
        int lo = 0, hi = R - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_qe[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const int64_t j = j0 + lo;
        const uint32_t u = (uint32_t)qv_in[j];
        v = col[qo_in[j] + (e - s_qe[lo])];
        if (!((vis[v >> 5] >> (v & 31)) & 1u)) {
          const uint32_t cur = reinterpret_cast<const uint32_t*>(parent)[v];
          if (cur > u) {
            const uint32_t old = atomicMin(reinterpret_cast<uint32_t*>(parent) + v, u);
            own = (old == 0xFFFFFFFFu);
          }
        }
      }
      int64_t vo = 0;
      int32_t deg = 0;
      if (own) {
        if (level) level[v] = k;
        vo = off[v];
        deg = (int32_t)(off[v + 1] - vo);
        ++my_reached;
      }
      const bool enq = own && deg > 0;
      const unsigned long long m = wave_ballot(enq);
      if (m) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&s_cnt, __popcll(m));
        base = __shfl(base, 0, 64);
        if (enq) {
          const int p = base + lanes_below(m);
          s_ov[p] = v;
          s_od[p] = deg;
          s_oo[p] = vo;
        }
      }
      // reached but nothing to expand (out-degree 0): fold(k) marks it visited
      const unsigned long long mz = wave_ballot(own && deg == 0);
      if (mz) {
        unsigned int base = 0;
        if (lane == 0) base = atomicAdd(&st->zcnt[k % 3], (unsigned int)__popcll(mz));
        base = __shfl(base, 0, 64);
        if (own && deg == 0) zq[base + lanes_below(mz)] = v;
      }
    }
    __syncthreads();

    // one global append per tile: slots and edge range in a single atomic
    const int C = s_cnt;
    if (C > 0) {
      long long local = 0;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int p = tid * ITEMS + i;
        if (p < C) local += s_od[p];
      }
      const long long incl = wave_incl_scan(local);
      if (lane == 63) s_wsum[wid] = incl;
      __syncthreads();
      long long wbase = 0, total = 0;
#pragma unroll
      for (int x = 0; x < WAVES; ++x) {
        const long long sx = s_wsum[x];
        if (x < wid) wbase += sx;
        total += sx;
      }
      if (tid == 0)
        s_base = atomicAdd(ctr_out, ((unsigned long long)total << cbits) | (unsigned long long)C);
      __syncthreads();
      const unsigned long long b = s_base;
      const int64_t bc = (int64_t)(b & cmask);
      long long run = (long long)(b >> cbits) + wbase + incl - local;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int p = tid * ITEMS + i;
        if (p < C) {
          qv_out[bc + p] = s_ov[p];
          qo_out[bc + p] = s_oo[p];
          qe_out[bc + p] = run;
          run += s_od[p];
        }
      }
    }
    __syncthreads();
  }

  // per-block totals
  unsigned int r = my_reached;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) r += __shfl_xor(r, d, 64);
  __shared__ unsigned int s_red[WAVES];
  if (lane == 0) s_red[wid] = r;
  __syncthreads();
  if (tid == 0) {
    unsigned int t = 0;
    for (int x = 0; x < WAVES; ++x) t += s_red[x];
    if (t) {
      atomicAdd(&st->reached, (unsigned long long)t);
      atomicMax(&st->depth, k);
    }
  }
}

int grid_for(int device, const void* kernel, int block, int cap_per_cu) {
  static int cus[64] = {0};
  if (device < 0 || device >= 64) device = 0;
  if (!cus[device]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        v <= 0)
      v = 256;
    cus[device] = v;
  }
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, 0) != hipSuccess ||
      occ <= 0)
    occ = 4;
  occ = std::min(occ, cap_per_cu);
  return cus[device] * occ;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

__global__ void k_validate_csr(int64_t n, int64_t nnz, const int64_t* __restrict__ off,
                               const int32_t* __restrict__ col, int32_t* err) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = i; v < n; v += stride)
    if (off[v + 1] < off[v]) atomicOr(err, 1);
  if (i == 0 && (off[0] != 0 || off[n] != nnz)) atomicOr(err, 2);
  for (int64_t e = i; e < nnz; e += stride) {
    const int32_t c = col[e];
    if (c < 0 || (int64_t)c >= n) atomicOr(err, 4);
  }
}

__global__ void k_widen_offsets(int64_t n1, const int32_t* __restrict__ src,
                                int64_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n1; i += stride)
    dst[i] = (int64_t)src[i];
}

}  // namespace

int csr_alloc_workspace(bfs_graph* g) {
  CsrDev& c = g->csr;
  c.nwords = (c.n + 31) / 32;
  c.njstart = c.nnz / kTile + 2;
  BFS_HIP(hipMalloc(&c.vis, (size_t)std::max<int64_t>(c.nwords, 1) * 4));
  for (int b = 0; b < 2; ++b) {
    BFS_HIP(hipMalloc(&c.qv[b], (size_t)c.n * 4));
    BFS_HIP(hipMalloc(&c.qo[b], (size_t)c.n * 8));
    BFS_HIP(hipMalloc(&c.qe[b], (size_t)c.n * 8));
  }
  BFS_HIP(hipMalloc(&c.jstart, (size_t)c.njstart * 4));
  BFS_HIP(hipMalloc(&c.zq, (size_t)c.n * 4));
  BFS_HIP(hipMalloc(&c.state, sizeof(LevelState)));
  BFS_HIP(hipMemset(c.state, 0, sizeof(LevelState)));
  g->device_bytes += std::max<int64_t>(c.nwords, 1) * 4 + 2 * c.n * 20 + c.njstart * 4 +
                     (int64_t)sizeof(LevelState);
  return BFS_OK;
}

void csr_free(bfs_graph* g) {
  CsrDev& c = g->csr;
  (void)hipFree(c.off);
  (void)hipFree(c.col);
  (void)hipFree(c.vis);
  for (int b = 0; b < 2; ++b) {
    (void)hipFree(c.qv[b]);
    (void)hipFree(c.qo[b]);
    (void)hipFree(c.qe[b]);
  }
  (void)hipFree(c.jstart);
  (void)hipFree(c.zq);
  (void)hipFree(c.state);
  (void)hipFree(c.tmp_parent);
  (void)hipFree(c.tmp_level);
  c = CsrDev{};
}

int csr_widen(const int32_t* d_src32, int64_t n1, int64_t* d_dst, hipStream_t s) {
  k_widen_offsets<<<1024, 256, 0, s>>>(n1, d_src32, d_dst);
  BFS_HIP(hipGetLastError());
  return BFS_OK;
}

int csr_validate(bfs_graph* g, hipStream_t s) {
  CsrDev& c = g->csr;
  int32_t* d_err = nullptr;
  BFS_HIP(hipMalloc(&d_err, 4));
  BFS_HIP(hipMemsetAsync(d_err, 0, 4, s));
  k_validate_csr<<<2048, 256, 0, s>>>(c.n, c.nnz, c.off, c.col, d_err);
  int32_t h = 0;
  hipError_t e = hipMemcpyAsync(&h, d_err, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_err);
  if (e != hipSuccess) return hip_fail(e, "csr validation");
  if (h & 2) return fail(BFS_ERR_FORMAT, "CSR row offsets must start at 0 and end at nnz");
  if (h & 1) return fail(BFS_ERR_FORMAT, "CSR row offsets must be non-decreasing");
  if (h & 4) return fail(BFS_ERR_FORMAT, "CSR column index out of [0, n)");
  return BFS_OK;
}

int csr_run(bfs_graph* g, int32_t root, int32_t* parent, int32_t* level, hipStream_t s,
            bool sync) {
  CsrDev& c = g->csr;
  if (root < 0 || (int64_t)root >= c.n) return fail(BFS_ERR_ARG, "root out of range");
  if (!parent) return fail(BFS_ERR_ARG, "parent output is required");

  int32_t* d_parent = parent;
  int32_t* d_level = level;
  const bool host_parent = !is_device_ptr(parent);
  const bool host_level = level && !is_device_ptr(level);
  if (host_parent) {
    if (!c.tmp_parent) BFS_HIP(hipMalloc(&c.tmp_parent, (size_t)c.n * 4));
    d_parent = c.tmp_parent;
  }
  if (host_level) {
    if (!c.tmp_level) BFS_HIP(hipMalloc(&c.tmp_level, (size_t)c.n * 4));
    d_level = c.tmp_level;
  }

  Queues q;
  for (int b = 0; b < 2; ++b) {
    q.qv[b] = c.qv[b];
    q.qo[b] = c.qo[b];
    q.qe[b] = c.qe[b];
  }
  const int ib = 256;
  const int igrid = (int)std::min<int64_t>((std::max(c.n, c.nwords) + ib - 1) / ib, 8192);
  if (g->opt.profile > 0) {
    while (g->ev.size() < 2) {
      hipEvent_t ev;
      BFS_HIP(hipEventCreate(&ev));
      g->ev.push_back(ev);
    }
    BFS_HIP(hipEventRecord(g->ev[0], s));
  }
  k_init<<<std::max(igrid, 1), ib, 0, s>>>(c.n, d_parent, d_level, c.vis, c.nwords);
  k_seed<<<1, 1, 0, s>>>(c.off, root, d_parent, d_level, q, c.state, c.cbits);

  static int ge_cache = 0, gf_cache = 0;
  if (!ge_cache) {
    ge_cache = grid_for(g->device, (const void*)k_expand<kBlock, kItems>, kBlock, 8);
    gf_cache = grid_for(g->device, (const void*)k_fold<kTile>, 256, 4);
  }
  const int ge = g->opt.grid_blocks > 0 ? g->opt.grid_blocks : ge_cache;
  const int gf = gf_cache;
  k_fold<kTile><<<gf, 256, 0, s>>>(q, c.state, c.vis, c.jstart, c.zq, c.cbits);
  BFS_HIP(hipGetLastError());

  const int batch = g->opt.batch_levels > 0 ? g->opt.batch_levels : 4;
  const unsigned long long cmask = (1ull << c.cbits) - 1;
  const bool prof = g->opt.profile > 0;
  g->profiled = prof ? 1 : 0;
  int64_t k = 0;
  for (;;) {
    for (int b = 0; b < batch; ++b) {
      if (prof) {
        const size_t need = 2 * (size_t)(k + 1) + 2;
        while (g->ev.size() < need) {
          hipEvent_t ev;
          BFS_HIP(hipEventCreate(&ev));
          g->ev.push_back(ev);
        }
        BFS_HIP(hipEventRecord(g->ev[2 + 2 * k], s));
      }
      k_expand<kBlock, kItems><<<ge, kBlock, 0, s>>>(c.off, c.col, c.vis, d_parent, d_level, q,
                                                     c.jstart, c.zq, c.state, c.cbits);
      if (prof) BFS_HIP(hipEventRecord(g->ev[3 + 2 * k], s));
      k_fold<kTile><<<gf, 256, 0, s>>>(q, c.state, c.vis, c.jstart, c.zq, c.cbits);
      ++k;
    }
    BFS_HIP(hipGetLastError());
    BFS_HIP(hipMemcpyAsync(g->h_ctr, &c.state->ctr[k % 3], sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    BFS_HIP(hipStreamSynchronize(s));
    if ((*g->h_ctr & cmask) == 0) break;
    if (k > c.n + 2) return fail(BFS_ERR_DEVICE, "level loop did not terminate");
  }
  g->expand_launches = (int)k;
  if (prof) BFS_HIP(hipEventRecord(g->ev[1], s));
  if (host_parent)
    BFS_HIP(hipMemcpyAsync(parent, d_parent, (size_t)c.n * 4, hipMemcpyDeviceToHost, s));
  if (host_level)
    BFS_HIP(hipMemcpyAsync(level, d_level, (size_t)c.n * 4, hipMemcpyDeviceToHost, s));
  g->last_stream = s;
  g->stats_valid = 1;
  if (sync || host_parent || host_level) BFS_HIP(hipStreamSynchronize(s));
  return BFS_OK;
}

int csr_read_stats(bfs_graph* g, bfs_run_stats_t* st) {
  LevelState h;
  BFS_HIP(hipStreamSynchronize(g->last_stream));
  BFS_HIP(hipMemcpy(&h, g->csr.state, sizeof(h), hipMemcpyDeviceToHost));
  *st = bfs_run_stats_t{};
  st->depth = h.depth;
  st->levels = h.levels;
  st->edges_traversed = (int64_t)h.edges;
  st->reached = (int64_t)h.reached;
  st->frontier_total = (int64_t)h.frontier_total;
  st->expand_launches = g->expand_launches;
  if (g->profiled) {
    double sum = 0.0;
    for (int k = 0; k < g->expand_launches; ++k) {
      float ms = 0.f;
      BFS_HIP(hipEventElapsedTime(&ms, g->ev[2 + 2 * k], g->ev[3 + 2 * k]));
      sum += ms;
    }
    float tot = 0.f;
    BFS_HIP(hipEventElapsedTime(&tot, g->ev[0], g->ev[1]));
    st->expand_ms = sum;
    st->total_ms = tot;
  }
  return BFS_OK;
}

}  // namespace bfsi
