// Multi-query BFS: many (graph, root) queries in one launch.
//
// Each workgroup runs whole queries, one at a time, level-synchronously
// (Algorithm 1's level loop, with the workgroup barrier as the per-level
// synchronisation of section 2.2). Within a level the workgroup expands its
// frontier in chunks of WG vertices: a workgroup-wide prefix sum of the
// chunk's degrees splits the chunk's adjacencies evenly over the threads
// (edge-balanced gather, so a hub row is shared by the whole workgroup),
// every adjacency tests the visited bitmap and claims unvisited vertices
// with atomicMin on parent[] (the (select, min) semiring of section 3.2),
// and the unique claimer of each vertex appends it to the next frontier
// through a workgroup-local counter in LDS.
//
// When the graph has at most kLdsBits vertices, the visited bitmap lives in
// LDS; otherwise in the query's global workspace. A query touches only its
// own parent/level/workspace, so all synchronisation is workgroup-local and
// queries of different sizes never wait for each other.
//
// The same kernel serves two callers:
//   - bfs_run_batch: workgroups pull queries from a list (largest estimated
//     cost first) and run each to completion;
//   - the server: one workgroup per active slot advances its query until it
//     finishes or a time budget expires at a level boundary, saving the
//     frontier level, its size and (in LDS mode) the bitmap in the slot.
#include "bfs_multi.h"

#include <algorithm>

namespace bfsi {
namespace {

template <int WG, int LDS_WORDS, int ROUND>
__global__ __launch_bounds__(WG) void k_bfs_multi(MQuery* __restrict__ qs,
                                                  const int32_t* __restrict__ order, int32_t count,
                                                  int32_t* __restrict__ next_counter,
                                                  int32_t pull, unsigned long long budget,
                                                  char* __restrict__ ws_base, int64_t ws_stride,
                                                  int64_t ws_qbytes) {
  constexpr int WAVES = WG / 64;
  __shared__ uint32_t s_vis[LDS_WORDS];
  __shared__ long long s_pre[WG];
  __shared__ long long s_off[WG];
  __shared__ int32_t s_u[WG];
  __shared__ long long s_wsum[WAVES];
  __shared__ int s_cnt;
  __shared__ int s_idx;
  __shared__ int s_yield;

  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;

  for (int round = 0;; ++round) {
    if (tid == 0) {
      int idx;
      if (pull) idx = atomicAdd(next_counter, 1);
      else idx = round == 0 ? (int)blockIdx.x : count;
      s_idx = idx;
    }
    __syncthreads();
    const int idx = s_idx;
    if (idx >= count) return;
    MQuery& Q = qs[order ? order[idx] : idx];
    const int64_t* __restrict__ off = Q.off;
    const int32_t* __restrict__ col = Q.col;
    int32_t* __restrict__ parent = Q.parent;
    int32_t* __restrict__ level = Q.level;
    const int32_t n = Q.n;
    const bool lds = n <= LDS_WORDS * 32;
    const int32_t nw = (n + 31) >> 5;
    uint32_t* __restrict__ gvis = Q.vis;
    int32_t* __restrict__ qbuf[2] = {Q.q[0], Q.q[1]};
    if (ws_base) {
      // per-workgroup workspace (queries run to completion on one workgroup)
      char* w = ws_base + (int64_t)blockIdx.x * ws_stride;
      qbuf[0] = reinterpret_cast<int32_t*>(w);
      qbuf[1] = reinterpret_cast<int32_t*>(w + ws_qbytes);
      gvis = reinterpret_cast<uint32_t*>(w + 2 * ws_qbytes);
    }
    const unsigned long long t0 = wall_clock64();

    int32_t k, F;
    unsigned long long edges;
    int32_t depth;
    if (Q.status == kQueryPending) {
      for (int32_t v = tid; v < n; v += WG) {
        parent[v] = -1;
        if (level) level[v] = -1;
      }
      if (lds) {
        for (int32_t w = tid; w < nw; w += WG) s_vis[w] = 0u;
      } else {
        for (int32_t w = tid; w < nw; w += WG) gvis[w] = 0u;
      }
      __syncthreads();
      if (tid == 0) {
        const int32_t r = Q.root;
        parent[r] = r;
        if (level) level[r] = 0;
        qbuf[0][0] = r;
        if (lds) s_vis[r >> 5] |= 1u << (r & 31);
        else gvis[r >> 5] |= 1u << (r & 31);
      }
      k = 0;
      F = 1;
      edges = 0ull;
      depth = 0;
    } else {
      k = Q.k;
      F = Q.F;
      edges = Q.edges;
      depth = Q.depth;
      if (lds)
        for (int32_t w = tid; w < nw; w += WG) s_vis[w] = gvis[w];
    }
    __syncthreads();

    bool yielded = false;
    while (F > 0) {
      if (budget) {
        if (tid == 0) s_yield = (wall_clock64() - t0) > budget;
        __syncthreads();
        if (s_yield) {
          yielded = true;
          break;
        }
      }
      const int32_t* __restrict__ cur = qbuf[k & 1];
      int32_t* __restrict__ nxt = qbuf[(k + 1) & 1];
      if (tid == 0) s_cnt = 0;
      const uint32_t kn = (uint32_t)(k + 1);
      for (int32_t c0 = 0; c0 < F; c0 += WG) {
        const int32_t i = c0 + tid;
        long long d = 0, o = 0;
        int32_t u = 0;
        if (i < F) {
          u = cur[i];
          o = off[u];
          d = off[u + 1] - o;
        }
        const long long incl = wave_incl_scan(d);
        if (lane == 63) s_wsum[wid] = incl;
        __syncthreads();
        long long wb = 0, tot = 0;
#pragma unroll
        for (int x = 0; x < WAVES; ++x) {
          const long long sx = s_wsum[x];
          if (x < wid) wb += sx;
          tot += sx;
        }
        s_pre[tid] = wb + incl - d;
        s_off[tid] = o;
        s_u[tid] = u;
        __syncthreads();
        const int rows = min(WG, F - c0);
        edges += (unsigned long long)tot;   // same value in every thread
        // the chunk's adjacencies, ROUND per thread per step with their
        // loads in flight together (targets, visited bits, parents, claims)
        for (long long e0 = 0; e0 < tot; e0 += (long long)WG * ROUND) {
          int32_t v[ROUND];
          uint32_t uu[ROUND];
#pragma unroll
          for (int i = 0; i < ROUND; ++i) {
            const long long e = e0 + (long long)i * WG + tid;
            v[i] = -1;
            uu[i] = 0u;
            if (e < tot) {
              int lo = 0, hi = rows - 1;
              while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pre[mid] <= e) lo = mid; else hi = mid - 1;
              }
              v[i] = col[s_off[lo] + (e - s_pre[lo])];
              uu[i] = (uint32_t)s_u[lo];
            }
          }
          bool fresh[ROUND];
#pragma unroll
          for (int i = 0; i < ROUND; ++i) {
            fresh[i] = false;
            if (v[i] >= 0) {
              const uint32_t bit = 1u << (v[i] & 31);
              fresh[i] = !(lds ? (s_vis[v[i] >> 5] & bit) : (gvis[v[i] >> 5] & bit));
            }
          }
          uint32_t pcur[ROUND];
#pragma unroll
          for (int i = 0; i < ROUND; ++i)
            pcur[i] = fresh[i] ? reinterpret_cast<uint32_t*>(parent)[v[i]] : 0u;
#pragma unroll
          for (int i = 0; i < ROUND; ++i) {
            bool own = false;
            if (fresh[i] && pcur[i] > uu[i]) {
              uint32_t* pp = reinterpret_cast<uint32_t*>(parent) + v[i];
              const uint32_t old = __hip_atomic_fetch_min(pp, uu[i], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_WORKGROUP);
              own = old == 0xFFFFFFFFu;
            }
            if (own && level) level[v[i]] = (int32_t)kn;
            const unsigned long long m = wave_ballot(own);
            if (m) {
              int base = 0;
              if (lane == 0) base = atomicAdd(&s_cnt, __popcll(m));
              base = __shfl(base, 0, 64);
              if (own) nxt[base + lanes_below(m)] = v[i];
            }
          }
        }
        __syncthreads();
      }
      const int32_t Fn = s_cnt;
      for (int32_t j = tid; j < Fn; j += WG) {
        const int32_t v = nxt[j];
        if (lds) atomicOr(&s_vis[v >> 5], 1u << (v & 31));
        else atomicOr(&gvis[v >> 5], 1u << (v & 31));
      }
      __syncthreads();
      if (Fn > 0) depth = k + 1;
      k += 1;
      F = Fn;
    }

    if (tid == 0) {
      Q.k = k;
      Q.F = F;
      Q.edges = edges;
      Q.depth = depth;
      Q.status = yielded ? kQueryRunning : kQueryDone;
    }
    if (yielded && lds)
      for (int32_t w = tid; w < nw; w += WG) gvis[w] = s_vis[w];
    __syncthreads();
  }
}

}  // namespace

constexpr int kMultiRound = 8;   // adjacencies per thread in flight

const void* multi_kernel() {
  return (const void*)k_bfs_multi<kMultiWG, kLdsWords, kMultiRound>;
}

int multi_launch(MQuery* d_qs, const int32_t* d_order, int32_t count, int32_t* d_counter,
                 int grid, bool pull, unsigned long long budget, char* ws_base,
                 int64_t ws_stride, int64_t ws_qbytes, hipStream_t s) {
  if (count <= 0) return BFS_OK;
  k_bfs_multi<kMultiWG, kLdsWords, kMultiRound><<<grid, kMultiWG, 0, s>>>(
      d_qs, d_order, count, d_counter,
                                                             pull ? 1 : 0, budget, ws_base,
                                                             ws_stride, ws_qbytes);
  BFS_HIP(hipGetLastError());
  return BFS_OK;
}

int multi_grid(int device) {
  static int cached[64] = {0};
  if (device < 0 || device >= 64) device = 0;
  if (!cached[device]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0)
      cus = 256;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, multi_kernel(), kMultiWG, 0) !=
            hipSuccess ||
        occ <= 0)
      occ = 1;
    cached[device] = cus * occ;
  }
  return cached[device];
}

__global__ void k_zero_i32(int32_t* p) { *p = 0; }

int multi_reset_counter(int32_t* d_counter, hipStream_t s) {
  k_zero_i32<<<1, 1, 0, s>>>(d_counter);
  BFS_HIP(hipGetLastError());
  return BFS_OK;
}

}  // namespace bfsi
