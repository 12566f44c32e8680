// Level-synchronous BFS on a CSR graph (Algorithm 1's level structure with
// one synchronisation per level, section 2.2). Each level evaluates the
// masked (select, min) product of section 3.2: the frontier's adjacencies
// are pushed, vertices already in the visited set are masked out, and every
// newly reached vertex takes the smallest frontier id among its neighbours
// as its parent.
//
// One level k is two launches, both reading the level number and the
// frontier counters from device memory (consecutive launches have identical
// arguments; a level whose input frontier is empty exits at once, so the
// host enqueues several levels between reads of the frontier size):
//
//   expand(k)  streams the adjacencies of frontier k-1 in edge-balanced
//              tiles (an exclusive degree prefix of the frontier maps every
//              edge to its row, so high-degree rows are split across tiles
//              and workgroups) and tests the visited bitmap, then claims the
//              unvisited targets in one of two ways, chosen per level from
//              the frontier's edge count:
//                claim  atomicMin on parent[]; the thread whose atomic turned
//                       parent from -1 into a frontier id appends the vertex
//                       to the next frontier (small frontiers: few atomics);
//                mark   a plain byte store marks the target as touched; no
//                       atomics per edge (large frontiers, symmetric graphs).
//   finish(k)  claim levels: sets the visited bits of the new frontier.
//              mark levels: scans the marks one 32-vertex word per thread,
//              gives each marked vertex its level and its parent, which is
//              the first neighbour one level up in its ascending adjacency
//              list (for an undirected graph that is the minimum frontier
//              id adjacent to it), appends it to the next frontier, sets
//              the visited word and clears the marks.
//
// Both ways give the same parents: the unique minimum-id neighbour one
// level up. Appends to the next frontier are aggregated per workgroup into
// one atomic on a packed (edge total, vertex count) counter, which also
// yields the degree prefix the next level needs to split its work by edges.
#include "bfs_internal.h"

#include <algorithm>

namespace bfsi {
namespace {

// jstart granularity and claim-path tile: 1024 edges (256 threads x 4)
constexpr int kTileJ = 1024;
// mark path: super-tiles of 4 x 1024 edges, 16 edges per thread
constexpr int kMarkSub = 4;
constexpr int kMarkItems = 16;
// LDS of the expand kernel: the larger of the two paths' needs
constexpr int kLdsQe = kTileJ * kMarkSub + 1;   // staged row starts (int64)
constexpr int kLdsBytes = kLdsQe * 8;
static_assert((kTileJ + 1) * 8 + kTileJ * (4 + 4 + 8) <= kLdsBytes, "claim path LDS");

struct Queues {
  int32_t* qv[2];
  int64_t* qo[2];
  int64_t* qe[2];
};

__device__ __forceinline__ bool mark_level(unsigned long long cin, int cbits, int symmetric,
                                           long long thresh) {
  return symmetric && (long long)(cin >> cbits) >= thresh;
}

__global__ void k_init(int64_t n, int32_t* __restrict__ parent, int32_t* __restrict__ level,
                       uint32_t* __restrict__ vis, int64_t nwords, uint4* __restrict__ mark) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = i; v < n; v += stride) {
    parent[v] = -1;
    if (level) level[v] = -1;
  }
  for (int64_t w = i; w < nwords; w += stride) {
    vis[w] = 0u;
    if (mark) {
      mark[2 * w] = make_uint4(0u, 0u, 0u, 0u);
      mark[2 * w + 1] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
}

__global__ void k_seed(const int64_t* __restrict__ off, int32_t root, int32_t* parent,
                       int32_t* level, uint32_t* vis, Queues q, int32_t* jstart, LevelState* st,
                       int cbits) {
  // jstart holds two maps (frontier parity 0 and 1); frontier 0 uses the first
  parent[root] = root;
  if (level) level[root] = 0;
  vis[root >> 5] |= 1u << (root & 31);
  const int64_t o = off[root];
  const int64_t d = off[root + 1] - o;
  q.qv[0][0] = root;
  q.qo[0][0] = o;
  q.qe[0][0] = 0;
  for (int64_t w = 0; w * kTileJ < d; ++w) jstart[w] = 0;
  st->ctr[0] = d > 0 ? (((unsigned long long)d << cbits) | 1ull) : 0ull;
  st->ctr[1] = 0ull;
  st->ctr[2] = 0ull;
  st->k_expand = 1;
  st->k_fold = 1;
  st->depth = 0;
  st->levels = 0;
  st->edges = 0ull;
  st->reached = 1ull;
  st->frontier_total = 0ull;
  st->zcnt[0] = st->zcnt[1] = st->zcnt[2] = 0u;
  st->error = 0;
  st->mark_levels = 0;
}

// Block-wide exclusive scan of (count, degree sum) pairs; returns the
// exclusive prefixes of this thread and writes the block totals.
template <int BLOCK>
__device__ __forceinline__ void block_scan2(long long c, long long d, long long* s_c,
                                            long long* s_d, long long& ex_c, long long& ex_d,
                                            long long& tot_c, long long& tot_d) {
  constexpr int WAVES = BLOCK / 64;
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const long long ic = wave_incl_scan(c);
  const long long id = wave_incl_scan(d);
  if (lane == 63) {
    s_c[wid] = ic;
    s_d[wid] = id;
  }
  __syncthreads();
  long long bc = 0, bd = 0;
  tot_c = 0;
  tot_d = 0;
#pragma unroll
  for (int x = 0; x < WAVES; ++x) {
    if (x < wid) {
      bc += s_c[x];
      bd += s_d[x];
    }
    tot_c += s_c[x];
    tot_d += s_d[x];
  }
  ex_c = bc + ic - c;
  ex_d = bd + id - d;
}

// Map the edge tiles of the next level that start inside [e, e + d) to
// queue entry j.
__device__ __forceinline__ void map_tiles(int32_t* __restrict__ jstart, long long e, long long d,
                                          int32_t j) {
  for (long long w = (e + kTileJ - 1) / kTileJ; w * kTileJ < e + d; ++w) jstart[w] = j;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_expand(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const uint32_t* __restrict__ vis, int32_t* __restrict__ parent, int32_t* __restrict__ level,
    uint8_t* __restrict__ mark, Queues q, int32_t* __restrict__ jstart_base, int64_t njs,
    int32_t* __restrict__ zq, LevelState* st, int cbits, int symmetric, long long thresh) {
  constexpr int WAVES = BLOCK / 64;
  __shared__ __align__(16) unsigned char s_raw[kLdsBytes];
  __shared__ long long s_wc[WAVES], s_wd[WAVES];
  __shared__ unsigned long long s_base;
  __shared__ int s_cnt;
  long long* s_qe = reinterpret_cast<long long*>(s_raw);

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
    if (F > 0) {
      st->levels = k;
      st->edges += (unsigned long long)T;
      st->frontier_total += (unsigned long long)F;
      if (mark_level(cin, cbits, symmetric, thresh)) st->mark_levels += 1;
    }
  }
  if (F == 0) return;
  const int64_t njt = (T + kTileJ - 1) / kTileJ;   // jstart tiles of this level
  // tile map of frontier k-1 (read) and of frontier k (written by the claim path)
  const int32_t* __restrict__ jstart = jstart_base + (int64_t)(kin & 1) * njs;
  int32_t* __restrict__ jstart_out = jstart_base + (int64_t)(k & 1) * njs;
  const int32_t* __restrict__ qv_in = q.qv[kin & 1];
  const int64_t* __restrict__ qo_in = q.qo[kin & 1];
  const int64_t* __restrict__ qe_in = q.qe[kin & 1];
  const int tid = threadIdx.x;

  if (mark_level(cin, cbits, symmetric, thresh)) {
    // ---------------------------------------------------------- mark path
    constexpr int TILE = kTileJ * kMarkSub;
    static_assert(BLOCK * kMarkItems == TILE, "mark tile shape");
    const int64_t nitems = (T + TILE - 1) / TILE;
    for (int64_t w = blockIdx.x; w < nitems; w += gridDim.x) {
      const int64_t e0 = w * TILE;
      const int64_t e1 = min(e0 + (int64_t)TILE, T);
      const int32_t j0 = jstart[w * kMarkSub];
      const int32_t j1 = ((w + 1) * kMarkSub < njt) ? jstart[(w + 1) * kMarkSub] : (int32_t)(F - 1);
      const int R = j1 - j0 + 1;
      for (int r = tid; r < R; r += BLOCK) s_qe[r] = qe_in[j0 + r];
      __syncthreads();
      int32_t vv[kMarkItems];
#pragma unroll
      for (int i = 0; i < kMarkItems; ++i) {
        const int64_t e = e0 + (int64_t)i * BLOCK + tid;
        vv[i] = -1;
        if (e < e1) {
          int lo = 0, hi = R - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_qe[mid] <= e) lo = mid; else hi = mid - 1;
          }
          vv[i] = col[qo_in[j0 + lo] + (e - s_qe[lo])];
        }
      }
      uint32_t wv[kMarkItems];
#pragma unroll
      for (int i = 0; i < kMarkItems; ++i) wv[i] = vv[i] >= 0 ? vis[vv[i] >> 5] : 0xFFFFFFFFu;
      uint8_t mk[kMarkItems];
#pragma unroll
      for (int i = 0; i < kMarkItems; ++i) {
        const bool unvisited = vv[i] >= 0 && !((wv[i] >> (vv[i] & 31)) & 1u);
        mk[i] = unvisited ? mark[vv[i]] : (uint8_t)1;
      }
#pragma unroll
      for (int i = 0; i < kMarkItems; ++i)
        if (mk[i] == 0) mark[vv[i]] = 1;
      __syncthreads();
    }
    return;
  }

  // ------------------------------------------------------------ claim path
  constexpr int ITEMS = kTileJ / BLOCK;
  int32_t* s_ov = reinterpret_cast<int32_t*>(s_raw + (kTileJ + 1) * 8);
  int32_t* s_od = s_ov + kTileJ;
  long long* s_oo = reinterpret_cast<long long*>(s_od + kTileJ);
  int32_t* __restrict__ qv_out = q.qv[k & 1];
  int64_t* __restrict__ qo_out = q.qo[k & 1];
  int64_t* __restrict__ qe_out = q.qe[k & 1];
  unsigned long long* ctr_out = &st->ctr[k % 3];
  const int lane = lane_id();
  unsigned int my_reached = 0;

  for (int64_t w = blockIdx.x; w < njt; w += gridDim.x) {
    const int64_t e0 = w * kTileJ;
    const int64_t e1 = min(e0 + (int64_t)kTileJ, T);
    const int32_t j0 = jstart[w];
    const int32_t j1 = (w + 1 < njt) ? jstart[w + 1] : (int32_t)(F - 1);
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
      // reached but nothing to expand (out-degree 0): finish(k) marks it visited
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
      long long c = 0, d = 0;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int p = tid * ITEMS + i;
        if (p < C) {
          ++c;
          d += s_od[p];
        }
      }
      long long ex_c, ex_d, tot_c, tot_d;
      block_scan2<BLOCK>(c, d, s_wc, s_wd, ex_c, ex_d, tot_c, tot_d);
      if (tid == 0)
        s_base = atomicAdd(ctr_out, ((unsigned long long)tot_d << cbits) |
                                        (unsigned long long)tot_c);
      __syncthreads();
      const unsigned long long b = s_base;
      const int64_t bc = (int64_t)(b & cmask);
      long long run = (long long)(b >> cbits) + ex_d;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int p = tid * ITEMS + i;
        if (p < C) {
          const int64_t slot = bc + p;
          qv_out[slot] = s_ov[p];
          qo_out[slot] = s_oo[p];
          qe_out[slot] = run;
          map_tiles(jstart_out, run, s_od[p], (int32_t)slot);
          run += s_od[p];
        }
      }
    }
    __syncthreads();
  }

  unsigned int r = my_reached;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) r += __shfl_xor(r, d, 64);
  __shared__ unsigned int s_red[WAVES];
  if (lane == 0) s_red[tid >> 6] = r;
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

// finish(k): see the header comment.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_finish(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, uint32_t* __restrict__ vis,
    int32_t* __restrict__ parent, int32_t* __restrict__ level, uint8_t* __restrict__ mark,
    Queues q, int32_t* __restrict__ jstart_base, int64_t njs, const int32_t* __restrict__ zq,
    LevelState* st, int cbits, int64_t nwords, int symmetric, long long thresh) {
  __shared__ long long s_wc[BLOCK / 64], s_wd[BLOCK / 64];
  __shared__ unsigned long long s_base;
  const int k = st->k_fold;
  const unsigned long long cmask = (1ull << cbits) - 1;
  const unsigned long long cin = st->ctr[(k - 1) % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) st->k_expand = k + 1;
  if ((cin & cmask) == 0) return;   // the level did not run
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int tid = threadIdx.x;

  if (!mark_level(cin, cbits, symmetric, thresh)) {
    // claim level: visited bits of the new frontier and of its out-degree-0
    // vertices
    const unsigned long long c = st->ctr[k % 3];
    const int64_t F = (int64_t)(c & cmask);
    const int64_t Z = (int64_t)st->zcnt[k % 3];
    const int32_t* __restrict__ qv = q.qv[k & 1];
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + tid; j < F; j += stride) {
      const int32_t v = qv[j];
      atomicOr(&vis[v >> 5], 1u << (v & 31));
    }
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + tid; j < Z; j += stride) {
      const int32_t v = zq[j];
      atomicOr(&vis[v >> 5], 1u << (v & 31));
    }
    return;
  }

  // mark level: resolve every marked vertex, one 32-vertex word per thread
  int32_t* __restrict__ jstart = jstart_base + (int64_t)(k & 1) * njs;
  int32_t* __restrict__ qv_out = q.qv[k & 1];
  int64_t* __restrict__ qo_out = q.qo[k & 1];
  int64_t* __restrict__ qe_out = q.qe[k & 1];
  unsigned long long* ctr_out = &st->ctr[k % 3];
  const uint4* __restrict__ mark4 = reinterpret_cast<const uint4*>(mark);
  const int32_t kprev = k - 1;
  unsigned int my_reached = 0;
  for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < nwords; base += stride) {
    const int64_t w = base + tid;
    uint32_t m = 0;
    if (w < nwords) {
      const uint4 a = mark4[2 * w], b = mark4[2 * w + 1];
      const uint32_t x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int byte = 0; byte < 4; ++byte)
          if ((x[i] >> (8 * byte)) & 0xFFu) m |= 1u << (4 * i + byte);
    }
    long long cnt = __popc(m), dsum = 0;
    for (uint32_t bits = m; bits; bits &= bits - 1) {
      const int64_t v = (w << 5) + (__ffs(bits) - 1);
      dsum += off[v + 1] - off[v];
    }
    long long ex_c, ex_d, tot_c, tot_d;
    block_scan2<BLOCK>(cnt, dsum, s_wc, s_wd, ex_c, ex_d, tot_c, tot_d);
    if (tot_c == 0) {
      __syncthreads();
      continue;
    }
    if (tid == 0)
      s_base = atomicAdd(ctr_out, ((unsigned long long)tot_d << cbits) |
                                      (unsigned long long)tot_c);
    __syncthreads();
    const unsigned long long b0 = s_base;
    __syncthreads();
    int64_t slot = (int64_t)(b0 & cmask) + ex_c;
    long long epos = (long long)(b0 >> cbits) + ex_d;
    for (uint32_t bits = m; bits; bits &= bits - 1) {
      const int32_t v = (int32_t)((w << 5) + (__ffs(bits) - 1));
      const int64_t o = off[v];
      const int64_t d = off[v + 1] - o;
      // parent: first neighbour one level up in the ascending adjacency
      int32_t p = -1;
      for (int64_t e = o; e < o + d; ++e) {
        const int32_t u = col[e];
        if (level[u] == kprev) {
          p = u;
          break;
        }
      }
      parent[v] = p;
      level[v] = k;
      qv_out[slot] = v;
      qo_out[slot] = o;
      qe_out[slot] = epos;
      map_tiles(jstart, epos, d, (int32_t)slot);
      ++slot;
      epos += d;
    }
    if (m) {
      uint4* mw = reinterpret_cast<uint4*>(mark);
      mw[2 * w] = make_uint4(0u, 0u, 0u, 0u);
      mw[2 * w + 1] = make_uint4(0u, 0u, 0u, 0u);
      vis[w] |= m;
      my_reached += __popc(m);
    }
  }
  unsigned int r = my_reached;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) r += __shfl_xor(r, d, 64);
  __shared__ unsigned int s_red[BLOCK / 64];
  if (lane_id() == 0) s_red[tid >> 6] = r;
  __syncthreads();
  if (tid == 0) {
    unsigned int t = 0;
    for (int x = 0; x < BLOCK / 64; ++x) t += s_red[x];
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

// Undirected with ascending rows: every row non-decreasing, and for every
// adjacency v in row u, u appears in row v (binary search). Sets *bad on the
// first violation found by a thread. Runs only on validated CSR arrays.
__global__ void k_check_symmetric(int64_t n, int64_t nnz, const int64_t* __restrict__ off,
                                  const int32_t* __restrict__ col, int32_t* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += stride) {
    // row of e: last u with off[u] <= e
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (off[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int64_t u = lo;
    const int32_t v = col[e];
    if (e > off[u] && col[e - 1] > v) {
      atomicOr(bad, 1);
      continue;
    }
    int64_t a = off[v], b = off[v + 1];
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if ((int64_t)col[mid] < u) a = mid + 1; else b = mid;
    }
    if (a >= off[v + 1] || (int64_t)col[a] != u) atomicOr(bad, 2);
  }
}

__global__ void k_widen_offsets(int64_t n1, const int32_t* __restrict__ src,
                                int64_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n1; i += stride)
    dst[i] = (int64_t)src[i];
}

constexpr int kExpandBlock = 256;
constexpr int kFinishBlock = 256;

}  // namespace

int csr_alloc_workspace(bfs_graph* g) {
  CsrDev& c = g->csr;
  c.nwords = (c.n + 31) / 32;
  c.njstart = c.nnz / kTileJ + 2 + kMarkSub;
  BFS_HIP(hipMalloc(&c.vis, (size_t)std::max<int64_t>(c.nwords, 1) * 4));
  for (int b = 0; b < 2; ++b) {
    BFS_HIP(hipMalloc(&c.qv[b], (size_t)c.n * 4));
    BFS_HIP(hipMalloc(&c.qo[b], (size_t)c.n * 8));
    BFS_HIP(hipMalloc(&c.qe[b], (size_t)c.n * 8));
  }
  BFS_HIP(hipMalloc(&c.jstart, (size_t)c.njstart * 2 * 4));
  BFS_HIP(hipMalloc(&c.zq, (size_t)c.n * 4));
  BFS_HIP(hipMalloc(&c.state, sizeof(LevelState)));
  BFS_HIP(hipMemset(c.state, 0, sizeof(LevelState)));
  if (c.symmetric) {
    BFS_HIP(hipMalloc(&c.mark, (size_t)std::max<int64_t>(c.nwords, 1) * 32));
    BFS_HIP(hipMemset(c.mark, 0, (size_t)std::max<int64_t>(c.nwords, 1) * 32));
    g->device_bytes += std::max<int64_t>(c.nwords, 1) * 32;
  }
  g->device_bytes += std::max<int64_t>(c.nwords, 1) * 4 + c.n * 44 + c.njstart * 8 +
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
  (void)hipFree(c.mark);
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

int csr_check_symmetric(bfs_graph* g, hipStream_t s, int* symmetric) {
  CsrDev& c = g->csr;
  *symmetric = 0;
  if (c.nnz == 0) {
    *symmetric = 1;
    return BFS_OK;
  }
  int32_t* d_bad = nullptr;
  BFS_HIP(hipMalloc(&d_bad, 4));
  BFS_HIP(hipMemsetAsync(d_bad, 0, 4, s));
  k_check_symmetric<<<4096, 256, 0, s>>>(c.n, c.nnz, c.off, c.col, d_bad);
  int32_t h = 0;
  hipError_t e = hipMemcpyAsync(&h, d_bad, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_bad);
  if (e != hipSuccess) return hip_fail(e, "symmetry check");
  *symmetric = h == 0;
  return BFS_OK;
}

int csr_run(bfs_graph* g, int32_t root, int32_t* parent, int32_t* level, hipStream_t s,
            bool sync) {
  CsrDev& c = g->csr;
  if (root < 0 || (int64_t)root >= c.n) return fail(BFS_ERR_ARG, "root out of range");
  if (!parent) return fail(BFS_ERR_ARG, "parent output is required");

  // claim policy of this run
  const int claim = g->opt.claim > 0 ? g->opt.claim : 3;
  const int use_mark = (claim != 1) && c.symmetric;
  long long thresh = g->opt.claim_threshold > 0 ? (long long)g->opt.claim_threshold
                                                : std::max<long long>(c.n / 64, 4096);
  if (claim == 2) thresh = 1;

  int32_t* d_parent = parent;
  int32_t* d_level = level;
  const bool host_parent = !is_device_ptr(parent);
  const bool host_level = level && !is_device_ptr(level);
  if (host_parent) {
    if (!c.tmp_parent) BFS_HIP(hipMalloc(&c.tmp_parent, (size_t)c.n * 4));
    d_parent = c.tmp_parent;
  }
  // the mark path reads levels, so it needs a level array even when the
  // caller does not ask for one
  if (host_level || (!level && use_mark)) {
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
  k_init<<<std::max(igrid, 1), ib, 0, s>>>(c.n, d_parent, d_level, c.vis, c.nwords,
                                           reinterpret_cast<uint4*>(c.mark));
  k_seed<<<1, 1, 0, s>>>(c.off, root, d_parent, d_level, c.vis, q, c.jstart, c.state, c.cbits);

  static int ge_cache = 0, gf_cache = 0;
  if (!ge_cache) {
    ge_cache = grid_for(g->device, (const void*)k_expand<kExpandBlock>, kExpandBlock, 4);
    gf_cache = grid_for(g->device, (const void*)k_finish<kFinishBlock>, kFinishBlock, 4);
  }
  const int ge = g->opt.grid_blocks > 0 ? g->opt.grid_blocks : ge_cache;
  const int gf = gf_cache;
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
      k_expand<kExpandBlock><<<ge, kExpandBlock, 0, s>>>(c.off, c.col, c.vis, d_parent, d_level,
                                                         c.mark, q, c.jstart, c.njstart, c.zq,
                                                         c.state, c.cbits, use_mark, thresh);
      if (prof) BFS_HIP(hipEventRecord(g->ev[3 + 2 * k], s));
      k_finish<kFinishBlock><<<gf, kFinishBlock, 0, s>>>(c.off, c.col, c.vis, d_parent, d_level,
                                                         c.mark, q, c.jstart, c.njstart, c.zq,
                                                         c.state, c.cbits, c.nwords, use_mark,
                                                         thresh);
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
  st->mark_levels = h.mark_levels;
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
