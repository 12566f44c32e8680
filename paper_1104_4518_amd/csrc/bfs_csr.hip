// Level-synchronous BFS on a CSR graph (Algorithm 1's level structure with
// one synchronisation per level, section 2.2). Each level evaluates the
// masked (select, min) product of section 3.2: the frontier's adjacencies
// are pushed, vertices already in the visited set are masked out, and every
// newly reached vertex takes the smallest frontier id among its neighbours
// as its parent.
//
// One level k is a fixed sequence of launches, all reading the level number
// and the frontier counters from device memory (consecutive levels have
// identical arguments; a launch whose level does not concern it exits at
// once, so the host enqueues several levels between reads of the frontier
// size). The level kernels work in the ids of the CSR they read (degree
// order when relabelled) and record a reached vertex as one word,
// (level << 32) | parent's caller id; k_out writes the caller's arrays from
// those words after the last level.
//
//   expand(k)  streams the adjacencies of frontier k-1 in edge-balanced
//              tiles (an exclusive degree prefix of the frontier maps every
//              edge to its row, so high-degree rows are split across tiles
//              and workgroups) and tests the visited bitmap, then claims the
//              unvisited targets in one of two ways, chosen per level from
//              the frontier's size:
//                claim  (k_expand) 64-bit atomicMin on the target's word;
//                       the thread whose atomic replaced the all-ones word
//                       appends the vertex to the next frontier (small
//                       frontiers: few atomics);
//                mark   (k_expand_mark, bfs_mark.hip) the target is recorded as touched,
//                       with no atomics per edge: in an LDS copy of the hot
//                       prefix of the visited bitmap, or by a byte store
//                       (large frontiers, symmetric graphs).
//   pull(k)    instead of the mark expand, once the frontier's adjacencies
//              outweigh those of the unvisited vertices: every unvisited
//              vertex searches its own adjacency list for a vertex of
//              frontier k-1 (the product evaluated by rows) and is marked
//              touched with its parent found.
//   finish(k)  claim levels: sets the visited bits of the new frontier.
//              mark levels: collects the touched vertices one 32-vertex word
//              per thread, appends them to the next frontier, sets their
//              visited bits and gives them the level's tag; large claim
//              levels whose claims were not waited for are collected the
//              same way, their vertices found by the level in their words.
//   resolve(k) push mark levels: gives each vertex of the new frontier its
//              level and its parent, the first neighbour one level up in
//              its ascending adjacency list (for an undirected graph that is
//              the minimum frontier id adjacent to it).
//
// All ways give the same parents: the unique minimum-id neighbour one
// level up. Appends to the next frontier are aggregated per workgroup into
// one atomic on a packed (edge total, vertex count) counter, which also
// yields the degree prefix the next level needs to split its work by edges.
#include "bfs_internal.h"
#include "bfs_level.h"
#include "bfs_search.h"

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <vector>

namespace bfsi {
namespace {

// The level kernels record a reached vertex as one word in their own ids,
// (level << 32) | parent's caller id, all ones while unreached (the claim
// path's 64-bit atomicMin then orders claims by level, then by parent id);
// k_out writes the caller's parent and level arrays from it at the end.
// Vertices of degree 0 past n_active are only ever reached as the root.
//
// k_init clears the run's state and seeds it with the root (level 0, its
// own parent, frontier 0 = {root}): parents are the caller's ids; everything
// else is indexed by the ids of the CSR the level kernels read (degree order
// when relabelled).
__global__ void k_init(int64_t n_active, unsigned long long* __restrict__ rpl,
                       uint32_t* __restrict__ vis, int64_t nwords, uint4* __restrict__ mark,
                       const int64_t* __restrict__ off, int32_t root,
                       const int32_t* __restrict__ rank, Queues q, int32_t* jstart,
                       LevelState* st, int cbits, uint32_t* __restrict__ fbits) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int32_t r = rank ? rank[root] : root;
  const unsigned long long seed = (unsigned long long)(uint32_t)root;   // level 0
  for (int64_t v = i; v < n_active; v += stride) rpl[v] = v == r ? seed : ~0ull;
  for (int64_t w = i; w < nwords; w += stride) {
    const bool rw = w == (r >> 5);
    vis[w] = rw ? 1u << (r & 31) : 0u;
    if (fbits) {   // upper-triangle graphs: frontier 0 = {root}, the other parity empty
      fbits[w] = rw ? 1u << (r & 31) : 0u;
      fbits[nwords + w] = 0u;
    }
    if (mark) {
      uint32_t x[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
      if (rw) x[(r & 31) >> 2] = (uint32_t)level_tag(0) << (8 * (r & 3));
      mark[2 * w] = make_uint4(x[0], x[1], x[2], x[3]);
      mark[2 * w + 1] = make_uint4(x[4], x[5], x[6], x[7]);
    }
  }
  if (i != 0) return;
  if (r >= n_active) rpl[r] = seed;
  const int64_t o = off[r];
  const int64_t d = off[r + 1] - o;
  // jstart holds two maps (frontier parity 0 and 1); frontier 0 uses the first
  q.qv[0][0] = r;
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
  // an upper-triangle graph's root without a stored row is still a frontier
  // vertex (its smaller neighbours find it in their rows): it counts as a
  // frontier vertex without adjacencies (its bits are set above)
  st->zcnt[0] = (d == 0 && fbits) ? 1u : 0u;
  st->zcnt[1] = st->zcnt[2] = 0u;
  st->error = 0;
  st->mark_levels = 0;
  st->pull = 0;
  st->pull_levels = 0;
  st->pull_edges = 0ull;
  st->pull_found = 0ull;
  st->pull_found_edges = 0ull;
  st->qskip = 0;
  st->kind_cur = 0;
  st->kind_prev = 0;
  st->groups = 0;
  st->small_levels = 0;
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

// Bitmap of the vertices at level k-1 (mark byte = its tag), built by the
// claim expand's threads at the start of every mark level: the searches of
// resolve and pull test it (8 times denser than the bytes), and their
// workgroups copy its hot prefix into LDS. No launch of level k changes a
// tag of level k-1 (they only turn 0 into 1 and 1 into the tag of level k).
__device__ __forceinline__ void build_prev_bits(const uint8_t* __restrict__ mark, int k,
                                                int64_t nwords,
                                                uint32_t* __restrict__ prev_bits) {
  const uint4* __restrict__ mark4 = reinterpret_cast<const uint4*>(mark);
  const uint32_t tp4 = 0x01010101u * level_tag(k - 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords; i += stride) {
    const uint4 a = mark4[2 * i], b = mark4[2 * i + 1];
    const uint32_t x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t bits = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const uint32_t e = x[t] ^ tp4;   // zero bytes = tag of level k-1
#pragma unroll
      for (int byte = 0; byte < 4; ++byte)
        if (((e >> (8 * byte)) & 0xFFu) == 0u) bits |= 1u << (4 * t + byte);
    }
    prev_bits[i] = bits;
  }
}

// expand(k), claim levels; on a mark level it only does the level's
// bookkeeping and builds the bitmap of level k-1, leaving the edges to
// k_expand_mark (push or pull).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_expand(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const uint32_t* __restrict__ vis, unsigned long long* __restrict__ rpl,
    uint8_t* __restrict__ mark, Queues q, int32_t* __restrict__ jstart_base, int64_t njs,
    int32_t* __restrict__ zq, LevelState* st, int cbits, MarkPolicy mp,
    const int32_t* __restrict__ inv, int64_t nwords, uint32_t* __restrict__ prev_bits,
    uint32_t* __restrict__ fbits, int opens_group) {
  constexpr int WAVES = BLOCK / 64;
  // the tile's rows: edge prefix, adjacency start, caller's id
  __shared__ __align__(16) long long s_qe[kTileJ + 1];
  __shared__ __align__(16) long long s_qo[kTileJ + 1];
  __shared__ uint32_t s_u[kTileJ + 1];
  __shared__ int32_t s_ov[kTileJ], s_od[kTileJ];
  __shared__ long long s_wc[WAVES], s_wd[WAVES];
  __shared__ unsigned long long s_base;
  __shared__ int s_cnt;

  const int k = st->k_expand;
  const int kin = k - 1;
  const unsigned long long cmask = (1ull << cbits) - 1;
  const unsigned long long cin = st->ctr[kin % 3];
  const int64_t F = (int64_t)(cin & cmask);
  const int64_t T = (int64_t)(cin >> cbits);
  // an upper-triangle graph's frontier may hold only vertices without
  // stored rows (counted in zcnt): the level still runs its reverse search
  const bool live = F > 0 || (fbits && st->zcnt[kin % 3] > 0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the launch group of this level's kernels: opened here, or by the
    // device level loop launched just before
    const int grp = opens_group ? st->groups++ : st->groups - 1;
    if (grp >= 0 && grp < kLevelHist) {
      if (opens_group) {
        st->grp_first[grp] = 1;
        st->grp_last[grp] = 0;
      }
      st->grp_level[grp] = live ? k : 0;
    }
    st->ctr[(k + 1) % 3] = 0ull;   // output counters of level k + 1
    st->zcnt[(k + 1) % 3] = 0u;
    st->k_fold = k;
    int pull = 0;
    if (live) st->levels = k;
    if (F > 0) {
      st->edges += (unsigned long long)T;
      st->frontier_total += (unsigned long long)F;
      if (mark_level(cin, cbits, mp)) {
        st->mark_levels += 1;
        pull = pull_level(cin, cbits, st->edges, mp);
        st->pull_levels += pull;
      }
    }
    st->pull = pull;
    st->pull_found = 0ull;
    st->pull_found_edges = 0ull;
    // the previous level's kind tells this level's mark kernel whether a
    // push level's resolve is pending (it runs there, see k_expand_mark)
    st->kind_prev = st->kind_cur;
    st->kind_cur = F > 0 ? (pull ? 2 : (mark_level(cin, cbits, mp) ? 1 : 0)) : 0;
    if (k < kLevelHist) {
      st->hist[k] = cin;
      st->hist_mark[k] = pull ? 2
                         : (mark_level(cin, cbits, mp) ? 1 : (claim_mark_level(cin, cbits, mp) ? 3 : 0));
      st->hist_pc[k] = 0ull;
      st->hist_pe[k] = 0ull;
    }
  }
  if (!live) return;
  if (fbits) {
    // upper-triangle graphs: the bitmap of parity k & 1 held frontier k - 2
    // and receives level k's vertices in finish(k); the reverse search of
    // this level reads the other one (frontier k - 1)
    uint32_t* __restrict__ fb = fbits + (int64_t)(k & 1) * nwords;
    for (int64_t w = blockIdx.x * (int64_t)BLOCK + threadIdx.x; w < nwords;
         w += (int64_t)gridDim.x * BLOCK)
      fb[w] = 0u;
  }
  if (F == 0) return;
  const bool cmark = claim_mark_level(cin, cbits, mp);
  if (mark_level(cin, cbits, mp)) {
    // level k's bitmap in buffer k & 1: the other buffer still holds level
    // k-1's, which the pending resolve of level k-1 reads
    build_prev_bits(mark, k, nwords, prev_bits + (int64_t)(k & 1) * nwords);
    return;
  }
  const int64_t njt = (T + kTileJ - 1) / kTileJ;   // jstart tiles of this level
  // tile map of frontier k-1 (read) and of frontier k (written here)
  const int32_t* __restrict__ jstart = jstart_base + (int64_t)(kin & 1) * njs;
  int32_t* __restrict__ jstart_out = jstart_base + (int64_t)(k & 1) * njs;
  const int32_t* __restrict__ qv_in = q.qv[kin & 1];
  const int64_t* __restrict__ qo_in = q.qo[kin & 1];
  const int64_t* __restrict__ qe_in = q.qe[kin & 1];
  const int tid = threadIdx.x;

  constexpr int ITEMS = kTileJ / BLOCK;
  int32_t* __restrict__ qv_out = q.qv[k & 1];
  int64_t* __restrict__ qo_out = q.qo[k & 1];
  int64_t* __restrict__ qe_out = q.qe[k & 1];
  unsigned long long* ctr_out = &st->ctr[k % 3];
  const int lane = lane_id();
  unsigned int my_reached = 0;
  // (read as every workgroup starts, before the workgroups of this launch add
  // their owners; either choice gives the same claims). After a push level
  // the words of its vertices are written by its resolve, which runs in this
  // level's mark kernel, after this one: then the visited word is needed.
  const bool resolve_pending =
      kin >= kLevelHist || (kin >= 1 && st->hist_mark[kin] == 1);
  const bool visf = resolve_pending || (int64_t)st->reached * 4 >= nwords * 32;

  for (int64_t w = blockIdx.x; w < njt; w += gridDim.x) {
    const int64_t e0 = w * kTileJ;
    const int64_t e1 = min(e0 + (int64_t)kTileJ, T);
    const int32_t j0 = jstart[w];
    const int32_t j1 = (w + 1 < njt) ? jstart[w + 1] : (int32_t)(F - 1);
    const int R = j1 - j0 + 1;
    for (int r = tid; r < R; r += BLOCK) {
      const int32_t uj = qv_in[j0 + r];
      s_qe[r] = qe_in[j0 + r];
      s_qo[r] = qo_in[j0 + r];
      s_u[r] = (uint32_t)(inv ? inv[uj] : uj);   // caller's id of the frontier vertex
    }
    if (tid == 0) s_cnt = 0;
    __syncthreads();

    if (cmark) {
      // every edge to an unvisited target: min into its word (finish finds
      // the level's vertices by their words; a touch byte per edge would
      // cost as much again as the claims)
      int32_t vv[ITEMS];
      unsigned long long key[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int64_t e = e0 + (int64_t)i * BLOCK + tid;
        vv[i] = -1;
        key[i] = 0ull;
        if (e < e1) {
          int lo = 0, hi = R - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_qe[mid] <= e) lo = mid; else hi = mid - 1;
          }
          key[i] = ((unsigned long long)k << 32) | s_u[lo];
          vv[i] = col[s_qo[lo] + (e - s_qe[lo])];
        }
      }
      uint32_t vw[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) vw[i] = vv[i] >= 0 ? vis[vv[i] >> 5] : 0xFFFFFFFFu;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i)
        if (vv[i] >= 0 && !((vw[i] >> (vv[i] & 31)) & 1u)) atomicMin(rpl + vv[i], key[i]);
      __syncthreads();
      continue;
    }

    // The thread's ITEMS edges advance stage by stage (targets, visited
    // words, current words, claims, degrees), so the loads of one stage
    // are in flight together.
    int32_t vv[ITEMS];
    unsigned long long key[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int64_t e = e0 + (int64_t)i * BLOCK + tid;
      vv[i] = -1;
      key[i] = 0ull;
      if (e < e1) {
        // row of edge e: last r with s_qe[r] <= e (rows are non-empty)
        int lo = 0, hi = R - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_qe[mid] <= e) lo = mid; else hi = mid - 1;
        }
        key[i] = ((unsigned long long)k << 32) | s_u[lo];
        vv[i] = col[s_qo[lo] + (e - s_qe[lo])];
      }
    }
    // the visited word filters the word reads only once a quarter of the
    // vertices is reached: before, nearly every target is unvisited and the
    // word read would only add a step to the chain before the claim (the
    // target's word alone tells a vertex of an earlier level: its word is
    // smaller than the key)
    uint32_t vw[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) vw[i] = (visf && vv[i] >= 0) ? vis[vv[i] >> 5] : 0u;
    unsigned long long cur[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
      cur[i] = (vv[i] >= 0 && !((vw[i] >> (vv[i] & 31)) & 1u)) ? rpl[vv[i]] : 0ull;
    bool own_i[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      own_i[i] = false;
      if (cur[i] > key[i]) own_i[i] = atomicMin(rpl + vv[i], key[i]) == ~0ull;
    }
    int64_t o0[ITEMS], o1[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      o0[i] = 0;
      o1[i] = 0;
      if (own_i[i]) {
        o0[i] = off[vv[i]];
        o1[i] = off[vv[i] + 1];
      }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const bool own = own_i[i];
      const int32_t v = vv[i];
      int32_t deg = 0;
      if (own) {
        if (mp.symmetric) mark[v] = level_tag(k);
        deg = (int32_t)(o1[i] - o0[i]);
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
        }
      }
      // reached but nothing to expand (out-degree 0): finish(k) marks it
      // visited (on an upper-triangle graph it stays a frontier vertex, found
      // by its smaller neighbours' reverse search)
      const bool zero = own && deg == 0;
      const unsigned long long mz = wave_ballot(zero);
      if (mz) {
        unsigned int base = 0;
        if (lane == 0) base = atomicAdd(&st->zcnt[k % 3], (unsigned int)__popcll(mz));
        base = __shfl(base, 0, 64);
        if (zero) zq[base + lanes_below(mz)] = v;
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
          qo_out[slot] = off[s_ov[p]];   // read moments ago by the owner: a cache hit
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
    const int64_t* __restrict__ off, uint32_t* __restrict__ vis, uint8_t* __restrict__ mark,
    const unsigned long long* __restrict__ rpl, Queues q, int32_t* __restrict__ jstart_base,
    int64_t njs, const int32_t* __restrict__ zq, LevelState* st, int cbits, int64_t n,
    int64_t n_active, int64_t nwords, MarkPolicy mp, int hw,
    const uint32_t* __restrict__ hot_new, int nslices, uint32_t* __restrict__ fbits) {
  __shared__ long long s_wc[BLOCK / 64], s_wd[BLOCK / 64];
  __shared__ unsigned long long s_base;
  __shared__ int s_exw[BLOCK / 64][64];
  __shared__ uint32_t s_m[BLOCK / 64][64];
  const int k = st->k_fold;
  const unsigned long long cmask = (1ull << cbits) - 1;
  const unsigned long long cin = st->ctr[(k - 1) % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) st->k_expand = k + 1;
  // the level did not run (an upper-triangle graph's frontier may hold only
  // vertices without stored rows)
  if ((cin & cmask) == 0 && !(fbits && st->zcnt[(k - 1) % 3] > 0)) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int tid = threadIdx.x;

  const bool cmark = claim_mark_level(cin, cbits, mp);
  if (!mark_level(cin, cbits, mp) && !cmark) {
    // claim level: visited bits of the new frontier and of its out-degree-0
    // vertices
    const unsigned long long c = st->ctr[k % 3];
    const int64_t F = (int64_t)(c & cmask);
    const int64_t Z = (int64_t)st->zcnt[k % 3];
    const int32_t* __restrict__ qv = q.qv[k & 1];
    if (mp.symmetric && F * 64 >= n) {
      // a large new frontier: its vertices carry this level's tag (set by
      // their claimers), so the words of the bitmap are rebuilt from the
      // tags instead of one atomic per vertex (vertices three levels up
      // share the tag and are visited already)
      const uint4* __restrict__ m4 = reinterpret_cast<const uint4*>(mark);
      const uint32_t t4 = 0x01010101u * level_tag(k);
      for (int64_t w = blockIdx.x * (int64_t)blockDim.x + tid; w < nwords; w += stride) {
        const uint4 a = m4[2 * w], b = m4[2 * w + 1];
        const uint32_t x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        uint32_t bits = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const uint32_t e = x[i] ^ t4;   // zero bytes = this level's tag
#pragma unroll
          for (int byte = 0; byte < 4; ++byte)
            if (((e >> (8 * byte)) & 0xFFu) == 0u) bits |= 1u << (4 * i + byte);
        }
        const uint32_t old = vis[w];
        if (bits & ~old) vis[w] = old | bits;
      }
    } else {
      for (int64_t j = blockIdx.x * (int64_t)blockDim.x + tid; j < F; j += stride) {
        const int32_t v = qv[j];
        atomicOr(&vis[v >> 5], 1u << (v & 31));
        if (fbits) atomicOr(&fbits[(int64_t)(k & 1) * nwords + (v >> 5)], 1u << (v & 31));
      }
    }
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + tid; j < Z; j += stride) {
      const int32_t v = zq[j];
      atomicOr(&vis[v >> 5], 1u << (v & 31));
      if (fbits) atomicOr(&fbits[(int64_t)(k & 1) * nwords + (v >> 5)], 1u << (v & 31));
    }
    return;
  }

  // mark level: collect the touched vertices one 32-vertex word per thread
  // (marks beyond the hot prefix, the OR of the expand workgroups' slices
  // within it), append them to the next frontier in vertex order, set their
  // visited bits and give them this level's tag. Parents come from the resolve
  // (run by the next level's mark kernel) after a push, and were set by the
  // pull on a pull level.
  int32_t* __restrict__ jstart = jstart_base + (int64_t)(k & 1) * njs;
  int32_t* __restrict__ qv_out = q.qv[k & 1];
  int64_t* __restrict__ qo_out = q.qo[k & 1];
  int64_t* __restrict__ qe_out = q.qe[k & 1];
  unsigned long long* ctr_out = &st->ctr[k % 3];
  uint4* __restrict__ mark4 = reinterpret_cast<uint4*>(mark);
  const uint32_t tcur = level_tag(k);
  // A pull level whose successor pulls too builds no queue (nothing reads
  // it): its own count of the vertices it found and their adjacencies is
  // the next level's input counter, and the successor's direction follows
  // from it as that level's expand will decide it.
  if (st->pull) {
    const unsigned long long pf = st->pull_found, pe = st->pull_found_edges;
    const unsigned long long cnext = (pe << cbits) | pf;
    if (pull_level(cnext, cbits, st->edges + pe, mp)) {
      uint4* __restrict__ m4 = reinterpret_cast<uint4*>(mark);
      for (int64_t w = blockIdx.x * (int64_t)BLOCK + tid; w < nwords; w += stride) {
        const uint4 a = m4[2 * w], b = m4[2 * w + 1];
        uint32_t x[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
          for (int byte = 0; byte < 4; ++byte)
            if (((x[i] >> (8 * byte)) & 0xFFu) == 1u) {
              m |= 1u << (4 * i + byte);
              x[i] = (x[i] & ~(0xFFu << (8 * byte))) | (tcur << (8 * byte));
            }
        if (m) {
          m4[2 * w] = make_uint4(x[0], x[1], x[2], x[3]);
          m4[2 * w + 1] = make_uint4(x[4], x[5], x[6], x[7]);
          vis[w] |= m;
        }
      }
      if (blockIdx.x == 0 && tid == 0) {
        st->ctr[k % 3] = cnext;
        st->qskip = 1;
        if (pf) {
          st->reached += pf;
          if (st->depth < k) st->depth = k;
        }
      }
      return;
    }
  }
  if (blockIdx.x == 0 && tid == 0) st->qskip = 0;
  // a pull level marks every vertex it reaches with a byte; the expand
  // workgroups' hot slices belong to the last push level then
  const int ns = (st->pull || cmark) ? 0 : nslices;
  unsigned int my_reached = 0;
  for (int64_t base = (int64_t)blockIdx.x * BLOCK; base < nwords; base += stride) {
    const int64_t w = base + tid;
    uint32_t m = 0;
    uint32_t x[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    if (w < nwords && cmark) {
      // a claim-touch level's vertices: the unvisited ones whose words hold
      // this level (set by their claims); the word's 32 parent words are read
      // only while some vertex of it is unvisited
      const uint32_t vw = vis[w];
      const int64_t vb = w << 5;
      if (vw != 0xFFFFFFFFu && vb < n_active) {
        uint32_t hit = 0;
        if (vb + 32 <= n_active) {
          const uint4* __restrict__ r4 = reinterpret_cast<const uint4*>(rpl + vb);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const uint4 t = r4[i];   // two words: high halves .y and .w hold the level
            hit |= (t.y == (uint32_t)k ? 1u : 0u) << (2 * i);
            hit |= (t.w == (uint32_t)k ? 1u : 0u) << (2 * i + 1);
          }
        } else {
          for (int i = 0; i < (int)(n_active - vb); ++i)
            hit |= ((uint32_t)(rpl[vb + i] >> 32) == (uint32_t)k ? 1u : 0u) << i;
        }
        m = hit & ~vw;
        if (m) {
          const uint4 a = mark4[2 * w], b = mark4[2 * w + 1];
          x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
          x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
        }
      }
    } else if (w < nwords) {
      const uint4 a = mark4[2 * w], b = mark4[2 * w + 1];
      x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
      x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int byte = 0; byte < 4; ++byte)
          if (((x[i] >> (8 * byte)) & 0xFFu) == 1u) m |= 1u << (4 * i + byte);
      if (w < hw && ns) {
        uint32_t h[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        int s = 0;
        for (; s + 8 <= ns; s += 8)
#pragma unroll
          for (int i = 0; i < 8; ++i) h[i] |= hot_new[(int64_t)(s + i) * hw + w];
        for (; s < ns; ++s) h[0] |= hot_new[(int64_t)s * hw + w];
#pragma unroll
        for (int i = 0; i < 8; ++i) m |= h[i];
      }
    }
    // row offsets of the word's 32 vertices, all loaded at once (the word's
    // slice of off[] is 256-byte aligned; the last word may be partial)
    int64_t o[33];
    long long cnt = __popc(m), dsum = 0;
    if (m) {
      const int64_t vb = w << 5;
      if (vb + 32 <= n) {
        const longlong2* __restrict__ o2 = reinterpret_cast<const longlong2*>(off + vb);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const longlong2 t = o2[i];
          o[2 * i] = t.x;
          o[2 * i + 1] = t.y;
        }
        o[32] = off[vb + 32];
      } else {
#pragma unroll
        for (int i = 0; i < 33; ++i) o[i] = off[min(vb + i, n)];
      }
#pragma unroll
      for (int b = 0; b < 32; ++b)
        if ((m >> b) & 1u) dsum += o[b + 1] - o[b];
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
    // The wave writes its entries in slot order, 64 consecutive slots per
    // step (coalesced stores): entry i belongs to the lane whose count range
    // holds it, and is the (i - start)-th marked vertex of that lane's word.
    {
      const int lane = lane_id();
      const int wid = tid >> 6;
      const long long c0 = __shfl(ex_c, 0, 64);     // the wave's first slot (block-relative)
      const long long d0 = __shfl(ex_d, 0, 64);
      const int wave_cnt = (int)(__shfl(ex_c + cnt, 63, 64) - c0);
      s_exw[wid][lane] = (int)(ex_c - c0);
      s_m[wid][lane] = m;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int64_t slot0 = (int64_t)(b0 & cmask) + c0;
      long long epos = (long long)(b0 >> cbits) + d0;
      const int64_t wbase = base + (wid << 6);      // word of lane 0
      for (int r = 0; r < wave_cnt; r += 64) {
        const int i = r + lane;
        int64_t d = 0, o0 = 0;
        int32_t v = 0;
        if (i < wave_cnt) {
          int lo = 0;   // last lane with s_exw <= i
#pragma unroll
          for (int step = 32; step; step >>= 1)
            if (lo + step <= 63 && s_exw[wid][lo + step] <= i) lo += step;
          v = (int32_t)(((wbase + lo) << 5) + select_bit(s_m[wid][lo], i - s_exw[wid][lo]));
          o0 = off[v];
          d = off[v + 1] - o0;
        }
        const long long incl = wave_incl_scan(d);
        const long long e = epos + incl - d;
        if (i < wave_cnt) {
          qv_out[slot0 + i] = v;
          qo_out[slot0 + i] = o0;
          qe_out[slot0 + i] = e;
          map_tiles(jstart, e, d, (int32_t)(slot0 + i));
        }
        epos += __shfl(incl, 63, 64);
      }
    }
    if (m) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int byte = 0; byte < 4; ++byte)
          if ((m >> (4 * i + byte)) & 1u)
            x[i] = (x[i] & ~(0xFFu << (8 * byte))) | (tcur << (8 * byte));
      mark4[2 * w] = make_uint4(x[0], x[1], x[2], x[3]);
      mark4[2 * w + 1] = make_uint4(x[4], x[5], x[6], x[7]);
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


// Upper-triangle graphs (each undirected edge stored once, in the row of its
// smaller endpoint, rows ascending): the first vertex of the frontier bitmap
// fb in row [o, end) of v, searched in ascending order, p = it and at = its
// position (p = -1, at = end when there is none). Each thread scans its row
// four entries at a time up to kSerialScan; the wave finishes longer rows
// together, 64 per step, so every lane of the wave must make the call.
__device__ __forceinline__ void upper_first_hit(const int32_t* __restrict__ col,
                                                const uint32_t* __restrict__ fb, int lane,
                                                int32_t v, int64_t o, int64_t end, int32_t& p,
                                                int64_t& at) {
  p = -1;
  at = end;
  bool pending = false;
  if (v >= 0) {
    const int64_t lim = min(end, o + (int64_t)kSerialScan);
    for (int64_t e = o; e < lim && p < 0; e += 4) {
      int32_t u4[4];
      uint32_t b4[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) u4[i] = e + i < lim ? col[e + i] : -1;
#pragma unroll
      for (int i = 0; i < 4; ++i) b4[i] = u4[i] >= 0 ? fb[u4[i] >> 5] : 0u;
#pragma unroll
      for (int i = 3; i >= 0; --i)
        if (u4[i] >= 0 && ((b4[i] >> (u4[i] & 31)) & 1u)) {
          p = u4[i];
          at = e + i;
        }
    }
    pending = p < 0 && end - o > kSerialScan;
  }
  for (;;) {
    const unsigned long long pend = wave_ballot(pending);
    if (!pend) break;
    const int leader = __ffsll((long long)pend) - 1;
    const int64_t lo = shfl_ll(o + kSerialScan, leader);
    const int64_t hi = shfl_ll(end, leader);
    int32_t found = -1;
    int64_t fat = hi;
    for (int64_t e0 = lo; e0 < hi; e0 += 64) {
      const int64_t e = e0 + lane;
      int32_t uu = 0;
      bool hit = false;
      if (e < hi) {
        uu = col[e];
        hit = (fb[uu >> 5] >> (uu & 31)) & 1u;
      }
      const unsigned long long hb = wave_ballot(hit);
      if (hb) {
        const int src = __ffsll((long long)hb) - 1;
        found = __shfl(uu, src, 64);
        fat = e0 + src;
        break;
      }
    }
    if (lane == leader) {
      p = found;
      at = fat;
      pending = false;
    }
  }
}

// reverse(k), upper-triangle graphs: the part of the level's product that
// the push cannot reach. Frontier vertex u pushes (k_expand's claim path)
// only to its larger neighbours, the ones stored in its own row; a vertex w
// adjacent to the frontier only through larger neighbours holds those edges
// in its own row. So every vertex unvisited before level k and not claimed
// by the push scans its row in ascending order for the first vertex of
// frontier k-1 (its bit in the frontier bitmap): that vertex is its parent,
// the minimum frontier neighbour, since it has none smaller (the push would
// have claimed it). Found vertices join the next frontier like claimed ones
// (one packed atomic per wave and round reserves their queue slots and
// edge range). Each wave takes 64 words of the visited bitmap (2048
// vertices) and lists their unvisited vertices in LDS.
constexpr int kRevBlock = 256;

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_reverse(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const uint32_t* __restrict__ vis, unsigned long long* __restrict__ rpl,
    const uint32_t* __restrict__ fbits, Queues q, int32_t* __restrict__ jstart_base, int64_t njs,
    int32_t* __restrict__ zq, LevelState* st, int cbits, int64_t n, int64_t nwords) {
  constexpr int WAVES = BLOCK / 64;
  __shared__ int s_exw[WAVES][64];
  __shared__ uint32_t s_m[WAVES][64];
  __shared__ unsigned long long s_red[3][WAVES];
  const int k = st->k_fold;
  const unsigned long long cmask = (1ull << cbits) - 1;
  const unsigned long long cin = st->ctr[(k - 1) % 3];
  if ((cin & cmask) == 0 && st->zcnt[(k - 1) % 3] == 0) return;   // empty frontier
  const uint32_t* __restrict__ fb = fbits + (int64_t)((k - 1) & 1) * nwords;
  int32_t* __restrict__ jstart = jstart_base + (int64_t)(k & 1) * njs;
  int32_t* __restrict__ qv_out = q.qv[k & 1];
  int64_t* __restrict__ qo_out = q.qo[k & 1];
  int64_t* __restrict__ qe_out = q.qe[k & 1];
  unsigned long long* ctr_out = &st->ctr[k % 3];
  const int tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
  const int64_t nchunks = (nwords + 63) >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * WAVES;
  unsigned long long my_found = 0, my_cand = 0, my_edges = 0;
  for (int64_t c = (int64_t)blockIdx.x * WAVES + wid; c < nchunks; c += nwaves) {
    const int64_t w = (c << 6) + lane;
    uint32_t m = 0u;
    if (w < nwords) {
      m = ~vis[w];
      const int64_t left = n - (w << 5);
      if (left < 32) m &= (1u << left) - 1u;
    }
    const int cnt = __popc(m);
    const int incl = (int)wave_incl_scan((long long)cnt);
    const int total = __shfl(incl, 63, 64);
    s_exw[wid][lane] = incl - cnt;
    s_m[wid][lane] = m;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int r = 0; r < total; r += 64) {
      const int i = r + lane;
      int32_t v = -1;
      if (i < total) {
        int lo = 0;   // last lane whose list starts at or before i
#pragma unroll
        for (int step = 32; step; step >>= 1)
          if (lo + step <= 63 && s_exw[wid][lo + step] <= i) lo += step;
        v = (int32_t)((((c << 6) + lo) << 5) + select_bit(s_m[wid][lo], i - s_exw[wid][lo]));
      }
      int64_t o = 0, e = 0;
      if (v >= 0) {
        if (rpl[v] != ~0ull) {
          v = -1;   // claimed by this level's push: its parent is smaller
        } else {
          o = off[v];
          e = off[v + 1];
        }
      }
      int32_t p;
      int64_t at;
      upper_first_hit(col, fb, lane, v, o, e, p, at);
      const bool found = p >= 0;
      if (v >= 0) {
        ++my_cand;
        my_edges += (unsigned long long)(found ? at - o + 1 : e - o);
      }
      if (found) rpl[v] = ((unsigned long long)k << 32) | (uint32_t)p;
      const int64_t d = found ? e - o : 0;
      const bool enq = found && d > 0;
      const unsigned long long mq = wave_ballot(enq);
      if (mq) {
        const long long dincl = wave_incl_scan(enq ? d : 0);
        const long long dsum = shfl_ll(dincl, 63);
        unsigned long long base = 0;
        if (lane == 0)
          base = atomicAdd(ctr_out, ((unsigned long long)dsum << cbits) |
                                        (unsigned long long)__popcll(mq));
        base = (unsigned long long)shfl_ll((long long)base, 0);
        if (enq) {
          const int64_t slot = (int64_t)(base & cmask) + lanes_below(mq);
          const long long ebeg = (long long)(base >> cbits) + dincl - d;
          qv_out[slot] = v;
          qo_out[slot] = o;
          qe_out[slot] = ebeg;
          map_tiles(jstart, ebeg, d, (int32_t)slot);
        }
      }
      // found, without a row of its own: a frontier vertex all the same
      // (finish(k) sets its bits)
      const unsigned long long mz = wave_ballot(found && d == 0);
      if (mz) {
        unsigned int base = 0;
        if (lane == 0) base = atomicAdd(&st->zcnt[k % 3], (unsigned int)__popcll(mz));
        base = __shfl(base, 0, 64);
        if (found && d == 0) zq[base + lanes_below(mz)] = v;
      }
      my_found += found;
    }
    __builtin_amdgcn_wave_barrier();   // the wave's lists are rewritten by its next chunk
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    my_found += __shfl_xor(my_found, d, 64);
    my_cand += __shfl_xor(my_cand, d, 64);
    my_edges += __shfl_xor(my_edges, d, 64);
  }
  if (lane == 0) {
    s_red[0][wid] = my_found;
    s_red[1][wid] = my_cand;
    s_red[2][wid] = my_edges;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long f = 0, a = 0, b = 0;
    for (int x = 0; x < WAVES; ++x) {
      f += s_red[0][x];
      a += s_red[1][x];
      b += s_red[2][x];
    }
    if (f) {
      atomicAdd(&st->reached, f);
      atomicMax(&st->depth, k);
    }
    if (k < kLevelHist && a) {
      atomicAdd(&st->hist_pc[k], a);
      atomicAdd(&st->hist_pe[k], b);
    }
  }
}

__global__ void k_build_head(int64_t n, const int64_t* __restrict__ off,
                             const int32_t* __restrict__ col, int4* __restrict__ head) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t o = off[v];
    const int64_t d = off[v + 1] - o;
    head[v] = make_int4(d > 0 ? col[o] : -1, d > 1 ? col[o + 1] : -1, d > 2 ? col[o + 2] : -1,
                        (int)d);
  }
}

// The caller's arrays from the level kernels' words: caller id x reads the
// word of its level-kernel id (a gather: the writes stay coalesced); ids of
// degree 0 past n_active other than the root were never reached.
//
// Workgroups are dealt to the 8 XCDs in turn, so workgroup b works in the
// (b mod 8)-th eighth of the caller ids: each XCD's L2 then sees one
// contiguous range, whose reads fall in a few ascending runs of level-kernel
// ids (the degree order keeps caller order within a degree), and a fetched
// line serves all of its words there. The grid is a multiple of 8.
constexpr int kXcds = 8;

__global__ void k_out(int64_t n, const int32_t* __restrict__ rank, int64_t n_active,
                      int32_t root, const unsigned long long* __restrict__ rpl,
                      int32_t* __restrict__ parent, int32_t* __restrict__ level) {
  constexpr int U = 4;   // ids per thread per step, their loads in flight together
  const int64_t span = (n + kXcds - 1) / kXcds;
  const int64_t lo = (int64_t)(blockIdx.x % kXcds) * span;
  const int64_t hi = min(n, lo + span);
  const int64_t bstride = (int64_t)(gridDim.x / kXcds) * blockDim.x;
  for (int64_t x0 = lo + (int64_t)(blockIdx.x / kXcds) * blockDim.x * U + threadIdx.x; x0 < hi;
       x0 += bstride * U) {
    int64_t r[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const int64_t x = x0 + (int64_t)i * blockDim.x;
      r[i] = x < hi ? (rank ? rank[x] : x) : -1;
    }
    unsigned long long w[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const int64_t x = x0 + (int64_t)i * blockDim.x;
      w[i] = (r[i] >= 0 && (r[i] < n_active || x == root)) ? rpl[r[i]] : ~0ull;
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const int64_t x = x0 + (int64_t)i * blockDim.x;
      if (x < hi) {
        parent[x] = (int32_t)(uint32_t)w[i];
        if (level) level[x] = (int32_t)(uint32_t)(w[i] >> 32);
      }
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

// Upper triangle: every adjacency v of row u has v > u and follows a
// smaller one in its row. Sets *bad on a violation. Runs only on validated
// CSR arrays.
__global__ void k_check_upper(int64_t n, int64_t nnz, const int64_t* __restrict__ off,
                              const int32_t* __restrict__ col, int32_t* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += stride) {
    int64_t prev = u;
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      if ((int64_t)col[e] <= prev) {
        atomicOr(bad, 1);
        break;
      }
      prev = col[e];
    }
  }
}

// Degree-ordered copy: row v' of the copy is row inv[v'] of the original with
// every adjacency mapped through rank (order within the row unchanged, so it
// stays ascending in original ids). One wave per row.
__global__ void k_permute_rows(int64_t n, const int64_t* __restrict__ off,
                               const int32_t* __restrict__ col, const int64_t* __restrict__ roff,
                               const int32_t* __restrict__ inv, const int32_t* __restrict__ rank,
                               int32_t* __restrict__ rcol) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int lane = lane_id();
  for (int64_t v = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); v < n;
       v += waves) {
    const int64_t src = off[inv[v]];
    const int64_t len = off[inv[v] + 1] - src;
    const int64_t dst = roff[v];
    for (int64_t i = lane; i < len; i += 64) rcol[dst + i] = rank[col[src + i]];
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
// graph mode: levels per captured graph
constexpr int kGraphLevels = 16;

}  // namespace

int csr_alloc_workspace(bfs_graph* g) {
  CsrDev& c = g->csr;
  // default grids of the claim expand and the finish on this handle's device
  c.grid_expand = grid_for(g->device, (const void*)k_expand<kExpandBlock>, kExpandBlock, 8);
  c.grid_finish = grid_for(g->device, (const void*)k_finish<kFinishBlock>, kFinishBlock, 4);
  c.nwords = (c.n + 31) / 32;
  c.njstart = c.nnz / kTileJ + 2;
  BFS_HIP(hipMalloc(&c.vis, (size_t)std::max<int64_t>(c.nwords, 1) * 4));
  BFS_HIP(hipMalloc(&c.rpl, (size_t)std::max<int64_t>(c.n, 1) * 8));
  for (int b = 0; b < 2; ++b) {
    BFS_HIP(hipMalloc(&c.qv[b], (size_t)c.n * 4));
    BFS_HIP(hipMalloc(&c.qo[b], (size_t)c.n * 8));
    BFS_HIP(hipMalloc(&c.qe[b], (size_t)c.n * 8));
  }
  BFS_HIP(hipMalloc(&c.jstart, (size_t)c.njstart * 2 * 4));
  BFS_HIP(hipMalloc(&c.zq, (size_t)c.n * 4));
  BFS_HIP(hipMalloc(&c.state, sizeof(LevelState)));
  BFS_HIP(hipMemset(c.state, 0, sizeof(LevelState)));
  if (c.upper) {
    BFS_HIP(hipMalloc(&c.fbits, (size_t)std::max<int64_t>(c.nwords, 1) * 8));
    g->device_bytes += std::max<int64_t>(c.nwords, 1) * 8;
  }
  if (c.symmetric) {
    BFS_HIP(hipMalloc(&c.mark, (size_t)std::max<int64_t>(c.nwords, 1) * 32));
    BFS_HIP(hipMemset(c.mark, 0, (size_t)std::max<int64_t>(c.nwords, 1) * 32));
    g->device_bytes += std::max<int64_t>(c.nwords, 1) * 32;
    // one slice of hot-prefix bits per mark-path workgroup (one per CU)
    c.hot_words = (int)std::min<int64_t>(std::max<int64_t>(c.nwords, 1), kHotWordsMax);
    c.hot_slices = mark_expand_grid(g->device);
    BFS_HIP(hipMalloc(&c.hot_new, (size_t)c.hot_slices * c.hot_words * 4));
    // two buffers: level k's and level k-1's (read by the deferred resolve)
    BFS_HIP(hipMalloc(&c.prev_bits, (size_t)std::max<int64_t>(c.nwords, 1) * 8));
    // head copy of the rows the searches read (the level kernels' CSR)
    if (!c.relabeled) c.n_active = c.n;
    BFS_HIP(hipMalloc(&c.head, (size_t)std::max<int64_t>(c.n_active, 1) * 16));
    k_build_head<<<4096, 256>>>(c.n_active, c.relabeled ? c.roff : c.off,
                                c.relabeled ? c.rcol : c.col, c.head);
    BFS_HIP(hipGetLastError());
    BFS_HIP(hipDeviceSynchronize());
    g->device_bytes += std::max<int64_t>(c.n_active, 1) * 16;
    g->device_bytes += std::max<int64_t>(c.nwords, 1) * 8;
    g->device_bytes += (int64_t)c.hot_slices * c.hot_words * 4;
  }
  g->device_bytes += std::max<int64_t>(c.nwords, 1) * 4 + c.n * 52 + c.njstart * 8 +
                     (int64_t)sizeof(LevelState);
  return BFS_OK;
}

void csr_free(bfs_graph* g) {
  CsrDev& c = g->csr;
  (void)hipFree(c.off);
  (void)hipFree(c.col);
  (void)hipFree(c.vis);
  (void)hipFree(c.rpl);
  (void)hipFree(c.head);
  for (int b = 0; b < 2; ++b) {
    (void)hipFree(c.qv[b]);
    (void)hipFree(c.qo[b]);
    (void)hipFree(c.qe[b]);
  }
  (void)hipFree(c.jstart);
  (void)hipFree(c.zq);
  (void)hipFree(c.mark);
  (void)hipFree(c.hot_new);
  (void)hipFree(c.prev_bits);
  (void)hipFree(c.fbits);
  (void)hipFree(c.state);
  if (c.gexec) (void)hipGraphExecDestroy(c.gexec);
  if (c.cap_stream) (void)hipStreamDestroy(c.cap_stream);
  (void)hipFree(c.tmp_parent);
  (void)hipFree(c.tmp_level);
  (void)hipFree(c.roff);
  (void)hipFree(c.rcol);
  (void)hipFree(c.rank);
  (void)hipFree(c.inv);
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

int csr_check_upper(bfs_graph* g, hipStream_t s, int* upper) {
  CsrDev& c = g->csr;
  *upper = 0;
  int32_t* d_bad = nullptr;
  BFS_HIP(hipMalloc(&d_bad, 4));
  BFS_HIP(hipMemsetAsync(d_bad, 0, 4, s));
  if (c.nnz > 0) k_check_upper<<<4096, 256, 0, s>>>(c.n, c.nnz, c.off, c.col, d_bad);
  int32_t h = 0;
  hipError_t e = hipMemcpyAsync(&h, d_bad, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_bad);
  if (e != hipSuccess) return hip_fail(e, "upper-triangle check");
  *upper = h == 0;
  return BFS_OK;
}

int csr_relabel(bfs_graph* g, const int64_t* host_off, hipStream_t s) {
  CsrDev& c = g->csr;
  const int64_t n = c.n;
  // counting sort by descending degree, ties by ascending id
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; ++v) maxdeg = std::max(maxdeg, host_off[v + 1] - host_off[v]);
  std::vector<int64_t> start((size_t)maxdeg + 2, 0);
  for (int64_t v = 0; v < n; ++v) ++start[(size_t)(maxdeg - (host_off[v + 1] - host_off[v]))];
  int64_t acc = 0;
  for (size_t b = 0; b < start.size(); ++b) {
    const int64_t t = start[b];
    start[b] = acc;
    acc += t;
  }
  std::vector<int32_t> inv((size_t)n), rank((size_t)n);
  for (int64_t v = 0; v < n; ++v) {
    const int64_t nv = start[(size_t)(maxdeg - (host_off[v + 1] - host_off[v]))]++;
    inv[(size_t)nv] = (int32_t)v;
    rank[(size_t)v] = (int32_t)nv;
  }
  std::vector<int64_t> roff((size_t)n + 1);
  roff[0] = 0;
  for (int64_t i = 0; i < n; ++i)
    roff[(size_t)i + 1] = roff[(size_t)i] + (host_off[inv[(size_t)i] + 1] - host_off[inv[(size_t)i]]);
  BFS_HIP(hipMalloc(&c.roff, (size_t)(n + 1) * 8));
  BFS_HIP(hipMalloc(&c.rcol, (size_t)std::max<int64_t>(c.nnz, 1) * 4));
  BFS_HIP(hipMalloc(&c.rank, (size_t)n * 4));
  BFS_HIP(hipMalloc(&c.inv, (size_t)n * 4));
  BFS_HIP(hipMemcpyAsync(c.roff, roff.data(), roff.size() * 8, hipMemcpyHostToDevice, s));
  BFS_HIP(hipMemcpyAsync(c.rank, rank.data(), rank.size() * 4, hipMemcpyHostToDevice, s));
  BFS_HIP(hipMemcpyAsync(c.inv, inv.data(), inv.size() * 4, hipMemcpyHostToDevice, s));
  k_permute_rows<<<4096, 256, 0, s>>>(n, c.off, c.col, c.roff, c.inv, c.rank, c.rcol);
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipStreamSynchronize(s));
  c.relabeled = 1;
  // degree-descending order: the vertices of positive degree come first;
  // only in a symmetric graph are the others unreachable (a directed graph
  // reaches vertices of out-degree 0)
  c.n_active = n;
  if (c.symmetric) {
    c.n_active = 0;
    while (c.n_active < n && roff[(size_t)c.n_active + 1] > roff[(size_t)c.n_active]) ++c.n_active;
  }
  g->device_bytes += (n + 1) * 8 + std::max<int64_t>(c.nnz, 1) * 4 + n * 8;
  return BFS_OK;
}

int csr_run(bfs_graph* g, int32_t root, int32_t* parent, int32_t* level, hipStream_t s,
            bool sync) {
  CsrDev& c = g->csr;
  if (root < 0 || (int64_t)root >= c.n) return fail(BFS_ERR_ARG, "root out of range");
  if (!parent) return fail(BFS_ERR_ARG, "parent output is required");

  // claim policy of this run
  const int claim = g->opt.claim > 0 ? g->opt.claim : 3;
  MarkPolicy mp;
  mp.symmetric = (claim != 1) && c.symmetric;
  mp.min_edges = g->opt.claim_threshold > 0 ? (long long)g->opt.claim_threshold
                                            : std::max<long long>(c.n / 64, 4096);
  mp.min_vertices = g->opt.claim_min_frontier > 0
                        ? (long long)g->opt.claim_min_frontier
                        : std::min<long long>(std::max<long long>(c.n / 1024, 1024), 4096);
  if (claim == 2) mp.min_edges = mp.min_vertices = 1;
  mp.nnz = (long long)c.nnz;
  mp.pull_alpha = g->opt.pull_alpha > 0 ? g->opt.pull_alpha : 0;

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
  const int64_t n_active = c.relabeled ? c.n_active : c.n;
  // the level kernels read the degree-ordered copy when there is one
  const int64_t* koff = c.relabeled ? c.roff : c.off;
  const int32_t* kcol = c.relabeled ? c.rcol : c.col;
  const int32_t* kinv = c.relabeled ? c.inv : nullptr;
  const int32_t* krank = c.relabeled ? c.rank : nullptr;
  k_init<<<std::max(igrid, 1), ib, 0, s>>>(n_active, c.rpl, c.vis, c.nwords,
                                           mp.symmetric ? reinterpret_cast<uint4*>(c.mark)
                                                        : nullptr,
                                           koff, root, krank, q, c.jstart, c.state, c.cbits,
                                           c.upper ? c.fbits : nullptr);

  // launch shapes: the claim expand and finish fill the chip with 256-thread
  // workgroups; the mark expand runs one 1024-thread workgroup per CU (its
  // LDS holds the hot prefix of the visited bitmap)

  const int ge = g->opt.grid_blocks > 0 ? g->opt.grid_blocks : c.grid_expand;
  const int gm = g->opt.grid_blocks > 0 ? std::min(g->opt.grid_blocks, c.hot_slices) : c.hot_slices;
  const int gf = c.grid_finish;
  BFS_HIP(hipGetLastError());

  const int batch = g->opt.batch_levels > 0 ? g->opt.batch_levels : 4;
  const unsigned long long cmask = (1ull << c.cbits) - 1;
  const bool prof = g->opt.profile > 0;
  const int probe = g->opt.cold_probe == 3 ? 0 : g->opt.cold_probe;
  // the device level loop for small frontiers (not for upper-triangle
  // graphs, whose levels also need the reverse search)
  const bool small_on = !c.upper && g->opt.small_frontier >= 0;
  // whether the launch groups being enqueued start with the loop: in mode 1
  // only while the frontier last read by the host was small enough for it
  // (a batch after a large frontier would mostly launch it for nothing; its
  // small levels then run through the level kernels until the next read)
  bool loop_now = small_on;
  SmallArgs sa;
  sa.off = koff;
  sa.col = kcol;
  sa.vis = c.vis;
  sa.rpl = c.rpl;
  sa.mark = c.mark;
  sa.inv = kinv;
  sa.q = q;
  sa.jstart = c.jstart;
  sa.njs = c.njstart;
  sa.st = c.state;
  sa.cbits = c.cbits;
  sa.mp = mp;
  sa.max_f = g->opt.small_frontier > 0
                 ? std::min<int64_t>(g->opt.small_frontier, small_max_frontier())
                 : small_max_frontier();
  sa.max_t = small_max_edges();
  // One launch group: the device level loop (it runs as many small claim
  // levels as it can, or returns at once), then one level's kernels for the
  // level it leaves. ev_base >= 0 brackets them with events ev_base ..
  // ev_base + 4 (loop | claim expand or level bitmap, and the reverse search
  // of upper-triangle graphs | mark expand or pull, after the previous push
  // level's resolve | finish).
  auto enqueue_group = [&](hipStream_t st, int64_t ev_base) -> int {
    if (ev_base >= 0) BFS_HIP(hipEventRecord(g->ev[(size_t)ev_base], st));
    if (loop_now) small_levels_launch(st, sa);
    if (ev_base >= 0) BFS_HIP(hipEventRecord(g->ev[(size_t)ev_base + 1], st));
    k_expand<kExpandBlock><<<ge, kExpandBlock, 0, st>>>(koff, kcol, c.vis, c.rpl,
                                                        c.mark, q, c.jstart, c.njstart, c.zq,
                                                        c.state, c.cbits, mp, kinv,
                                                        c.nwords, c.prev_bits,
                                                        c.upper ? c.fbits : nullptr,
                                                        loop_now ? 0 : 1);
    if (c.upper)
      k_reverse<kRevBlock><<<gf, kRevBlock, 0, st>>>(koff, kcol, c.vis, c.rpl, c.fbits, q,
                                                     c.jstart, c.njstart, c.zq, c.state,
                                                     c.cbits, c.n, c.nwords);
    if (ev_base >= 0) BFS_HIP(hipEventRecord(g->ev[(size_t)ev_base + 2], st));
    if (mp.symmetric) {
      MarkArgs a;
      a.col = kcol;
      a.off = koff;
      a.head = c.head;
      a.vis = c.vis;
      a.mark = c.mark;
      a.rpl = c.rpl;
      a.inv = kinv;
      a.q = q;
      a.jstart = c.jstart;
      a.njs = c.njstart;
      a.st = c.state;
      a.cbits = c.cbits;
      a.mp = mp;
      a.hw = c.hot_words;
      a.hot_new = c.hot_new;
      a.prev_bits = c.prev_bits;
      a.n = c.n;
      a.n_active = n_active;
      a.nwords = c.nwords;
      a.probe = probe;
      mark_expand_launch(gm, st, a);
    }
    if (ev_base >= 0) BFS_HIP(hipEventRecord(g->ev[(size_t)ev_base + 3], st));
    k_finish<kFinishBlock><<<gf, kFinishBlock, 0, st>>>(koff, c.vis, c.mark, c.rpl, q,
                                                        c.jstart, c.njstart, c.zq, c.state,
                                                        c.cbits, c.n, n_active, c.nwords, mp,
                                                        c.hot_words, c.hot_new, gm,
                                                        c.upper ? c.fbits : nullptr);
    if (ev_base >= 0) BFS_HIP(hipEventRecord(g->ev[(size_t)ev_base + 4], st));
    return BFS_OK;
  };
  // the frontier the next group would expand: the counter of level
  // k_expand - 1 (the host reads the counters and k_expand together)
  int64_t k = 0;   // launch groups enqueued
  static_assert(offsetof(LevelState, zcnt) + sizeof(LevelState::zcnt) <= 16 * 8,
                "the host check reads the state's head into 16 words");
  auto frontier_left = [&]() -> int {
    BFS_HIP(hipMemcpyAsync(g->h_ctr, c.state, offsetof(LevelState, zcnt) + 12,
                           hipMemcpyDeviceToHost, s));
    BFS_HIP(wait_stream(s));
    const char* head = reinterpret_cast<const char*>(g->h_ctr);
    int32_t kx = 0;
    std::memcpy(&kx, head + offsetof(LevelState, k_expand), 4);
    // a search has at most n levels; every launch group enqueued after its
    // last one advances the level number by one more
    if (kx < 1 || (int64_t)kx > c.n + 2 + k)
      return fail(BFS_ERR_DEVICE, "level loop did not terminate");
    unsigned long long ctr = 0;
    unsigned int z = 0;
    std::memcpy(&ctr, head + offsetof(LevelState, ctr) + 8 * ((kx - 1) % 3), 8);
    std::memcpy(&z, head + offsetof(LevelState, zcnt) + 4 * ((kx - 1) % 3), 4);
    loop_now = small_on && (int64_t)(ctr & cmask) <= sa.max_f &&
               (int64_t)(ctr >> c.cbits) <= sa.max_t;
    if (ctr & cmask) return 1;
    // rowless frontier vertices of an upper-triangle graph
    return (c.upper && z > 0) ? 1 : 0;
  };
  if (g->opt.mode == 2) {
    // Graph mode: kGraphLevels launch groups captured once per (outputs,
    // policy, launch shapes) and replayed until the frontier is empty;
    // replays between host checks double up to 8.
    GraphKey key{};
    key.mp_sym = mp.symmetric;
    key.mp_edges = mp.min_edges;
    key.mp_vertices = mp.min_vertices;
    key.probe = probe;
    key.grids[0] = ge;
    key.grids[1] = gm;
    key.grids[2] = gf;
    key.grids[3] = small_on ? (int)sa.max_f : -1;
    key.mp_alpha = mp.pull_alpha;
    key.pad = 0;
    if (!c.gexec || std::memcmp(&key, &c.gkey, sizeof(key)) != 0) {
      if (c.gexec) (void)hipGraphExecDestroy(c.gexec);
      c.gexec = nullptr;
      if (!c.cap_stream) BFS_HIP(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
      BFS_HIP(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal));
      int rc = BFS_OK;
      for (int l = 0; l < kGraphLevels && rc == BFS_OK; ++l) rc = enqueue_group(c.cap_stream, -1);
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(c.cap_stream, &graph);
      if (rc != BFS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
      const hipError_t ei = hipGraphInstantiate(&c.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        c.gexec = nullptr;
        return hip_fail(ei, "hipGraphInstantiate");
      }
      c.gkey = key;
    }
    int replays = 1;
    for (;;) {
      for (int r = 0; r < replays; ++r) {
        BFS_HIP(hipGraphLaunch(c.gexec, s));
        k += kGraphLevels;
      }
      const int left = frontier_left();
      if (left < 0) return left;
      if (!left) break;
      replays = std::min(replays * 2, 8);
    }
    g->profiled = prof ? 2 : 0;   // whole-run time only
  } else {
    g->profiled = prof ? 1 : 0;
    for (;;) {
      for (int b = 0; b < batch; ++b) {
        if (prof) {
          const size_t need = 5 * (size_t)(k + 1) + 2;
          while (g->ev.size() < need) {
            hipEvent_t ev;
            BFS_HIP(hipEventCreate(&ev));
            g->ev.push_back(ev);
          }
        }
        const int rc = enqueue_group(s, prof ? 2 + 5 * k : -1);
        if (rc != BFS_OK) return rc;
        ++k;
      }
      BFS_HIP(hipGetLastError());
      const int left = frontier_left();
      if (left < 0) return left;
      if (!left) break;
    }
  }
  g->expand_launches = (int)k;
  const int ogrid = std::max(kXcds, igrid / kXcds * kXcds);
  k_out<<<ogrid, ib, 0, s>>>(c.n, krank, n_active, root, c.rpl, d_parent, d_level);
  BFS_HIP(hipGetLastError());
  if (prof) BFS_HIP(hipEventRecord(g->ev[1], s));
  if (host_parent)
    BFS_HIP(hipMemcpyAsync(parent, d_parent, (size_t)c.n * 4, hipMemcpyDeviceToHost, s));
  if (host_level)
    BFS_HIP(hipMemcpyAsync(level, d_level, (size_t)c.n * 4, hipMemcpyDeviceToHost, s));
  g->last_stream = s;
  g->stats_valid = 1;
  if (sync || host_parent || host_level) BFS_HIP(wait_stream(s));
  return BFS_OK;
}

namespace {

float elapsed(const std::vector<hipEvent_t>& ev, size_t a, size_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ev[a], ev[b]) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms;
}

// Per launch group of the last profiled run: the level its level kernels
// processed and the levels its device loop ran.
struct Groups {
  std::vector<int32_t> level, first, last;
};

int read_groups(bfs_graph* g, Groups* gr) {
  const int ng = std::min(g->expand_launches, kLevelHist);
  gr->level.assign((size_t)ng, 0);
  gr->first.assign((size_t)ng, 1);
  gr->last.assign((size_t)ng, 0);
  if (ng == 0) return BFS_OK;
  BFS_HIP(hipMemcpy(gr->level.data(), g->csr.state->grp_level, (size_t)ng * 4,
                    hipMemcpyDeviceToHost));
  BFS_HIP(hipMemcpy(gr->first.data(), g->csr.state->grp_first, (size_t)ng * 4,
                    hipMemcpyDeviceToHost));
  BFS_HIP(hipMemcpy(gr->last.data(), g->csr.state->grp_last, (size_t)ng * 4,
                    hipMemcpyDeviceToHost));
  return BFS_OK;
}

}  // namespace

int csr_read_stats(bfs_graph* g, bfs_run_stats_t* st) {
  LevelState h;
  BFS_HIP(hipStreamSynchronize(g->last_stream));
  // the counters only, not the per-level history
  BFS_HIP(hipMemcpy(&h, g->csr.state, offsetof(LevelState, hist), hipMemcpyDeviceToHost));
  *st = bfs_run_stats_t{};
  st->depth = h.depth;
  st->levels = h.levels;
  st->edges_traversed = (int64_t)h.edges;
  st->reached = (int64_t)h.reached;
  st->frontier_total = (int64_t)h.frontier_total;
  st->expand_launches = g->expand_launches;
  st->mark_levels = h.mark_levels;
  st->pull_levels = h.pull_levels;
  st->pull_edges = (int64_t)h.pull_edges;
  st->small_levels = h.small_levels;
  if (g->profiled == 1) {
    // the mark kernel's time goes to mark_ms on push levels, pull_ms on
    // pull levels
    Groups gr;
    int rc = read_groups(g, &gr);
    if (rc != BFS_OK) return rc;
    std::vector<int32_t> kind(kLevelHist, 0);
    BFS_HIP(hipMemcpy(kind.data(), g->csr.state->hist_mark, kind.size() * 4,
                      hipMemcpyDeviceToHost));
    double sum = 0.0, msum = 0.0, psum = 0.0, ssum = 0.0, fsum = 0.0;
    for (int t = 0; t < g->expand_launches; ++t) {
      const size_t b = 2 + 5 * (size_t)t;
      ssum += elapsed(g->ev, b, b + 1);
      sum += elapsed(g->ev, b + 1, b + 3);
      const float mm = elapsed(g->ev, b + 2, b + 3);
      const int lv = t < (int)gr.level.size() ? gr.level[(size_t)t] : 0;
      if (lv > 0 && lv < kLevelHist && kind[(size_t)lv] == 2) psum += mm;
      else msum += mm;
      fsum += elapsed(g->ev, b + 3, b + 4);
    }
    st->mark_ms = msum;
    st->pull_ms = psum;
    st->expand_ms = sum;
    st->small_ms = ssum;
    st->finish_ms = fsum;
  }
  if (g->profiled) st->total_ms = elapsed(g->ev, 0, 1);
  return BFS_OK;
}

int csr_level_info(bfs_graph* g, bfs_level_info_t* out, int32_t capacity, int32_t* count) {
  BFS_HIP(hipStreamSynchronize(g->last_stream));
  Groups gr;
  int rc = read_groups(g, &gr);
  if (rc != BFS_OK) return rc;
  // levels with a record: every level a group's kernels or loop touched
  int top = 0;
  for (size_t t = 0; t < gr.level.size(); ++t) {
    top = std::max(top, gr.level[t]);
    if (gr.first[t] <= gr.last[t]) top = std::max(top, gr.last[t]);
  }
  // the launches after the last level find an empty frontier: one record
  // for the level that found it
  top = std::min(top + 1, kLevelHist - 1);
  const int n = std::min<int>(capacity, top);
  std::vector<unsigned long long> hist((size_t)n + 1);
  std::vector<int32_t> hmark((size_t)n + 1);
  std::vector<unsigned long long> hpc((size_t)n + 1), hpe((size_t)n + 1);
  BFS_HIP(hipMemcpy(hist.data(), g->csr.state->hist, hist.size() * 8, hipMemcpyDeviceToHost));
  BFS_HIP(hipMemcpy(hmark.data(), g->csr.state->hist_mark, hmark.size() * 4,
                    hipMemcpyDeviceToHost));
  BFS_HIP(hipMemcpy(hpc.data(), g->csr.state->hist_pc, hpc.size() * 8, hipMemcpyDeviceToHost));
  BFS_HIP(hipMemcpy(hpe.data(), g->csr.state->hist_pe, hpe.size() * 8, hipMemcpyDeviceToHost));
  const unsigned long long cmask = (1ull << g->csr.cbits) - 1;
  // level -> the group whose level kernels processed it, and the group whose
  // loop started at it
  std::vector<int> by_kernels((size_t)n + 1, -1), loop_start((size_t)n + 1, -1);
  for (size_t t = 0; t < gr.level.size(); ++t) {
    const int lv = gr.level[t];
    if (lv > 0 && lv <= n && by_kernels[(size_t)lv] < 0) by_kernels[(size_t)lv] = (int)t;
    if (gr.first[t] <= gr.last[t] && gr.first[t] <= n) loop_start[(size_t)gr.first[t]] = (int)t;
  }
  for (int i = 0; i < n; ++i) {
    const int k = i + 1;
    bfs_level_info_t& L = out[i];
    L = bfs_level_info_t{};
    L.level = k;
    L.mark = hmark[(size_t)k];
    L.frontier = (int64_t)(hist[(size_t)k] & cmask);
    L.edges = (int64_t)(hist[(size_t)k] >> g->csr.cbits);
    L.pull_candidates = (int64_t)hpc[(size_t)k];
    L.pull_edges = (int64_t)hpe[(size_t)k];
    if (g->profiled != 1) continue;   // per-launch events exist only level by level
    const int t = by_kernels[(size_t)k];
    if (t >= 0) {
      const size_t b = 2 + 5 * (size_t)t;
      const double m = elapsed(g->ev, b + 2, b + 3);
      L.expand_ms = elapsed(g->ev, b + 1, b + 3);
      L.mark_ms = L.mark == 2 ? 0.0 : m;
      L.pull_ms = L.mark == 2 ? m : 0.0;
      L.finish_ms = elapsed(g->ev, b + 3, b + 4);
    }
    const int tl = loop_start[(size_t)k];
    if (tl >= 0) L.small_ms = elapsed(g->ev, 2 + 5 * (size_t)tl, 3 + 5 * (size_t)tl);
  }
  *count = n;
  return BFS_OK;
}

}  // namespace bfsi
