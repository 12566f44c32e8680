// Expand step of the mark-and-resolve levels (the large frontiers of
// level-synchronous BFS, section 3.2's masked (select, min) product): every
// adjacency of the frontier is streamed once and its target recorded as
// touched, without atomics per edge. finish(k) and resolve(k) in bfs_csr.hip
// turn the touched set into the next frontier and give it parents. The same
// launch runs a pull level's product by rows (pull_body) instead.
#include "bfs_level.h"
#include "bfs_search.h"

#include <algorithm>

namespace bfsi {
namespace {

// Row data of one 1024-edge tile of the mark path: its first frontier entry
// and row count (from the tile map) and, when it has at most 64 rows, lane
// r's copy of row r's edge prefix and adjacency start.
struct TileRows {
  int32_t j0, R;
  int64_t qe, qo;
};

// (w is the same for the whole wave, so are the values: readfirstlane lets
// the compiler keep them, and the branches on them, scalar)
__device__ __forceinline__ void tile_map(const int32_t* __restrict__ jstart, int64_t w,
                                         int64_t njt, int64_t F, TileRows& t) {
  const int32_t j0 = jstart[w];
  const int32_t j1 = (w + 1 < njt) ? jstart[w + 1] : (int32_t)(F - 1);
  t.j0 = __builtin_amdgcn_readfirstlane(j0);
  t.R = __builtin_amdgcn_readfirstlane(j1 - j0 + 1);
}

__device__ __forceinline__ void tile_rows(const int64_t* __restrict__ qe_in,
                                          const int64_t* __restrict__ qo_in, int lane,
                                          TileRows& t) {
  if (t.R <= 64 && lane < t.R) {
    t.qe = qe_in[t.j0 + lane];
    t.qo = qo_in[t.j0 + lane];
  }
}

// Target vertex of each of the lane's STEPS edges of tile w (-1 past the
// last edge): lane l takes edges i*64 + l. The row of an edge is the number
// of row starts at or before it in the tile's 1024-bit start mask (per-wave
// LDS), its position the distance from the last such start.
template <int STEPS>
__device__ __forceinline__ void tile_targets(const int32_t* __restrict__ col,
                                             const int64_t* __restrict__ qe_in,
                                             const int64_t* __restrict__ qo_in,
                                             uint32_t* __restrict__ starts, int lane, int64_t w,
                                             int64_t T, const TileRows& t, int32_t* vv) {
  const int64_t e0 = w * kTileJ;
  const int n_e = (int)min((int64_t)kTileJ, T - e0);
  const bool staged = t.R <= 64;
  if (lane < kTileJ / 32) starts[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int row0_pos;   // position of the tile's first edge in row 0
  if (staged) {
    row0_pos = (int)(e0 - shfl_ll(t.qe, 0));
    if (lane >= 1 && lane < t.R) {
      const int64_t rel = t.qe - e0;
      if (rel < n_e) atomicOr(&starts[rel >> 5], 1u << (rel & 31));
    }
  } else {
    row0_pos = (int)(e0 - qe_in[t.j0]);
    for (int r = 1 + lane; r < t.R; r += 64) {
      const int64_t rel = qe_in[t.j0 + r] - e0;
      if (rel < n_e) atomicOr(&starts[rel >> 5], 1u << (rel & 31));
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // Row of each edge (the number of row starts at or before it), then its
  // target. In a staged tile lane r holds row r's adjacency start minus its
  // tile-relative edge prefix, so an edge's adjacency index is that value
  // (shuffled from its row's lane, an LDS-path operation: the adjacency loads
  // never wait on one another) plus its position in the tile. A tile of more
  // than 64 rows gathers the row start from the queue and derives the
  // position in the row from the last start at or before the edge. The start
  // masks are the same for the whole wave (readfirstlane keeps their
  // bookkeeping scalar). Edges past the tile's end load col[0] and are
  // dropped.
  const uint32_t lo_below = lane < 32 ? (2u << lane) - 1u : 0xFFFFFFFFu;
  const uint32_t hi_below = lane < 32 ? 0u : (2u << (lane - 32)) - 1u;
  int base = 0;   // row starts before this step's window
  if (staged) {
    const int64_t cb = t.qo - t.qe + e0;
#pragma unroll
    for (int i = 0; i < STEPS; ++i) {
      const uint32_t mlo = __builtin_amdgcn_readfirstlane(starts[2 * i]);
      const uint32_t mhi = __builtin_amdgcn_readfirstlane(starts[2 * i + 1]);
      const int row = base + __popc(mlo & lo_below) + __popc(mhi & hi_below);   // <= R - 1
      base += __popc(mlo) + __popc(mhi);
      const int e = i * 64 + lane;
      const bool ok = e < n_e;
      // the shuffle runs in every lane (an inactive source lane would give
      // an undefined value); only the index is selected afterwards
      const int64_t rb = shfl_ll(cb, row & 63);
      const int32_t x = col[ok ? rb + e : 0];
      vv[i] = ok ? x : -1;
    }
  } else {
    int carry = row0_pos;    // position of the window's first edge in row `base`
    const int64_t* __restrict__ qo_t = qo_in + t.j0;
#pragma unroll
    for (int i = 0; i < STEPS; ++i) {
      const uint32_t mlo = __builtin_amdgcn_readfirstlane(starts[2 * i]);
      const uint32_t mhi = __builtin_amdgcn_readfirstlane(starts[2 * i + 1]);
      const uint32_t blo = mlo & lo_below, bhi = mhi & hi_below;
      const int c = __popc(blo) + __popc(bhi);
      const int last = bhi ? 63 - __clz(bhi) : 31 - __clz(blo);   // last start <= lane
      const int row = base + c;                                    // <= R - 1
      const int pos = c ? lane - last : carry + lane;
      base += __popc(mlo) + __popc(mhi);
      // the next window's first edge: just past the last start seen, or 64
      // further along the same row
      carry = mhi ? 64 - (63 - __clz(mhi)) : (mlo ? 64 - (31 - __clz(mlo)) : carry + 64);
      const bool ok = i * 64 + lane < n_e;
      const int32_t x = col[ok ? qo_t[row] + pos : 0];
      vv[i] = ok ? x : -1;
    }
  }
}

// expand(k), mark levels. One 1024-thread workgroup per CU keeps the first
// hw words of the visited bitmap in LDS for the whole level (the bitmap is
// read-only until finish(k)). A target in that hot prefix sets its bit in the
// LDS copy, which then also filters later touches of it by this workgroup; a
// target beyond it is checked in global memory and, when neither visited nor
// touched yet, gets a plain byte store of 1 in mark[] (an unvisited vertex's
// byte holds 0 or 1, so concurrent stores agree). At the end each workgroup
// writes the bits its LDS copy gained to its own slice of hot_new; finish(k)
// ORs the slices.
//
// Each wave takes whole 1024-edge tiles on its own (no workgroup barrier per
// tile). Lane l handles edges i*64 + l, i = 0..15. The row of an edge comes
// from a 1024-bit mask of the tile's row starts: the number of starts at or
// before the edge (mbcnt over the 64-bit window of step i plus a running
// count), and its position in the row from the last start at or before it.
//
// A target beyond the hot prefix reads its mark byte (nonzero = visited or
// touched) and stores 1 only when it is zero. Once a quarter of the graph is
// reached (probe = 0), or always (probe = 2), the visited word is read first
// and the mark byte only for an unvisited target: the bitmap is eight times
// denser than the bytes and stays in L2, which pays once most targets are
// visited. probe = 1 always reads the byte.
constexpr int kPushLdsBytes = kHotWordsMax * 4 + (kMarkBlock / 64) * (kTileJ / 32) * 4;
constexpr int kResolveLdsBytes = kHotWordsMax * 4 + 2 * (kResolveBlock / 64) * 8;
constexpr int kMarkLds1 = kPushLdsBytes > kPullLdsBytes ? kPushLdsBytes : kPullLdsBytes;
constexpr int kMarkLdsBytes = kMarkLds1 > kResolveLdsBytes ? kMarkLds1 : kResolveLdsBytes;
static_assert(kPullLdsBytes <= kPushLdsBytes, "the pull fits in the push level's LDS");
static_assert(kResolveBlock == kMarkBlock, "the resolve runs in the mark expand's workgroups");
static_assert(kPullBlock == kMarkBlock, "the pull runs in the mark expand's workgroups");

__global__ __launch_bounds__(kMarkBlock) void k_expand_mark(MarkArgs a) {
  constexpr int WAVES = kMarkBlock / 64;
  constexpr int STEPS = kTileJ / 64;   // edges per lane per tile
  __shared__ __align__(16) uint8_t s_lds[kMarkLdsBytes];
  const int kl = a.st->k_expand;   // this launch's level
  // a push level's resolve, deferred to this (the next) level's launch
  if (a.st->kind_prev == 1) {
    resolve_body(kl - 1, a.col, a.head, a.rpl, a.q, a.st, a.cbits, a.inv, a.hw,
                 a.prev_bits + (int64_t)((kl - 1) & 1) * a.nwords, s_lds);
    __syncthreads();
  }
  if (a.st->pull) {
    pull_body(a.off, a.col, a.head, a.vis, a.rpl, a.mark, a.st, a.mp, a.inv, a.hw,
              a.prev_bits + (int64_t)(kl & 1) * a.nwords, a.n_active, s_lds);
    return;
  }
  const int32_t* __restrict__ col = a.col;
  const uint32_t* __restrict__ vis = a.vis;
  uint8_t* __restrict__ mark = a.mark;
  const Queues& q = a.q;
  const int32_t* __restrict__ jstart_base = a.jstart;
  const int64_t njs = a.njs;
  const LevelState* __restrict__ st = a.st;
  const int cbits = a.cbits;
  const MarkPolicy& mp = a.mp;
  const int hw = a.hw;
  uint32_t* __restrict__ hot_new = a.hot_new;
  const int64_t n = a.n;
  const int probe = a.probe;
  uint32_t* s_hot = reinterpret_cast<uint32_t*>(s_lds);
  uint32_t (*s_starts)[kTileJ / 32] =
      reinterpret_cast<uint32_t (*)[kTileJ / 32]>(s_lds + kHotWordsMax * 4);

  const int k = st->k_expand;
  const int kin = k - 1;
  const unsigned long long cmask = (1ull << cbits) - 1;
  const unsigned long long cin = st->ctr[kin % 3];
  const int64_t F = (int64_t)(cin & cmask);
  const int64_t T = (int64_t)(cin >> cbits);
  if (F == 0 || !mark_level(cin, cbits, mp)) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < hw; i += kMarkBlock) s_hot[i] = vis[i];
  __syncthreads();
  const int32_t hot32 = hw << 5;
  const bool visf = probe == 2 || (probe == 0 && (int64_t)st->reached * 4 >= n);
  const int64_t njt = (T + kTileJ - 1) / kTileJ;
  const int32_t* __restrict__ jstart = jstart_base + (int64_t)(kin & 1) * njs;
  const int64_t* __restrict__ qo_in = q.qo[kin & 1];
  const int64_t* __restrict__ qe_in = q.qe[kin & 1];
  const int wid = tid >> 6;
  const int lane = lane_id();
  uint32_t* __restrict__ starts = s_starts[wid];
  const int64_t nwaves = (int64_t)gridDim.x * WAVES;
  // Three-stage software pipeline over the wave's tiles t0, t1, t2, ...:
  // while the probes of tile t0 are in flight, so are the adjacency loads of
  // t1, the row data of t2 (lane r holds row r's edge prefix and adjacency
  // start, for tiles of at most 64 rows) and the tile map of t3.
  int64_t w = (int64_t)blockIdx.x * WAVES + wid;
  if (w < njt) {
    // A: row data of the next tile (loads in flight), B: tile map of the one
    // after it
    TileRows cur{}, A{}, B{};
    tile_map(jstart, w, njt, F, cur);
    tile_rows(qe_in, qo_in, lane, cur);
    if (w + nwaves < njt) {
      tile_map(jstart, w + nwaves, njt, F, A);
      tile_rows(qe_in, qo_in, lane, A);
    }
    if (w + 2 * nwaves < njt) tile_map(jstart, w + 2 * nwaves, njt, F, B);
    int32_t vv[STEPS], vn[STEPS];
    tile_targets<STEPS>(col, qe_in, qo_in, starts, lane, w, T, cur, vv);
    for (; w < njt; w += nwaves) {
      const int64_t w1 = w + nwaves, w2 = w1 + nwaves, w3 = w2 + nwaves;
      // stage 1: adjacency loads of the next tile
      if (w1 < njt) tile_targets<STEPS>(col, qe_in, qo_in, starts, lane, w1, T, A, vn);
      // stage 2: row data of the tile after it, tile map of the third
      TileRows C{};
      if (w2 < njt) {
        tile_rows(qe_in, qo_in, lane, B);
        if (w3 < njt) tile_map(jstart, w3, njt, F, C);
      }
      // stage 3: probes of this tile
      uint32_t mk[STEPS];
      if (visf) {
        uint32_t wv[STEPS];
#pragma unroll
        for (int i = 0; i < STEPS; ++i) wv[i] = vv[i] >= hot32 ? vis[vv[i] >> 5] : 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < STEPS; ++i)
          mk[i] = (vv[i] >= hot32 && !((wv[i] >> (vv[i] & 31)) & 1u)) ? (uint32_t)mark[vv[i]] : 1u;
      } else {
#pragma unroll
        for (int i = 0; i < STEPS; ++i) mk[i] = vv[i] >= hot32 ? (uint32_t)mark[vv[i]] : 1u;
      }
      // hot targets: read the LDS words first (most bits are already set:
      // visited, or touched by this workgroup), then set the missing ones
      uint32_t hb[STEPS];
#pragma unroll
      for (int i = 0; i < STEPS; ++i) hb[i] = (vv[i] >= 0 && vv[i] < hot32) ? s_hot[vv[i] >> 5] : 0xFFFFFFFFu;
#pragma unroll
      for (int i = 0; i < STEPS; ++i) {
        const int32_t v = vv[i];
        if (v < 0) continue;
        if (v < hot32) {
          const uint32_t bit = 1u << (v & 31);
          if (!(hb[i] & bit)) atomicOr(&s_hot[v >> 5], bit);
        } else if (mk[i] == 0u) {
          mark[v] = 1;
        }
      }
      if (w1 < njt) {
#pragma unroll
        for (int i = 0; i < STEPS; ++i) vv[i] = vn[i];
      }
      A = B;
      B = C;
    }
  }
  __syncthreads();
  uint32_t* __restrict__ slice = hot_new + (int64_t)blockIdx.x * hw;
  for (int i = tid; i < hw; i += kMarkBlock) slice[i] = s_hot[i] & ~vis[i];
}

}  // namespace

int mark_expand_grid(int device) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0)
    cus = 256;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_expand_mark, kMarkBlock,
                                                   0) != hipSuccess ||
      occ <= 0)
    occ = 1;
  return cus * std::min(occ, 1);
}

void mark_expand_launch(int grid, hipStream_t s, const MarkArgs& a) {
  k_expand_mark<<<grid, kMarkBlock, 0, s>>>(a);
}

}  // namespace bfsi
