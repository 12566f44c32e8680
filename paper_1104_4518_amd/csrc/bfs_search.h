// Search helpers shared by the level kernels of bfs_csr.hip (finish) and
// bfs_mark.hip (the mark-level kernel, which also runs the pull levels and
// the deferred resolve): selecting a set bit, the head copy's first step and
// the rest of the searches for a neighbour one level up, the resolve and the
// pull.
#pragma once

#include "bfs_level.h"

namespace bfsi {

// Position of the r-th (0-based) set bit of x; x has more than r set bits.
__device__ __forceinline__ int select_bit(uint32_t x, int r) {
  int pos = 0;
  int c = __popc(x & 0xFFFFu);
  if (r >= c) { r -= c; x >>= 16; pos += 16; }
  c = __popc(x & 0xFFu);
  if (r >= c) { r -= c; x >>= 8; pos += 8; }
  c = __popc(x & 0xFu);
  if (r >= c) { r -= c; x >>= 4; pos += 4; }
  c = __popc(x & 0x3u);
  if (r >= c) { r -= c; x >>= 2; pos += 2; }
  if (r >= (int)(x & 1u)) pos += 1;
  return pos;
}

// Vertex u at level k-1: its bit in the LDS copy of the hot prefix (below
// hotv) or in the level's bitmap pbits (built from the tags at the start of
// the level).
__device__ __forceinline__ bool prev_level(int32_t u, int64_t hotv, const uint32_t* s_prev,
                                           const uint32_t* __restrict__ pbits) {
  return ((u < hotv ? s_prev[u >> 5] : pbits[u >> 5]) >> (u & 31)) & 1u;
}


// Dense copy of every vertex's first kHead adjacencies with its degree,
// (u0, u1, u2, degree), entries past the degree -1. The searches of pull
// and resolve test a vertex's first neighbours from it, reading it in vertex
// order (coalesced) instead of one scattered row start per vertex, and read
// the row itself only when those do not decide.
constexpr int kHead = 3;


// First step of the searches for a neighbour one level up (a bit of the
// level-(k-1) bitmap pbits, or of its LDS copy s_prev below hotv): the first
// kHead adjacencies of each of the thread's RV vertices, from the head copy. p[t] = the first
// such neighbour and pos[t] its index (< kHead), or p[t] = -1; deg[t] = the
// vertex's degree (0 for v[t] < 0). The LDS tests of hot neighbours come
// first, so bitmap words are read only for the cold ones ahead of a hot hit.
template <int RV>
__device__ __forceinline__ void head_step(const int4* __restrict__ head,
                                          const uint32_t* __restrict__ pbits,
                                          const uint32_t* s_prev, int64_t hotv,
                                          const int32_t (&v)[RV], int32_t (&p)[RV],
                                          int (&pos)[RV], int32_t (&deg)[RV]) {
  int32_t u[RV][kHead];
#pragma unroll
  for (int t = 0; t < RV; ++t) {
    const int4 h = v[t] >= 0 ? head[v[t]] : make_int4(-1, -1, -1, 0);
    u[t][0] = h.x;
    u[t][1] = h.y;
    u[t][2] = h.z;
    deg[t] = h.w;
  }
  int hh[RV];
#pragma unroll
  for (int t = 0; t < RV; ++t) {
    hh[t] = kHead;
#pragma unroll
    for (int i = kHead - 1; i >= 0; --i)
      if (u[t][i] >= 0 && u[t][i] < hotv && ((s_prev[u[t][i] >> 5] >> (u[t][i] & 31)) & 1u))
        hh[t] = i;
  }
  uint32_t cw[RV][kHead];
#pragma unroll
  for (int t = 0; t < RV; ++t)
#pragma unroll
    for (int i = 0; i < kHead; ++i)
      cw[t][i] = (i < hh[t] && u[t][i] >= hotv) ? pbits[u[t][i] >> 5] : 0u;
#pragma unroll
  for (int t = 0; t < RV; ++t) {
    p[t] = hh[t] < kHead ? u[t][hh[t] < kHead ? hh[t] : 0] : -1;
    pos[t] = hh[t];
#pragma unroll
    for (int i = kHead - 1; i >= 0; --i)
      if (i < hh[t] && ((cw[t][i] >> (u[t][i] & 31)) & 1u)) {
        p[t] = u[t][i];
        pos[t] = i;
      }
  }
}

// The rest of the searches head_step left open: for each t with p[t] < 0,
// the adjacencies [o[t] + kHead, end[t]) of its row in order; p[t] = the
// first neighbour one level up and at[t] = its position, or at[t] = end[t].
// Each thread advances its open searches four adjacencies at a time up to
// kSerialScan; the wave finishes the longer ones together, 64 adjacencies
// per step, so every lane of the wave must make the call.
template <int RV>
__device__ __forceinline__ void first_up_rest(const int32_t* __restrict__ col,
                                              const uint32_t* __restrict__ pbits,
                                              const uint32_t* s_prev, int64_t hotv,
                                              int lane, const int32_t (&v)[RV],
                                              const int64_t (&o)[RV], const int64_t (&end)[RV],
                                              int32_t (&p)[RV], int64_t (&at)[RV]) {
#pragma unroll
  for (int t = 0; t < RV; ++t) at[t] = end[t];
  // continuation up to kSerialScan adjacencies, four per step, the RV
  // searches of the thread advancing together (their loads overlap)
  bool pending[RV];
  {
    int64_t e[RV], lim[RV];
#pragma unroll
    for (int t = 0; t < RV; ++t) {
      e[t] = o[t] + kHead;
      lim[t] = min(end[t], o[t] + (int64_t)kSerialScan);
    }
    for (;;) {
      bool any = false;
      int32_t w4[RV][4];
#pragma unroll
      for (int t = 0; t < RV; ++t) {
        const bool act = p[t] < 0 && e[t] < lim[t];
        any |= act;
#pragma unroll
        for (int i = 0; i < 4; ++i) w4[t][i] = (act && e[t] + i < lim[t]) ? col[e[t] + i] : -1;
      }
      if (!any) break;
      uint32_t m4[RV][4];
#pragma unroll
      for (int t = 0; t < RV; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          m4[t][i] = (w4[t][i] >= hotv) ? pbits[w4[t][i] >> 5] : 0u;
#pragma unroll
      for (int t = 0; t < RV; ++t) {
#pragma unroll
        for (int i = 3; i >= 0; --i) {
          const int32_t u = w4[t][i];
          if (u < 0) continue;
          const bool hit = ((u < hotv ? s_prev[u >> 5] : m4[t][i]) >> (u & 31)) & 1u;
          if (hit) {
            p[t] = u;
            at[t] = e[t] + i;
          }
        }
        e[t] += 4;
      }
    }
#pragma unroll
    for (int t = 0; t < RV; ++t)
      pending[t] = v[t] >= 0 && p[t] < 0 && end[t] - o[t] > kSerialScan;
  }
  // the wave scans the rest of each long adjacency list together
#pragma unroll
  for (int t = 0; t < RV; ++t) {
    for (;;) {
      const unsigned long long pend = wave_ballot(pending[t]);
      if (!pend) break;
      const int leader = __ffsll((long long)pend) - 1;
      const int64_t lo = shfl_ll(o[t] + kSerialScan, leader);
      const int64_t hi = shfl_ll(end[t], leader);
      int32_t found = -1;
      int64_t fat = hi;
      for (int64_t e0 = lo; e0 < hi; e0 += 64) {
        const int64_t e = e0 + lane;
        int32_t uu = 0;
        bool hit = false;
        if (e < hi) {
          uu = col[e];
          hit = prev_level(uu, hotv, s_prev, pbits);
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
        p[t] = found;
        at[t] = fat;
        pending[t] = false;
      }
    }
  }
}

// resolve(k), push mark levels: the parent of each vertex of level k's new
// frontier is its first neighbour one level up (level k-1) in ascending
// adjacency order, i.e. the minimum-id frontier vertex adjacent to it. Each
// thread takes RV vertices at once (head_step, then first_up_rest). For a
// large frontier the workgroup first copies the hot prefix of the level-(k-1)
// bitmap into LDS, so most tests (hub neighbours) stay in LDS. It runs at the
// start of level k+1's mark kernel (nothing of level k+1 reads or writes what
// it touches: level k's queue and counter, the level-(k-1) bitmap buffer and
// the words of level k's vertices), which saves a launch per level; a level
// that reached vertices is always followed by another launched level.
constexpr int kResolveBlock = 1024;
constexpr int kResolveRV = 4;

__device__ __forceinline__ void resolve_body(
    int k, const int32_t* __restrict__ col, const int4* __restrict__ head,
    unsigned long long* __restrict__ rpl, const Queues& q, LevelState* st, int cbits,
    const int32_t* __restrict__ inv, int hw, const uint32_t* __restrict__ pbits,
    uint8_t* lds) {
  constexpr int WAVES = kResolveBlock / 64;
  uint32_t* s_prev = reinterpret_cast<uint32_t*>(lds);
  unsigned long long (*s_red)[WAVES] =
      reinterpret_cast<unsigned long long (*)[WAVES]>(lds + kHotWordsMax * 4);
  const unsigned long long cmask = (1ull << cbits) - 1;
  const unsigned long long c = st->ctr[k % 3];
  const int64_t F = (int64_t)(c & cmask);
  const int64_t T = (int64_t)(c >> cbits);
  const int32_t* __restrict__ qv = q.qv[k & 1];
  const int64_t* __restrict__ qo = q.qo[k & 1];
  const int64_t* __restrict__ qe = q.qe[k & 1];
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;
  // stage the hot prefix only when the frontier is large enough to repay it
  const int64_t hotv = F >= ((int64_t)hw << 5) ? ((int64_t)hw << 5) : 0;
  if (hotv) {
    for (int i = tid; i < hw; i += kResolveBlock) s_prev[i] = pbits[i];
    __syncthreads();
  }
  unsigned long long my_cand = 0, my_edges = 0;
  const int64_t chunk = (int64_t)kResolveBlock * kResolveRV;
  const int64_t stride = (int64_t)gridDim.x * chunk;
  for (int64_t base = (int64_t)blockIdx.x * chunk; base < F; base += stride) {
    int32_t v[kResolveRV], p[kResolveRV];
    int64_t o[kResolveRV], end[kResolveRV], at[kResolveRV];
    // queue entries of the RV vertices, loaded together (indices clamped so
    // the loads need no branch; entries past F are dropped)
#pragma unroll
    for (int t = 0; t < kResolveRV; ++t) {
      const int64_t j = base + t * kResolveBlock + tid;
      const int64_t jc = j < F ? j : F - 1;
      const int64_t jn = jc + 1 < F ? jc + 1 : jc;
      const int32_t vj = qv[jc];
      const int64_t oj = qo[jc], e0 = qe[jc], e1 = qe[jn];
      const bool ok = j < F;
      v[t] = ok ? vj : -1;
      o[t] = ok ? oj : 0;
      end[t] = ok ? oj + ((jc + 1 < F ? e1 : T) - e0) : 0;
    }
    int pos[kResolveRV];
    int32_t deg[kResolveRV];
    head_step<kResolveRV>(head, pbits, s_prev, hotv, v, p, pos, deg);
    bool in_head[kResolveRV];
#pragma unroll
    for (int t = 0; t < kResolveRV; ++t) in_head[t] = p[t] >= 0;
    first_up_rest<kResolveRV>(col, pbits, s_prev, hotv, lane, v, o, end, p, at);
#pragma unroll
    for (int t = 0; t < kResolveRV; ++t) {
      if (v[t] < 0) continue;
      ++my_cand;
      my_edges += in_head[t] ? (unsigned long long)(pos[t] + 1)
                             : (p[t] >= 0 ? (unsigned long long)(at[t] - o[t] + 1)
                                          : (unsigned long long)(end[t] - o[t]));
      const int32_t pc = (inv && p[t] >= 0) ? inv[p[t]] : p[t];
      rpl[v[t]] = ((unsigned long long)k << 32) | (uint32_t)pc;
    }
  }
  // statistics of level k: vertices resolved, adjacencies examined
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    my_cand += __shfl_xor(my_cand, d, 64);
    my_edges += __shfl_xor(my_edges, d, 64);
  }
  if (lane == 0) {
    s_red[0][wid] = my_cand;
    s_red[1][wid] = my_edges;
  }
  __syncthreads();
  if (tid == 0 && k < kLevelHist) {
    unsigned long long a = 0, b = 0;
    for (int x = 0; x < WAVES; ++x) {
      a += s_red[0][x];
      b += s_red[1][x];
    }
    if (a) {
      atomicAdd(&st->hist_pc[k], a);
      atomicAdd(&st->hist_pe[k], b);
    }
  }
}

// pull(k), the product of a level computed by rows: every unvisited vertex
// of positive degree searches its ascending adjacency list for the first
// vertex one level up (head_step, first_up_rest), which is its parent; the masked product
// of section 3.2 restricted to the rows the mask leaves, the same entries
// as the push. A vertex that finds one gets its parent and level and is
// marked touched (byte 1) for finish(k). Each wave takes 64 words of the
// visited bitmap (2048 vertices), lists their unvisited vertices in LDS and
// hands them to its lanes RV at a time, so the searches fill the wave.
// It runs inside the mark expand's launch (bfs_mark.hip), one 1024-thread
// workgroup per CU, on that kernel's LDS.
constexpr int kPullBlock = 1024;
// hot prefix staged by the pull: 133.5 KiB of bits, 8 KiB of wave lists and
// 16 KiB of deferred searches (kPullDefer per wave), within the mark
// kernel's LDS (the push level's share, the largest)
constexpr int kPullHotWords = 34176;
constexpr int kPullDefer = 256;
constexpr int kPullLdsBytes = kPullHotWords * 4 + 2 * (kPullBlock / 64) * 64 * 4 +
                              4 * (kPullBlock / 64) * 8 + (kPullBlock / 64) * kPullDefer * 4;
// searches per thread
constexpr int kPullRV = 2;

__device__ __forceinline__ void pull_body(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const int4* __restrict__ head,
    const uint32_t* __restrict__ vis, unsigned long long* __restrict__ rpl,
    uint8_t* __restrict__ mark, LevelState* st, const MarkPolicy& mp,
    const int32_t* __restrict__ inv, int hw, const uint32_t* __restrict__ prev_bits,
    int64_t n_active, uint8_t* lds) {
  constexpr int WAVES = kPullBlock / 64;
  uint32_t* s_prev = reinterpret_cast<uint32_t*>(lds);
  int (*s_exw)[64] = reinterpret_cast<int (*)[64]>(lds + kPullHotWords * 4);
  uint32_t (*s_m)[64] = reinterpret_cast<uint32_t (*)[64]>(lds + kPullHotWords * 4 + WAVES * 256);
  unsigned long long (*s_red)[WAVES] = reinterpret_cast<unsigned long long (*)[WAVES]>(
      lds + kPullHotWords * 4 + 2 * WAVES * 256);
  int32_t (*s_def)[kPullDefer] = reinterpret_cast<int32_t (*)[kPullDefer]>(
      lds + kPullHotWords * 4 + 2 * WAVES * 256 + 4 * WAVES * 8);
  const int k = st->k_fold;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;
  // the hot prefix goes to LDS when the unvisited vertices' adjacencies
  // (what the searches read at most) number at least 4 per staged vertex
  const int hwp = min(hw, kPullHotWords);
  const unsigned long long seen = st->edges;
  const unsigned long long rest =
      (unsigned long long)mp.nnz > seen ? (unsigned long long)mp.nnz - seen : 0ull;
  const int64_t hotv = rest >= ((unsigned long long)hwp << 7) ? ((int64_t)hwp << 5) : 0;
  if (hotv)
    for (int i = tid; i < hwp; i += kPullBlock) s_prev[i] = prev_bits[i];
  __syncthreads();
  const int64_t nw = (n_active + 31) >> 5;
  const int64_t nchunks = (nw + 63) >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * WAVES;
  unsigned long long my_cand = 0, my_edges = 0, my_found = 0, my_fdeg = 0;
  auto found = [&](int32_t v, int32_t p, long long d) {
    const int32_t pc = inv ? inv[p] : p;
    rpl[v] = ((unsigned long long)k << 32) | (uint32_t)pc;
    mark[v] = 1;
    ++my_found;
    my_fdeg += (unsigned long long)d;
  };
  // A search the head entry leaves open waits in the wave's LDS list; the
  // row scans run kPullRV per lane once a full round has gathered, so one
  // long scan does not hold up a round of searches the head copy decides.
  int nd = 0;   // searches in the wave's list (the same in every lane)
  auto scan_deferred = [&](int cnt) {
    int32_t v[kPullRV], p[kPullRV];
    int64_t o[kPullRV], end[kPullRV], at[kPullRV];
#pragma unroll
    for (int t = 0; t < kPullRV; ++t) {
      const int i = t * 64 + lane;
      v[t] = i < cnt ? s_def[wid][i] : -1;
      p[t] = -1;
      o[t] = 0;
      end[t] = 0;
      if (v[t] >= 0) {
        o[t] = off[v[t]];
        end[t] = off[v[t] + 1];
      }
    }
    first_up_rest<kPullRV>(col, prev_bits, s_prev, hotv, lane, v, o, end, p, at);
#pragma unroll
    for (int t = 0; t < kPullRV; ++t) {
      if (v[t] < 0) continue;
      ++my_cand;   // an open search's row is longer than kHead
      my_edges += p[t] >= 0 ? (unsigned long long)(at[t] - o[t] + 1)
                            : (unsigned long long)(end[t] - o[t]);
      if (p[t] >= 0) found(v[t], p[t], end[t] - o[t]);
    }
  };
  for (int64_t c = (int64_t)blockIdx.x * WAVES + wid; c < nchunks; c += nwaves) {
    const int64_t w = (c << 6) + lane;
    uint32_t m = 0u;
    if (w < nw) {
      m = ~vis[w];
      const int64_t left = n_active - (w << 5);   // >= 1 for w < nw
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
    for (int r = 0; r < total; r += 64 * kPullRV) {
      int32_t v[kPullRV], p[kPullRV], deg[kPullRV];
      int pos[kPullRV];
#pragma unroll
      for (int t = 0; t < kPullRV; ++t) {
        const int i = r + t * 64 + lane;
        v[t] = -1;
        if (i < total) {
          int lo = 0;   // last lane whose list starts at or before i
#pragma unroll
          for (int step = 32; step; step >>= 1)
            if (lo + step <= 63 && s_exw[wid][lo + step] <= i) lo += step;
          v[t] = (int32_t)((((c << 6) + lo) << 5) + select_bit(s_m[wid][lo], i - s_exw[wid][lo]));
        }
      }
      head_step<kPullRV>(head, prev_bits, s_prev, hotv, v, p, pos, deg);
#pragma unroll
      for (int t = 0; t < kPullRV; ++t) {
        // open: no frontier vertex among the first kHead adjacencies of a
        // longer row (nd < 64 * kPullRV here, so the list has room)
        const bool open = v[t] >= 0 && p[t] < 0 && deg[t] > kHead;
        const unsigned long long mo = wave_ballot(open);
        if (open) s_def[wid][nd + lanes_below(mo)] = v[t];
        nd += __popcll(mo);
        if (v[t] < 0 || open) continue;
        my_cand += deg[t] > 0;   // vertices of degree 0 have nothing to search
        my_edges += p[t] >= 0 ? (unsigned long long)(pos[t] + 1) : (unsigned long long)deg[t];
        if (p[t] >= 0) found(v[t], p[t], deg[t]);
      }
      if (nd >= 64 * kPullRV) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        scan_deferred(64 * kPullRV);
        // the rest (fewer than a round) moves to the front of the list
        const int left = nd - 64 * kPullRV;
        int32_t keep[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const int i = x * 64 + lane;
          keep[x] = i < left ? s_def[wid][64 * kPullRV + i] : 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const int i = x * 64 + lane;
          if (i < left) s_def[wid][i] = keep[x];
        }
        nd = left;
      }
    }
    // the wave's lists are rewritten by its next chunk
    __builtin_amdgcn_wave_barrier();
  }
  if (nd > 0) {   // the searches left in the list (nd is uniform, so the whole wave scans)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    scan_deferred(nd);
  }
  // statistics: candidates and examined adjacencies of the level
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    my_cand += __shfl_xor(my_cand, d, 64);
    my_edges += __shfl_xor(my_edges, d, 64);
    my_found += __shfl_xor(my_found, d, 64);
    my_fdeg += __shfl_xor(my_fdeg, d, 64);
  }
  if (lane == 0) {
    s_red[0][wid] = my_cand;
    s_red[1][wid] = my_edges;
    s_red[2][wid] = my_found;
    s_red[3][wid] = my_fdeg;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long a = 0, b = 0, f = 0, fd = 0;
    for (int x = 0; x < WAVES; ++x) {
      a += s_red[0][x];
      b += s_red[1][x];
      f += s_red[2][x];
      fd += s_red[3][x];
    }
    if (f) {
      atomicAdd(&st->pull_found, f);
      atomicAdd(&st->pull_found_edges, fd);
    }
    if (b) atomicAdd(&st->pull_edges, b);
    if (k < kLevelHist && a) {
      atomicAdd(&st->hist_pc[k], a);
      atomicAdd(&st->hist_pe[k], b);
    }
  }
}

}  // namespace bfsi
