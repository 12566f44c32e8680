// Device-side level loop for small frontiers (Algorithm 1's level loop with
// the per-level synchronisation of section 2.2 taken inside one workgroup).
//
// The level kernels of bfs_csr.hip spread a level over the whole GPU, which
// pays off when the frontier holds many adjacencies; a level of a few
// thousand adjacencies then costs mostly its three launches. Graphs of high
// diameter (grids, road-like graphs: thousands of levels) and the first and
// last levels of every search are such levels. This kernel runs consecutive
// small claim levels in one 1024-thread workgroup, with the workgroup
// barrier as the level barrier, and hands the search back to the level
// kernels, in exactly the state they expect, once the next level is large
// or needs the mark-and-resolve / pull evaluation.
//
// One level k here: the frontier (level k-1) is staged in LDS (row start,
// exclusive edge prefix, caller id); every thread takes up to kSmallRound of
// the level's adjacencies per round; each phase of a round (adjacencies,
// claims, the owners' rows) issues all of its memory operations before it
// waits, since one workgroup is bound by the latency of their chain. Every
// target takes the (select, min) semiring's claim, a 64-bit atomicMin of
// (k << 32 | caller id of u) on its word, without a filtering read (a word
// set at an earlier level is smaller and stays); the claimer of a fresh word
// appends the vertex to the next queue (one LDS reservation per wave and
// round) with its degree and caller id, sets its visited bit and tag. The
// queue entries carry (degree << 32 | caller id) in the edge prefix slot
// while the loop runs; the hand-off rewrites them as prefixes and builds the
// tile map.
#include "bfs_level.h"

#include <algorithm>

namespace bfsi {
namespace {

constexpr int kSmallBlock = 1024;
constexpr int kSmallMaxF = 8192;                  // frontier entries staged in LDS
constexpr int kSmallMaxT = 16384;                 // adjacencies of a level taken here
constexpr int kSmallRound = 8;                    // adjacencies per thread in flight
constexpr int kSmallSPT = kSmallMaxF / kSmallBlock;   // staged entries per thread

// Block-wide exclusive scan of one value per thread; returns the total.
__device__ __forceinline__ long long small_scan(long long v, long long* s_w, long long& ex) {
  constexpr int WAVES = kSmallBlock / 64;
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const long long incl = wave_incl_scan(v);
  if (lane == 63) s_w[wid] = incl;
  __syncthreads();
  long long b = 0, tot = 0;
#pragma unroll
  for (int x = 0; x < WAVES; ++x) {
    if (x < wid) b += s_w[x];
    tot += s_w[x];
  }
  __syncthreads();
  ex = b + incl - v;
  return tot;
}

__global__ __launch_bounds__(kSmallBlock) void k_small_levels(SmallArgs a) {
  __shared__ uint32_t s_e[kSmallMaxF];     // exclusive edge prefix of the staged frontier
  __shared__ long long s_o[kSmallMaxF];    // row start
  __shared__ uint32_t s_u[kSmallMaxF];     // caller id (the parent the claims select)
  __shared__ long long s_w[kSmallBlock / 64];
  __shared__ int s_cnt;                    // next frontier: entries, their adjacencies
  __shared__ unsigned long long s_tsum;
  __shared__ unsigned int s_own;           // vertices claimed by the level
  LevelState* st = a.st;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const unsigned long long cmask = (1ull << a.cbits) - 1;
  int k = st->k_expand;
  unsigned long long cin = st->ctr[(k - 1) % 3];
  // the launch group this kernel opens (bookkeeping for the per-level record)
  const int grp = st->groups;
  if (tid == 0) {
    st->groups = grp + 1;
    if (grp < kLevelHist) {
      st->grp_level[grp] = 0;
      st->grp_first[grp] = 1;
      st->grp_last[grp] = 0;
    }
  }
  {
    const int64_t F = (int64_t)(cin & cmask), T = (int64_t)(cin >> a.cbits);
    // a pending resolve of a push level (it runs in the next mark kernel) or
    // a level the policy gives to the level kernels: nothing to do here
    if (F == 0 || F > a.max_f || T > a.max_t || st->kind_cur == 1 ||
        mark_level(cin, a.cbits, a.mp) || claim_mark_level(cin, a.cbits, a.mp))
      return;
  }
  bool first = true;
  unsigned long long reached = 0;
  int depth = 0;
  // the levels' edge, frontier and level counts, added to the state at the
  // hand-off (no read of the state on a level's critical path)
  unsigned long long acc_edges = 0, acc_front = 0;
  int acc_levels = 0;
  const int kind_entry = st->kind_cur;
  for (;;) {
    const int F = (int)(cin & cmask);
    const long long T = (long long)(cin >> a.cbits);
    const int kin = k - 1;
    const int32_t* __restrict__ qv_in = a.q.qv[kin & 1];
    const int64_t* __restrict__ qo_in = a.q.qo[kin & 1];
    const int64_t* __restrict__ qe_in = a.q.qe[kin & 1];
    // stage frontier k-1: on entry its queue holds edge prefixes (built by
    // the level kernels), inside the loop (degree << 32 | caller id)
    if (first) {
      for (int j = tid; j < F; j += kSmallBlock) {
        const int32_t v = qv_in[j];
        s_o[j] = qo_in[j];
        s_e[j] = (uint32_t)qe_in[j];
        s_u[j] = (uint32_t)(a.inv ? a.inv[v] : v);
      }
    } else {
      // the thread's entries, all loads issued before any is used (indices
      // past F read entry F - 1 and are dropped)
      unsigned long long w[kSmallSPT];
      long long o[kSmallSPT];
#pragma unroll
      for (int i = 0; i < kSmallSPT; ++i) {
        const int j = min(tid * kSmallSPT + i, F - 1);
        w[i] = (unsigned long long)qe_in[j];
        o[i] = qo_in[j];
      }
      long long d[kSmallSPT];
      long long mine = 0;
#pragma unroll
      for (int i = 0; i < kSmallSPT; ++i) {
        const int j = tid * kSmallSPT + i;
        d[i] = 0;
        if (j < F) {
          d[i] = (long long)(w[i] >> 32);
          s_u[j] = (uint32_t)w[i];
          s_o[j] = o[i];
        }
        mine += d[i];
      }
      long long ex;
      (void)small_scan(mine, s_w, ex);
#pragma unroll
      for (int i = 0; i < kSmallSPT; ++i) {
        const int j = tid * kSmallSPT + i;
        if (j < F) s_e[j] = (uint32_t)ex;
        ex += d[i];
      }
    }
    if (tid == 0) {
      s_cnt = 0;
      s_tsum = 0ull;
      s_own = 0u;
      // the level's bookkeeping, as the expand kernel's
      st->k_fold = k;
      st->levels = k;
      acc_edges += (unsigned long long)T;
      acc_front += (unsigned long long)F;
      ++acc_levels;
      st->pull = 0;
      st->kind_prev = first ? kind_entry : 0;
      st->kind_cur = 0;
      if (k < kLevelHist) {
        st->hist[k] = cin;
        st->hist_mark[k] = 4;
        st->hist_pc[k] = 0ull;
        st->hist_pe[k] = 0ull;
      }
      if (grp < kLevelHist) {
        if (first) st->grp_first[grp] = k;
        st->grp_last[grp] = k;
      }
    }
    __syncthreads();

    // expand: every adjacency of the frontier, in rounds of kSmallRound per
    // thread whose loads are in flight together
    const unsigned long long kk = (unsigned long long)k << 32;
    int32_t* __restrict__ qv_out = a.q.qv[k & 1];
    int64_t* __restrict__ qo_out = a.q.qo[k & 1];
    int64_t* __restrict__ qe_out = a.q.qe[k & 1];
    unsigned int my_own = 0;
    for (long long r0 = 0; r0 < T; r0 += (long long)kSmallRound * kSmallBlock) {
      int32_t vv[kSmallRound], row[kSmallRound];
#pragma unroll
      for (int i = 0; i < kSmallRound; ++i) {
        const long long e = r0 + (long long)i * kSmallBlock + tid;
        vv[i] = -1;
        row[i] = 0;
        if (e < T) {
          int lo = 0, hi = F - 1;   // last row whose prefix is <= e (rows are non-empty)
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if ((long long)s_e[mid] <= e) lo = mid; else hi = mid - 1;
          }
          row[i] = lo;
          vv[i] = a.col[s_o[lo] + (e - (long long)s_e[lo])];
        }
      }
      // the claims: every item issues its atomic (an empty one on the
      // thread's sink word), so the round waits for all of them at once;
      // a target reached earlier keeps its smaller word
      bool own[kSmallRound];
      {
        unsigned long long old[kSmallRound];
#pragma unroll
        for (int i = 0; i < kSmallRound; ++i) {
          const unsigned long long key = kk | s_u[row[i]];
          old[i] = atomicMin(vv[i] >= 0 ? a.rpl + vv[i] : a.st->sink + tid, key);
        }
#pragma unroll
        for (int i = 0; i < kSmallRound; ++i) own[i] = vv[i] >= 0 && old[i] == ~0ull;
      }
      // the owners' rows and caller ids, loaded together (others read
      // vertex 0's and drop them)
      int64_t ob[kSmallRound];
      int32_t dg[kSmallRound];   // degree (< 2^31)
      uint32_t cids[kSmallRound];
      {
        int64_t oe[kSmallRound];
#pragma unroll
        for (int i = 0; i < kSmallRound; ++i) {
          const int32_t vs = own[i] ? vv[i] : 0;
          ob[i] = a.off[vs];
          oe[i] = a.off[vs + 1];
          cids[i] = (uint32_t)(a.inv ? a.inv[vs] : vs);
        }
#pragma unroll
        for (int i = 0; i < kSmallRound; ++i) dg[i] = own[i] ? (int32_t)(oe[i] - ob[i]) : 0;
      }
      // the owners: visited bit and tag; those with adjacencies join the
      // next queue through one LDS reservation per wave and round
      int my_cnt = 0;
      long long my_d = 0;
#pragma unroll
      for (int i = 0; i < kSmallRound; ++i) {
        if (!own[i]) continue;
        const int32_t v = vv[i];
        atomicOr(&a.vis[v >> 5], 1u << (v & 31));
        if (a.mp.symmetric) a.mark[v] = level_tag(k);
        ++my_own;
        if (dg[i] > 0) {
          ++my_cnt;
          my_d += dg[i];
        }
      }
      const long long cincl = wave_incl_scan((long long)my_cnt);
      const long long dincl = wave_incl_scan(my_d);
      int base = 0;
      unsigned long long dbase = 0;
      if (lane == 63 && cincl > 0) {
        base = atomicAdd(&s_cnt, (int)cincl);
        dbase = atomicAdd(&s_tsum, (unsigned long long)dincl);
      }
      (void)dbase;
      base = __shfl(base, 63, 64);
      if (my_cnt > 0) {
        int slot = base + (int)(cincl - my_cnt);
#pragma unroll
        for (int i = 0; i < kSmallRound; ++i) {
          if (dg[i] <= 0) continue;
          qv_out[slot] = vv[i];
          qo_out[slot] = ob[i];
          qe_out[slot] = (int64_t)(((unsigned long long)(uint32_t)dg[i] << 32) | cids[i]);
          ++slot;
        }
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) my_own += __shfl_xor(my_own, d, 64);
    if (lane == 0 && my_own) atomicAdd(&s_own, my_own);
    __syncthreads();
    const int Fn = s_cnt;
    const unsigned long long Tn = s_tsum;
    if (s_own) {
      reached += s_own;
      depth = k;
    }
    const unsigned long long cnext = (Tn << a.cbits) | (unsigned long long)Fn;
    const bool go_on = Fn > 0 && Fn <= a.max_f && (long long)Tn <= a.max_t &&
                       !mark_level(cnext, a.cbits, a.mp) && !claim_mark_level(cnext, a.cbits, a.mp);
    if (!go_on) {
      // hand-off after level k: frontier k as the level kernels build it
      // (queue entries with edge prefixes, tile map, counters)
      if (Fn > 0) {
        int32_t* __restrict__ jstart = a.jstart + (int64_t)(k & 1) * a.njs;
        long long carry = 0;
        for (int base = 0; base < Fn; base += kSmallBlock * kSmallSPT) {
          long long d[kSmallSPT];
          long long mine = 0;
#pragma unroll
          for (int i = 0; i < kSmallSPT; ++i) {
            const int j = base + tid * kSmallSPT + i;
            d[i] = j < Fn ? (long long)((unsigned long long)qe_out[j] >> 32) : 0;
            mine += d[i];
          }
          long long ex;
          const long long tot = small_scan(mine, s_w, ex);
          ex += carry;
#pragma unroll
          for (int i = 0; i < kSmallSPT; ++i) {
            const int j = base + tid * kSmallSPT + i;
            if (j < Fn) {
              qe_out[j] = ex;
              map_tiles(jstart, ex, d[i], j);
            }
            ex += d[i];
          }
          carry += tot;
        }
      }
      if (tid == 0) {
        st->ctr[k % 3] = cnext;
        st->ctr[(k + 1) % 3] = 0ull;
        st->zcnt[k % 3] = 0u;
        st->zcnt[(k + 1) % 3] = 0u;
        st->reached += reached;
        if (depth > st->depth) st->depth = depth;
        st->edges += acc_edges;
        st->frontier_total += acc_front;
        st->small_levels += acc_levels;
        st->k_expand = k + 1;
      }
      return;
    }
    __syncthreads();
    first = false;
    cin = cnext;
    ++k;
  }
}

}  // namespace

void small_levels_launch(hipStream_t s, const SmallArgs& a) {
  k_small_levels<<<1, kSmallBlock, 0, s>>>(a);
}

int64_t small_max_frontier() { return kSmallMaxF; }
int64_t small_max_edges() { return kSmallMaxT; }

}  // namespace bfsi
