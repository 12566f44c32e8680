// Definitions shared by the CSR level kernels (bfs_csr.hip) and the
// mark-and-resolve expand kernel (bfs_mark.hip): launch constants, the
// frontier queues, the per-level choice between the two ways of claiming new
// vertices, and the mark-byte tags.
#pragma once

#include "bfs_internal.h"

namespace bfsi {

// jstart granularity and claim-path tile: 1024 edges (256 threads x 4)
constexpr int kTileJ = 1024;
// mark path: one 1024-thread workgroup per CU, each wave on its own
// 1024-edge tiles
constexpr int kMarkBlock = 1024;
// Hot prefix of the visited bitmap kept in LDS by the mark path: the first
// 39936 * 32 vertices (156 KiB of the CU's 160 KiB; the rest holds the
// waves' row-start masks). In a degree-ordered copy these are the
// highest-degree vertices, the targets of most probes.
constexpr int kHotWordsMax = 39936;
// mark-and-resolve: vertices of degree above this search their parent with
// the whole wave instead of one thread
constexpr int kSerialScan = 64;

// Mark bytes: 0 = not reached, 1 = touched by the current level's frontier,
// 2 + (level mod 3) = reached at that level. A neighbour of a vertex at level
// k lies at level k-1, k or k+1 (or is unreached), so the tag identifies
// "one level up" exactly.
__device__ __forceinline__ uint8_t level_tag(int k) { return (uint8_t)(2 + k % 3); }

// Map the edge tiles of the next level that start inside [e, e + d) to
// queue entry j.
__device__ __forceinline__ void map_tiles(int32_t* __restrict__ jstart, long long e, long long d,
                                          int32_t j) {
  for (long long w = (e + kTileJ - 1) / kTileJ; w * kTileJ < e + d; ++w) jstart[w] = j;
}

struct Queues {
  int32_t* qv[2];
  int64_t* qo[2];
  int64_t* qe[2];
};

// Level selection: mark-and-resolve when the graph is symmetric and the
// input frontier is large in both edges and vertices (a small frontier makes
// every new vertex search far for one of its few frontier neighbours), or
// whatever its vertex count when pull_alpha times its adjacencies reach
// all of the graph's: such a level always pulls (below), and a frontier of
// a few hubs is where pulling pays most, since the unvisited vertices find
// a hub among their first neighbours.
struct MarkPolicy {
  int symmetric;
  long long min_edges;
  long long min_vertices;
  // a mark level pulls (computes its product by rows) when
  // pull_alpha * frontier adjacencies >= adjacencies not yet visited;
  // 0 = never
  long long nnz;
  int pull_alpha;
};

__device__ __forceinline__ bool mark_level(unsigned long long cin, int cbits,
                                           const MarkPolicy& mp) {
  const unsigned long long cmask = (1ull << cbits) - 1;
  const long long F = (long long)(cin & cmask), T = (long long)(cin >> cbits);
  return mp.symmetric && F > 0 && T >= mp.min_edges &&
         (F >= mp.min_vertices ||
          (mp.pull_alpha > 0 && T >= (mp.nnz + mp.pull_alpha - 1) / mp.pull_alpha));
}

// A large claim level on a symmetric graph whose frontier holds at least
// 1/64 of the adjacencies spread over many vertices (at most 128 per
// frontier vertex on average, so most targets are new and reached once):
// every edge to an unvisited target does a 64-bit atomicMin whose result is
// not waited for; finish then collects the level's vertices in vertex order,
// as on mark levels, by the level in their words, with the parents already
// final. Saves the per-edge ownership test and appends. A frontier of a few
// hubs instead reaches each target many times, and there the claim's plain
// read before the atomic filters most of them.
__device__ __forceinline__ bool claim_mark_level(unsigned long long cin, int cbits,
                                                 const MarkPolicy& mp) {
  const unsigned long long cmask = (1ull << cbits) - 1;
  const long long F = (long long)(cin & cmask), T = (long long)(cin >> cbits);
  return mp.symmetric && F > 0 && !mark_level(cin, cbits, mp) && T * 64 >= mp.nnz &&
         T <= 128 * F;
}

// Direction of a mark level's product with input counter cin: by rows (pull)
// once pull_alpha times the frontier's adjacencies reach those of the
// vertices still unvisited, which the searches read at most; seen = the
// adjacencies of every visited vertex, the frontier's included. The level's
// own expand decides, and the finish of a pull level decides ahead for the
// next one from the same inputs.
__device__ __forceinline__ bool pull_level(unsigned long long cin, int cbits,
                                           unsigned long long seen, const MarkPolicy& mp) {
  if (!mark_level(cin, cbits, mp) || mp.pull_alpha <= 0) return false;
  const unsigned long long T = cin >> cbits;
  const unsigned long long rest =
      (unsigned long long)mp.nnz > seen ? (unsigned long long)mp.nnz - seen : 0ull;
  const unsigned long long a = (unsigned long long)mp.pull_alpha;
  return T >= (rest + a - 1) / a;
}


// The mark-level kernel (bfs_mark.hip): on a push level the mark expand, on
// a pull level the pull; one 1024-thread workgroup per CU (its LDS holds
// the hot prefix of a bitmap). probe: 0 = by reached fraction, 1 = mark
// byte, 2 = visited word first (push levels).
struct MarkArgs {
  const int32_t* col;
  const int64_t* off;
  const int4* head;
  const uint32_t* vis;
  uint8_t* mark;
  unsigned long long* rpl;
  const int32_t* inv;
  Queues q;
  const int32_t* jstart;
  int64_t njs;
  LevelState* st;
  int cbits;
  MarkPolicy mp;
  int hw;
  uint32_t* hot_new;
  const uint32_t* prev_bits;
  int64_t n, n_active, nwords;
  int probe;
};
int mark_expand_grid(int device);

// The device level loop for small frontiers (bfs_small.hip): one workgroup
// runs claim levels while a level's frontier holds at most max_f vertices and
// max_t adjacencies (at most small_max_frontier() / small_max_edges()).
struct SmallArgs {
  const int64_t* off;
  const int32_t* col;
  uint32_t* vis;
  unsigned long long* rpl;
  uint8_t* mark;
  const int32_t* inv;
  Queues q;
  int32_t* jstart;
  int64_t njs;
  LevelState* st;
  int cbits;
  MarkPolicy mp;
  int64_t max_f, max_t;
};
void small_levels_launch(hipStream_t s, const SmallArgs& a);
int64_t small_max_frontier();
int64_t small_max_edges();
void mark_expand_launch(int grid, hipStream_t s, const MarkArgs& a);

}  // namespace bfsi
