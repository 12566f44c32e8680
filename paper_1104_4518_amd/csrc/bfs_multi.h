// Query descriptors and launchers of the multi-query kernel (bfs_multi.hip),
// used by bfs_run_batch and by the continuous-batching server.
#pragma once

#include "bfs_internal.h"

namespace bfsi {

constexpr int kMultiWG = 512;          // threads per workgroup (8 waves of 64)
constexpr int kLdsWords = 16384;       // 64 KiB LDS bitmap: graphs up to 2^19 vertices

enum QueryStatus : int32_t { kQueryPending = 0, kQueryRunning = 1, kQueryDone = 2 };

// One query as the device sees it. The host fills the inputs and the
// workspace pointers; the kernel owns k, F, edges, depth and status.
struct MQuery {
  const int64_t* off;
  const int32_t* col;
  int32_t* parent;
  int32_t* level;       // may be null
  int32_t* q[2];        // two frontier queues of n entries
  uint32_t* vis;        // ceil(n / 32) words (unused for LDS-mode graphs in batches)
  int32_t n;
  int32_t root;
  int32_t k;            // level of the current frontier
  int32_t F;            // its size
  unsigned long long edges;
  int32_t depth;
  int32_t status;
};

const void* multi_kernel();
int multi_grid(int device);
int multi_reset_counter(int32_t* d_counter, hipStream_t s);
// pull: workgroups take queries from *d_counter until `count` (run to
// completion, budget ignored when 0); otherwise workgroup i runs order[i].
// ws_base != null: workgroup b uses the workspace at ws_base + b * ws_stride
// (two queues of ws_qbytes, then the bitmap) instead of the query's own.
int multi_launch(MQuery* d_qs, const int32_t* d_order, int32_t count, int32_t* d_counter,
                 int grid, bool pull, unsigned long long budget, char* ws_base,
                 int64_t ws_stride, int64_t ws_qbytes, hipStream_t s);

// Bytes of one frontier queue / of the bitmap for a graph of n vertices
// (256-byte aligned).
inline int64_t multi_q_bytes(int64_t n) { return ((n * 4 + 255) / 256) * 256; }
inline int64_t multi_vis_bytes(int64_t n) { return ((((n + 31) / 32) * 4 + 255) / 256) * 256; }
inline int64_t multi_ws_bytes(int64_t n) { return 2 * multi_q_bytes(n) + multi_vis_bytes(n); }

}  // namespace bfsi
