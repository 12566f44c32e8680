// BFS over a p_r x p_c grid of DCSC shares on one GPU: the 2D-partitioned
// algorithm (Algorithm 3, section 3.2) with every share resident on the
// device and the collectives replaced by device gathers. Per level:
//
//   column gather   the sorted frontier (global ids) is split by column
//                   block; each piece is turned into local column ids and
//                   keeps the global ids as the selected values
//   local product   bfs_spmspv on each share (section 4.2's SPA or sort
//                   path): per row, the minimum global id of the frontier
//                   columns that reach it
//   row fold        every share's output is folded with min into a
//                   candidate array over global rows, for rows not yet
//                   reached (the mask of unvisited vertices)
//   apply           a scan of the candidate bitmap gives the new vertices in
//                   ascending order: parent = candidate, level = k, and the
//                   next frontier (pi <- pi + t, f <- t)
#include "bfs_internal.h"

#include <algorithm>
#include <mutex>
#include <vector>

namespace bfsi {
namespace {

constexpr int kApplyBlock = 256;
constexpr int kApplyWords = 8;   // bitmap words per thread
constexpr int kApplyPerBlock = kApplyBlock * kApplyWords;

__global__ void k2_init(int64_t n, int32_t* __restrict__ parent, int32_t* __restrict__ level,
                        int32_t* __restrict__ cand, uint32_t* __restrict__ newbit,
                        int64_t nwords, int32_t root, int32_t* __restrict__ f) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    parent[v] = v == root ? root : -1;
    if (level) level[v] = v == root ? 0 : -1;
    cand[v] = 0x7FFFFFFF;
  }
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < nwords; w += stride)
    newbit[w] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) f[0] = root;
}

// Local column id of every frontier entry, and bounds[j] = first entry of
// column block j (bounds[pc] = F).
__global__ void k2_split(const int32_t* __restrict__ f, int64_t F, int64_t C, int pc,
                         int32_t* __restrict__ fl, int64_t* __restrict__ bounds) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < F; t += stride)
    fl[t] = (int32_t)(f[t] - (f[t] / C) * C);
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j <= pc; j += blockDim.x) {
      const int64_t key = (int64_t)j * C;
      int64_t lo = 0, hi = F;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)f[mid] < key) lo = mid + 1; else hi = mid;
      }
      bounds[j] = j == pc ? F : lo;
    }
}

// One share's product folded into the candidates of unreached global rows.
__global__ void k2_fold(int64_t cnt, const int32_t* __restrict__ oidx,
                        const int32_t* __restrict__ oval, int64_t row0,
                        const int32_t* __restrict__ parent, int32_t* __restrict__ cand,
                        uint32_t* __restrict__ newbit) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < cnt; e += stride) {
    const int64_t g = row0 + oidx[e];
    if (parent[g] != -1) continue;
    const int32_t v = oval[e];
    if (cand[g] > v) atomicMin(&cand[g], v);
    const uint32_t bit = 1u << (g & 31);
    if (!(newbit[g >> 5] & bit)) atomicOr(&newbit[g >> 5], bit);
  }
}

__global__ __launch_bounds__(kApplyBlock) void k2_count(const uint32_t* __restrict__ newbit,
                                                        int64_t nwords,
                                                        int64_t* __restrict__ blk) {
  const int64_t w0 = blockIdx.x * (int64_t)kApplyPerBlock + threadIdx.x * kApplyWords;
  int c = 0;
#pragma unroll
  for (int i = 0; i < kApplyWords; ++i)
    if (w0 + i < nwords) c += __popc(newbit[w0 + i]);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  __shared__ int s[kApplyBlock / 64];
  if (lane_id() == 0) s[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int x = 0; x < kApplyBlock / 64; ++x) t += s[x];
    blk[blockIdx.x] = t;
  }
}

// Exclusive scan of the block counts in one workgroup; total -> *total.
__global__ void k2_scan(int64_t* __restrict__ blk, int64_t nblk, int64_t* __restrict__ total) {
  __shared__ long long s_carry;
  __shared__ long long s_w[4];
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nblk; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const long long v = i < nblk ? blk[i] : 0;
    const long long incl = wave_incl_scan(v);
    const int wid = threadIdx.x >> 6;
    if (lane_id() == 63) s_w[wid] = incl;
    __syncthreads();
    long long wb = 0, tot = 0;
    for (int x = 0; x < (int)(blockDim.x >> 6); ++x) {
      if (x < wid) wb += s_w[x];
      tot += s_w[x];
    }
    const long long carry = s_carry;
    if (i < nblk) blk[i] = carry + wb + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = s_carry;
}

// New vertices in ascending order: parent, level, next frontier; the
// candidate entries and bits are reset.
__global__ __launch_bounds__(kApplyBlock) void k2_apply(
    uint32_t* __restrict__ newbit, int64_t nwords, int32_t* __restrict__ cand,
    const int64_t* __restrict__ blk, int32_t k, int32_t* __restrict__ parent,
    int32_t* __restrict__ level, int32_t* __restrict__ fnext) {
  const int64_t w0 = blockIdx.x * (int64_t)kApplyPerBlock + threadIdx.x * kApplyWords;
  uint32_t words[kApplyWords];
  int c = 0;
#pragma unroll
  for (int i = 0; i < kApplyWords; ++i) {
    words[i] = (w0 + i < nwords) ? newbit[w0 + i] : 0u;
    c += __popc(words[i]);
  }
  const long long incl = wave_incl_scan(c);
  __shared__ long long s_w[kApplyBlock / 64];
  const int wid = threadIdx.x >> 6;
  if (lane_id() == 63) s_w[wid] = incl;
  __syncthreads();
  long long wb = 0;
  for (int x = 0; x < wid; ++x) wb += s_w[x];
  long long pos = blk[blockIdx.x] + wb + incl - c;
#pragma unroll
  for (int i = 0; i < kApplyWords; ++i) {
    uint32_t bits = words[i];
    if (!bits) continue;
    while (bits) {
      const int b = __ffs(bits) - 1;
      bits &= bits - 1;
      const int64_t g = ((w0 + i) << 5) + b;
      parent[g] = cand[g];
      if (level) level[g] = k;
      cand[g] = 0x7FFFFFFF;
      fnext[pos++] = (int32_t)g;
    }
    newbit[w0 + i] = 0u;
  }
}


bool on_device(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Device pointers of one run's workspace (about 24 n bytes).
struct View2d {
  int32_t *f, *fnext, *fl, *cand, *oidx, *oval;
  uint32_t* newbit;
  int64_t *bounds, *blk, *total;
};

// Bytes of that workspace, carved in 256-byte aligned pieces.
int64_t ws2d_bytes(int64_t n, int64_t max_rows, int pc) {
  auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t nwords = (n + 31) / 32;
  const int64_t nblk = (nwords + kApplyPerBlock - 1) / kApplyPerBlock;
  return 4 * al(n * 4) + 2 * al(max_rows * 4) + al(nwords * 4) + al((int64_t)(pc + 1) * 8) +
         al(std::max<int64_t>(nblk, 1) * 8) + al(8);
}

View2d ws2d_carve(char* base, int64_t n, int64_t max_rows, int pc) {
  auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t nwords = (n + 31) / 32;
  const int64_t nblk = (nwords + kApplyPerBlock - 1) / kApplyPerBlock;
  View2d v;
  char* p = base;
  auto take = [&](int64_t bytes) {
    char* q = p;
    p += al(bytes);
    return q;
  };
  v.f = reinterpret_cast<int32_t*>(take(n * 4));
  v.fnext = reinterpret_cast<int32_t*>(take(n * 4));
  v.fl = reinterpret_cast<int32_t*>(take(n * 4));
  v.cand = reinterpret_cast<int32_t*>(take(n * 4));
  v.oidx = reinterpret_cast<int32_t*>(take(max_rows * 4));
  v.oval = reinterpret_cast<int32_t*>(take(max_rows * 4));
  v.newbit = reinterpret_cast<uint32_t*>(take(nwords * 4));
  v.bounds = reinterpret_cast<int64_t*>(take((int64_t)(pc + 1) * 8));
  v.blk = reinterpret_cast<int64_t*>(take(std::max<int64_t>(nblk, 1) * 8));
  v.total = reinterpret_cast<int64_t*>(take(8));
  return v;
}

constexpr int kMaxShares = 1024;

// Checks the arguments of a 2D run and collects the shares (row-major) and
// their largest row count; every share must have the shape of its block.
int check_2d(bfs_graph_t* const* shares, int32_t pr, int32_t pc, int64_t n, int32_t root,
             int32_t* parent, int32_t* level, bfs_graph** all, int64_t* max_rows) {
  if (!shares || !parent || pr < 1 || pc < 1 || n < 1 || n >= ((int64_t)1 << 31))
    return fail(BFS_ERR_ARG, "bad arguments to bfs_run_2d");
  if ((int64_t)pr * pc > kMaxShares)
    return fail(BFS_ERR_UNSUPPORTED, "at most 1024 shares in a 2D grid");
  if (root < 0 || (int64_t)root >= n) return fail(BFS_ERR_ARG, "root out of range");
  const int64_t R = (n + pr - 1) / pr, C = (n + pc - 1) / pc;
  if ((int64_t)(pr - 1) * R >= n || (int64_t)(pc - 1) * C >= n)
    return fail(BFS_ERR_ARG, "every share needs at least one row and one column");
  *max_rows = 1;
  for (int i = 0; i < pr; ++i)
    for (int j = 0; j < pc; ++j) {
      bfs_graph* g = shares[(size_t)i * pc + j];
      if (!g || g->kind != kDcsc) return fail(BFS_ERR_ARG, "every share must be a DCSC handle");
      const int64_t nr = std::min<int64_t>(R, n - i * R), nc = std::min<int64_t>(C, n - j * C);
      if (g->dcsc.nrows != nr || g->dcsc.ncols != nc)
        return fail(BFS_ERR_ARG, "share shape does not match the p_r x p_c split of n");
      all[(size_t)i * pc + j] = g;
      *max_rows = std::max<int64_t>(*max_rows, nr);
    }
  const int cnt = pr * pc;
  std::sort(all, all + cnt);
  if (std::adjacent_find(all, all + cnt) != all + cnt)
    return fail(BFS_ERR_ARG, "the same handle appears twice in the share grid");
  if (!on_device(parent) || (level && !on_device(level)))
    return fail(BFS_ERR_ARG, "bfs_run_2d needs device output arrays");
  return BFS_OK;
}

// The level loop of a 2D run on a carved workspace; h holds pc + 2 host
// int64 (the column bounds, then the frontier size). Allocates nothing.
int run_2d_core(bfs_graph_t* const* shares, int32_t pr, int32_t pc, int64_t n, int32_t root,
                int32_t* parent, int32_t* level, int64_t max_rows, const View2d& w, int64_t* h,
                hipStream_t s) {
  const int64_t R = (n + pr - 1) / pr, C = (n + pc - 1) / pc;
  const int64_t nwords = (n + 31) / 32;
  const int64_t nblk = (nwords + kApplyPerBlock - 1) / kApplyPerBlock;
  const int ib = 256;
  const int igrid = (int)std::min<int64_t>((n + ib - 1) / ib, 8192);
  int32_t* f = w.f;
  int32_t* fnext = w.fnext;
  k2_init<<<igrid, ib, 0, s>>>(n, parent, level, w.cand, w.newbit, nwords, root, f);
  BFS_HIP(hipGetLastError());
  int64_t F = 1;
  for (int32_t k = 1; F > 0; ++k) {
    const int sgrid = (int)std::min<int64_t>((F + ib - 1) / ib, 4096);
    k2_split<<<sgrid, ib, 0, s>>>(f, F, C, pc, w.fl, w.bounds);
    BFS_HIP(hipMemcpyAsync(h, w.bounds, (size_t)(pc + 1) * 8, hipMemcpyDeviceToHost, s));
    BFS_HIP(wait_stream(s));
    for (int j = 0; j < pc; ++j) {
      const int64_t lo = h[j], hi = h[j + 1];
      if (hi <= lo) continue;
      for (int i = 0; i < pr; ++i) {
        bfs_svec_t fv{hi - lo, hi - lo, w.fl + lo, f + lo};
        bfs_svec_t out{0, max_rows, w.oidx, w.oval};
        const int rc = dcsc_spmspv(shares[(size_t)i * pc + j], &fv, &out, s);
        if (rc != BFS_OK) return rc;
        if (out.nnz > 0) {
          const int fgrid = (int)std::min<int64_t>((out.nnz + ib - 1) / ib, 4096);
          k2_fold<<<fgrid, ib, 0, s>>>(out.nnz, w.oidx, w.oval, (int64_t)i * R, parent, w.cand,
                                       w.newbit);
        }
      }
    }
    k2_count<<<(int)nblk, kApplyBlock, 0, s>>>(w.newbit, nwords, w.blk);
    k2_scan<<<1, 256, 0, s>>>(w.blk, nblk, w.total);
    k2_apply<<<(int)nblk, kApplyBlock, 0, s>>>(w.newbit, nwords, w.cand, w.blk, k, parent,
                                               level, fnext);
    BFS_HIP(hipGetLastError());
    BFS_HIP(hipMemcpyAsync(h + pc + 1, w.total, 8, hipMemcpyDeviceToHost, s));
    BFS_HIP(wait_stream(s));
    F = h[pc + 1];
    std::swap(f, fnext);
    if (k > n + 1) return fail(BFS_ERR_DEVICE, "2D level loop did not terminate");
  }
  return BFS_OK;
}

// ------------------------------------------------------------ no-allocation entry
// Workspace of bfs_run_2d_noalloc: a file-scope device array, one copy per
// GPU for the life of the process, shared by every call on that GPU (its
// contents are whatever the last call left; each call initialises what it
// reads). Host code reaches it only through the per-device address from
// hipGetSymbolAddress; the array's name is not a device address there.
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 20;
constexpr int kNoAllocMaxPc = 256;
constexpr int64_t kScratchBytes = 26 * ((int64_t)1 << 20);
static_assert(kScratchBytes >= 4 * kNoAllocMaxN * 4 + 2 * kNoAllocMaxN * 4 +
                                   kNoAllocMaxN / 8 + 10 * 256 + (kNoAllocMaxPc + 1) * 8 + 4096,
              "scratch holds the workspace of the largest accepted run");
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {nullptr};

// The calling thread's current device's copy of `scratch`, looked up once
// per device with that device current.
int scratch_for_device(char** out) {
  int dev = 0;
  BFS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(BFS_ERR_UNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return BFS_OK;
}

}  // namespace
}  // namespace bfsi

using namespace bfsi;

extern "C" int bfs_run_2d(bfs_graph_t* const* shares, int32_t pr, int32_t pc, int64_t n,
                          int32_t root, int32_t* parent, int32_t* level, void* hip_stream) {
  bfs_graph* all[kMaxShares];
  int64_t max_rows = 1;
  int rc = check_2d(shares, pr, pc, n, root, parent, level, all, &max_rows);
  if (rc != BFS_OK) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    // the shares' accumulators are used by this run: hold their run locks
    // (taken in address order)
    std::vector<std::unique_lock<std::mutex>> locks;
    for (int i = 0; i < pr * pc; ++i) locks.emplace_back(all[i]->run_mu);
    char* ws = nullptr;
    BFS_HIP(hipMalloc(&ws, (size_t)ws2d_bytes(n, max_rows, pc)));
    int64_t* h = nullptr;
    hipError_t e = hipHostMalloc(&h, (size_t)(pc + 2) * 8, hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipFree(ws);
      return hip_fail(e, "hipHostMalloc");
    }
    rc = run_2d_core(shares, pr, pc, n, root, parent, level, max_rows,
                     ws2d_carve(ws, n, max_rows, pc), h, s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(ws);
    (void)hipHostFree(h);
    return rc;
  } catch (...) {
    return fail(BFS_ERR_DEVICE, "exception in bfs_run_2d");
  }
}

extern "C" int bfs_run_2d_noalloc(bfs_graph_t* const* shares, int32_t pr, int32_t pc,
                                  int64_t n, int32_t root, int32_t* parent, int32_t* level,
                                  void* hip_stream) {
  bfs_graph* all[kMaxShares];
  int64_t max_rows = 1;
  int rc = check_2d(shares, pr, pc, n, root, parent, level, all, &max_rows);
  if (rc != BFS_OK) return rc;
  if (n > kNoAllocMaxN)
    return fail(BFS_ERR_CAPACITY, "bfs_run_2d_noalloc: n above 2^20 (its fixed workspace); "
                                  "use bfs_run_2d");
  if (pc > kNoAllocMaxPc)
    return fail(BFS_ERR_CAPACITY, "bfs_run_2d_noalloc: more than 256 column blocks");
  if (ws2d_bytes(n, max_rows, pc) > kScratchBytes)
    return fail(BFS_ERR_CAPACITY, "bfs_run_2d_noalloc: workspace exceeds the fixed scratch");
  hipStream_t s = (hipStream_t)hip_stream;
  try {
    char* ws = nullptr;
    rc = scratch_for_device(&ws);
    if (rc != BFS_OK) return rc;
    std::unique_lock<std::mutex> locks[kMaxShares];
    for (int i = 0; i < pr * pc; ++i) locks[i] = std::unique_lock<std::mutex>(all[i]->run_mu);
    int64_t h[kNoAllocMaxPc + 2];   // column bounds and frontier size (host stack)
    return run_2d_core(shares, pr, pc, n, root, parent, level, max_rows,
                       ws2d_carve(ws, n, max_rows, pc), h, s);
  } catch (...) {
    return fail(BFS_ERR_DEVICE, "exception in bfs_run_2d_noalloc");
  }
}
