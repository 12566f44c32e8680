// C ABI entry points: argument checks, handle lifetime, uploads, dispatch.
// Every entry point returns a status and never lets an exception escape.
#include "bfs_internal.h"

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

namespace bfsi {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  (void)hipGetLastError();
  return e == hipErrorOutOfMemory ? BFS_ERR_OOM : BFS_ERR_DEVICE;
}

hipError_t wait_stream(hipStream_t s) {
  for (;;) {
    const hipError_t e = hipStreamQuery(s);
    if (e != hipErrorNotReady) return e;
    __builtin_ia32_pause();
  }
}

int csr_widen(const int32_t* d_src32, int64_t n1, int64_t* d_dst, hipStream_t s);

namespace {

int copy_in(void* dst, const void* src, size_t bytes, bool device_src, hipStream_t s) {
  if (bytes == 0) return BFS_OK;
  BFS_HIP(hipMemcpyAsync(dst, src, bytes,
                         device_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  return BFS_OK;
}

int ceil_log2_plus(int64_t n) {
  int b = 1;
  while (b < 63 && ((int64_t)1 << b) <= n) ++b;
  return b;
}

void default_options(bfs_options_t* o) {
  o->mode = 1;
  o->batch_levels = 4;
  o->grid_blocks = 0;
  o->lds_bitmap = 0;
  o->profile = -1;
  o->claim = 3;
  o->claim_threshold = 0;
  o->claim_min_frontier = 0;
  o->cold_probe = 3;
  o->spmspv_sort_max = 512;
  o->pull_alpha = 14;
  o->small_frontier = 0;
}

}  // namespace
}  // namespace bfsi

using namespace bfsi;

extern "C" {

const char* bfs_last_error(void) { return g_last_error.c_str(); }

const char* bfs_version(void) { return "bfs-mi355x 0.1 (gfx950)"; }

int bfs_graph_create_csr(int64_t n, int64_t nnz, const void* row_offsets, int offset_bytes,
                         const int32_t* col_idx, uint32_t flags, bfs_graph_t** out) {
  try {
    if (!out) return fail(BFS_ERR_ARG, "out handle pointer is NULL");
    *out = nullptr;
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(BFS_ERR_ARG, "n must be in [1, 2^31)");
    if (nnz < 0) return fail(BFS_ERR_ARG, "nnz must be >= 0");
    if (!row_offsets || (nnz > 0 && !col_idx)) return fail(BFS_ERR_ARG, "NULL input array");
    if (offset_bytes != 4 && offset_bytes != 8)
      return fail(BFS_ERR_ARG, "offset_bytes must be 4 or 8");
    if (offset_bytes == 4 && nnz >= ((int64_t)1 << 31))
      return fail(BFS_ERR_ARG, "nnz does not fit 32-bit offsets");
    const int cbits = ceil_log2_plus(n);
    if (cbits >= 62 || (nnz >> (64 - cbits)) != 0)
      return fail(BFS_ERR_UNSUPPORTED, "nnz too large for the packed frontier counter");
    const bool dev = (flags & BFS_DEVICE_PTRS) != 0;

    bfs_graph* g = new (std::nothrow) bfs_graph();
    if (!g) return fail(BFS_ERR_OOM, "host allocation failed");
    (void)hipGetDevice(&g->device);
    g->kind = kCsr;
    default_options(&g->opt);
    CsrDev& c = g->csr;
    c.n = n;
    c.nnz = nnz;
    c.cbits = cbits;
    hipStream_t s = nullptr;
    int rc = BFS_OK;
    auto bail = [&](int code) {
      csr_free(g);
      if (g->h_ctr) (void)hipHostFree(g->h_ctr);
      delete g;
      return code;
    };
    hipError_t e = hipMalloc(&c.off, (size_t)(n + 1) * 8);
    if (e == hipSuccess) e = hipMalloc(&c.col, (size_t)std::max<int64_t>(nnz, 1) * 4);
    if (e != hipSuccess) return bail(hip_fail(e, "allocating CSR arrays"));
    g->device_bytes = (n + 1) * 8 + std::max<int64_t>(nnz, 1) * 4;
    if (offset_bytes == 8) {
      rc = copy_in(c.off, row_offsets, (size_t)(n + 1) * 8, dev, s);
    } else if (dev) {
      rc = csr_widen(static_cast<const int32_t*>(row_offsets), n + 1, c.off, s);
    } else {
      std::vector<int64_t> w((size_t)(n + 1));
      const int32_t* src = static_cast<const int32_t*>(row_offsets);
      for (int64_t i = 0; i <= n; ++i) w[(size_t)i] = src[i];
      rc = copy_in(c.off, w.data(), w.size() * 8, false, s);
      if (rc == BFS_OK) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "upload");
      }
    }
    if (rc == BFS_OK) rc = copy_in(c.col, col_idx, (size_t)nnz * 4, dev, s);
    if (rc == BFS_OK) {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = hip_fail(e, "upload");
    }
    if (rc == BFS_OK && !(flags & BFS_TRUSTED)) rc = csr_validate(g, s);
    const bool upper = (flags & BFS_UPPER) != 0;
    if (rc == BFS_OK && upper) {
      // the symmetric closure is searched; the stored half is traversed in
      // its own ids (no degree-ordered copy, which would double it)
      c.upper = 1;
      if (!(flags & BFS_TRUSTED)) {
        int ok = 0;
        rc = csr_check_upper(g, s, &ok);
        if (rc == BFS_OK && !ok)
          rc = fail(BFS_ERR_FORMAT,
                    "BFS_UPPER: every adjacency v of row u must satisfy v > u, rows ascending");
      }
    } else if (rc == BFS_OK) {
      if (flags & BFS_SYMMETRIC) c.symmetric = 1;
      else if (!(flags & BFS_TRUSTED)) rc = csr_check_symmetric(g, s, &c.symmetric);
    }
    // degree-ordered copy for the level kernels (large graphs)
    if (rc == BFS_OK && !upper && !(flags & BFS_NO_RELABEL) && n >= ((int64_t)1 << 20) &&
        nnz > 0) {
      std::vector<int64_t> hoff;
      const int64_t* ho = nullptr;
      if (offset_bytes == 8 && !dev) {
        ho = static_cast<const int64_t*>(row_offsets);
      } else {
        hoff.resize((size_t)(n + 1));
        e = hipMemcpy(hoff.data(), c.off, hoff.size() * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = hip_fail(e, "offsets readback");
        ho = hoff.data();
      }
      if (rc == BFS_OK) rc = csr_relabel(g, ho, s);
    }
    if (rc == BFS_OK) rc = csr_alloc_workspace(g);
    if (rc == BFS_OK) {
      e = hipHostMalloc(&g->h_ctr, 16 * sizeof(unsigned long long), hipHostMallocDefault);
      if (e != hipSuccess) rc = hip_fail(e, "pinned counter");
    }
    if (rc != BFS_OK) return bail(rc);
    *out = g;
    return BFS_OK;
  } catch (...) {
    return fail(BFS_ERR_OOM, "exception during create");
  }
}

int bfs_graph_create_dcsc(int32_t nrows, int32_t ncols, int32_t nzc, int64_t nnz,
                          const int32_t* jc, const int32_t* cp, const int32_t* ir,
                          uint32_t flags, bfs_graph_t** out) {
  try {
    if (!out) return fail(BFS_ERR_ARG, "out handle pointer is NULL");
    *out = nullptr;
    if (nrows < 0 || ncols < 0 || nzc < 0 || nnz < 0)
      return fail(BFS_ERR_ARG, "negative DCSC size");
    if (nnz >= ((int64_t)1 << 31)) return fail(BFS_ERR_UNSUPPORTED, "nnz must be < 2^31");
    if (nzc > ncols || (int64_t)nzc > nnz) return fail(BFS_ERR_FORMAT, "nzc exceeds ncols or nnz");
    if (!cp || (nzc > 0 && (!jc || !ir))) return fail(BFS_ERR_ARG, "NULL input array");
    const bool dev = (flags & BFS_DEVICE_PTRS) != 0;
    bfs_graph* g = new (std::nothrow) bfs_graph();
    if (!g) return fail(BFS_ERR_OOM, "host allocation failed");
    (void)hipGetDevice(&g->device);
    g->kind = kDcsc;
    default_options(&g->opt);
    DcscDev& d = g->dcsc;
    d.nrows = nrows;
    d.ncols = ncols;
    d.nzc = nzc;
    d.nnz = nnz;
    hipStream_t s = nullptr;
    auto bail = [&](int code) {
      dcsc_free(g);
      delete g;
      return code;
    };
    hipError_t e = hipMalloc(&d.jc, (size_t)std::max(nzc, 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&d.cp, (size_t)(nzc + 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&d.ir, (size_t)std::max<int64_t>(nnz, 1) * 4);
    if (e != hipSuccess) return bail(hip_fail(e, "allocating DCSC arrays"));
    g->device_bytes = (int64_t)std::max(nzc, 1) * 4 + (int64_t)(nzc + 1) * 4 +
                      std::max<int64_t>(nnz, 1) * 4;
    int rc = copy_in(d.jc, jc, (size_t)nzc * 4, dev, s);
    if (rc == BFS_OK) rc = copy_in(d.cp, cp, (size_t)(nzc + 1) * 4, dev, s);
    if (rc == BFS_OK) rc = copy_in(d.ir, ir, (size_t)nnz * 4, dev, s);
    if (rc == BFS_OK) {
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = hip_fail(e, "upload");
    }
    if (rc == BFS_OK) rc = dcsc_setup(g, s, !(flags & BFS_TRUSTED));
    if (rc != BFS_OK) return bail(rc);
    *out = g;
    return BFS_OK;
  } catch (...) {
    return fail(BFS_ERR_OOM, "exception during create");
  }
}

int bfs_graph_destroy(bfs_graph_t* g) {
  if (!g) return fail(BFS_ERR_ARG, "NULL handle");
  if (g->users.load() > 0) return fail(BFS_ERR_BUSY, "graph is referenced by in-flight queries");
  if (g->last_stream) (void)hipStreamSynchronize(g->last_stream);
  (void)hipDeviceSynchronize();
  if (g->kind == kCsr) csr_free(g);
  if (g->kind == kDcsc) dcsc_free(g);
  if (g->h_ctr) (void)hipHostFree(g->h_ctr);
  for (hipEvent_t ev : g->ev) (void)hipEventDestroy(ev);
  delete g;
  return BFS_OK;
}

int bfs_graph_info(const bfs_graph_t* g, int64_t* n, int64_t* nnz, int64_t* device_bytes) {
  if (!g) return fail(BFS_ERR_ARG, "NULL handle");
  if (n) *n = g->kind == kCsr ? g->csr.n : g->dcsc.nrows;
  if (nnz) *nnz = g->kind == kCsr ? g->csr.nnz : g->dcsc.nnz;
  if (device_bytes) *device_bytes = g->device_bytes;
  return BFS_OK;
}

int bfs_graph_set_options(bfs_graph_t* g, const bfs_options_t* opt) {
  if (!g || !opt) return fail(BFS_ERR_ARG, "NULL argument");
  if (opt->mode < 0 || opt->mode > 2 || opt->batch_levels < 0 || opt->grid_blocks < 0 ||
      opt->claim < 0 || opt->claim > 3 || opt->claim_threshold < 0 ||
      opt->claim_min_frontier < 0)
    return fail(BFS_ERR_ARG, "option out of range");
  if (opt->cold_probe < 0 || opt->cold_probe > 3)
    return fail(BFS_ERR_ARG, "cold_probe must be 1, 2 or 3");
  if (opt->spmspv_sort_max < -1) return fail(BFS_ERR_ARG, "spmspv_sort_max must be >= -1");
  if (opt->pull_alpha < -1) return fail(BFS_ERR_ARG, "pull_alpha must be >= -1");
  if (opt->small_frontier < -1) return fail(BFS_ERR_ARG, "small_frontier must be >= -1");
  // every field checked: apply
  if (opt->cold_probe) g->opt.cold_probe = opt->cold_probe;
  if (opt->spmspv_sort_max) g->opt.spmspv_sort_max = opt->spmspv_sort_max;
  if (opt->pull_alpha) g->opt.pull_alpha = opt->pull_alpha;
  if (opt->small_frontier) g->opt.small_frontier = opt->small_frontier < 0 ? -1 : opt->small_frontier;
  if (opt->claim) g->opt.claim = opt->claim;
  if (opt->claim_threshold) g->opt.claim_threshold = opt->claim_threshold;
  if (opt->claim_min_frontier) g->opt.claim_min_frontier = opt->claim_min_frontier;
  if (opt->mode) g->opt.mode = opt->mode;
  if (opt->batch_levels) g->opt.batch_levels = opt->batch_levels;
  if (opt->grid_blocks) g->opt.grid_blocks = opt->grid_blocks;
  if (opt->lds_bitmap) g->opt.lds_bitmap = opt->lds_bitmap > 0 ? 1 : 0;
  if (opt->profile) g->opt.profile = opt->profile > 0 ? 1 : -1;
  return BFS_OK;
}

int bfs_graph_get_options(const bfs_graph_t* g, bfs_options_t* opt) {
  if (!g || !opt) return fail(BFS_ERR_ARG, "NULL argument");
  *opt = g->opt;
  return BFS_OK;
}

int bfs_run_async(bfs_graph_t* g, int32_t root, int32_t* parent, int32_t* level,
                  void* hip_stream) {
  if (!g) return fail(BFS_ERR_ARG, "NULL handle");
  if (g->kind != kCsr) return fail(BFS_ERR_ARG, "bfs_run needs a CSR graph");
  try {
    std::lock_guard<std::mutex> lk(g->run_mu);
    return csr_run(g, root, parent, level, static_cast<hipStream_t>(hip_stream), false);
  } catch (...) {
    return fail(BFS_ERR_DEVICE, "exception in bfs_run");
  }
}

int bfs_run(bfs_graph_t* g, int32_t root, int32_t* parent, int32_t* level) {
  if (!g) return fail(BFS_ERR_ARG, "NULL handle");
  if (g->kind != kCsr) return fail(BFS_ERR_ARG, "bfs_run needs a CSR graph");
  try {
    std::lock_guard<std::mutex> lk(g->run_mu);
    return csr_run(g, root, parent, level, nullptr, true);
  } catch (...) {
    return fail(BFS_ERR_DEVICE, "exception in bfs_run");
  }
}

int bfs_last_stats(bfs_graph_t* g, bfs_run_stats_t* st) {
  if (!g || !st) return fail(BFS_ERR_ARG, "NULL argument");
  if (g->kind != kCsr || !g->stats_valid) return fail(BFS_ERR_ARG, "no completed run");
  return csr_read_stats(g, st);
}

int bfs_last_level_info(bfs_graph_t* g, bfs_level_info_t* out, int32_t capacity,
                        int32_t* count) {
  if (!g || !count || (capacity > 0 && !out)) return fail(BFS_ERR_ARG, "NULL argument");
  if (g->kind != kCsr || !g->stats_valid || !g->profiled)
    return fail(BFS_ERR_ARG, "no profiled run");
  return csr_level_info(g, out, capacity, count);
}

int bfs_spmspv(bfs_graph_t* block, const bfs_svec_t* frontier, bfs_svec_t* out,
               void* hip_stream) {
  if (!block || !frontier || !out) return fail(BFS_ERR_ARG, "NULL argument");
  if (block->kind != kDcsc) return fail(BFS_ERR_ARG, "bfs_spmspv needs a DCSC block");
  try {
    return dcsc_spmspv(block, frontier, out, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return fail(BFS_ERR_DEVICE, "exception in bfs_spmspv");
  }
}

}  // extern "C"
