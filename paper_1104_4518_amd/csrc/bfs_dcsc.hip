// Local sparse-matrix x sparse-vector product on one hypersparse 2D share
// stored as DCSC (section 4.1; Algorithm 3's SpMSV step, section 4.2).
//
// The product is the union of the columns A(:, k) for every k in the
// frontier, each row keeping the minimum selected value. It is formed with
// a sparse accumulator (SPA, section 4.2): a dense array of values, an
// occupied bitmap, and an explicit ordering of the occupied rows. Here the
// ordering comes from scanning the bitmap, which yields rows ascending
// without a sort, and the same scan resets every touched SPA entry so the
// accumulator is clean for the next call.
//
//   lookup   frontier index k -> position p of k in JC, via a bucket index
//            over column ids (aux[b] = first p with JC[p] >= b * width)
//            followed by a short search inside the bucket
//   expand   rows IR[CP[p] .. CP[p+1]) of each found column
//   combine  atomicMin into the SPA value, atomicOr into the occupied bits
//   emit     bitmap scan -> ascending (row, value), SPA reset
//
// Very sparse frontiers take the other branch of the paper's polyalgorithm
// (section 4.2: a SPA for denser products, a sort-based merge when the
// product is small): one workgroup looks up the columns, writes the
// products as packed (row, value) keys into LDS, sorts them (bitonic) and
// keeps the first key of each row, so no work is proportional to nrows.
#include "bfs_internal.h"

#include <algorithm>

namespace bfsi {
namespace {

constexpr int kEmitBlock = 256;
constexpr int kWordsPerThread = 8;
constexpr int kWordsPerBlock = kEmitBlock * kWordsPerThread;

__global__ void k_dcsc_validate(int32_t nrows, int32_t ncols, int32_t nzc, int64_t nnz,
                                const int32_t* __restrict__ jc, const int32_t* __restrict__ cp,
                                const int32_t* __restrict__ ir, int32_t* err) {
  const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = i0; p < nzc; p += stride) {
    const int32_t c = jc[p];
    if (c < 0 || c >= ncols) atomicOr(err, 1);
    if (p > 0 && jc[p - 1] >= c) atomicOr(err, 2);
    if (cp[p + 1] <= cp[p]) atomicOr(err, 4);
  }
  if (i0 == 0 && (cp[0] != 0 || (int64_t)cp[nzc] != nnz)) atomicOr(err, 8);
  for (int64_t q = i0; q < nnz; q += stride) {
    const int32_t r = ir[q];
    if (r < 0 || r >= nrows) atomicOr(err, 16);
  }
}

// aux[b] = first p with jc[p] >= (b << shift), for b in [0, naux)
__global__ void k_build_aux(const int32_t* __restrict__ jc, int32_t nzc, int shift, int64_t naux,
                            int32_t* __restrict__ aux) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < naux; b += stride) {
    const int64_t key = b << shift;
    int64_t lo = 0, hi = nzc;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)jc[mid] < key) lo = mid + 1; else hi = mid;
    }
    aux[b] = (int32_t)lo;
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// One thread per frontier entry: lookup, expand, combine. Values are stored
// order-preserving as (val ^ 0x80000000) so that unsigned atomicMin gives the
// signed minimum.
__global__ void k_spmspv_scatter(int64_t fnnz, const int32_t* __restrict__ fidx,
                                 const int32_t* __restrict__ fval, int32_t ncols,
                                 const int32_t* __restrict__ jc, const int32_t* __restrict__ cp,
                                 const int32_t* __restrict__ ir, const int32_t* __restrict__ aux,
                                 int shift, uint32_t* __restrict__ spa_val,
                                 uint32_t* __restrict__ spa_occ,
                                 unsigned long long* __restrict__ counters) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < fnnz; i += stride) {
    const int32_t k = fidx[i];
    if (k < 0 || k >= ncols || (i > 0 && fidx[i - 1] >= k)) {
      atomicOr(&counters[1], 1ull);
      continue;
    }
    const uint32_t key = (uint32_t)(fval ? fval[i] : k) ^ 0x80000000u;
    const int64_t b = (int64_t)k >> shift;
    int32_t lo = aux[b], hi = aux[b + 1];
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (jc[mid] < k) lo = mid + 1; else hi = mid;
    }
    if (lo >= aux[b + 1] || jc[lo] != k) continue;   // empty column
    const int32_t q1 = cp[lo + 1];
    for (int32_t qq = cp[lo]; qq < q1; ++qq) {
      const int32_t r = ir[qq];
      // products rarely share a row, so the min is not filtered by a read
      // of the (large) value array and its result is not waited for
      atomicMin(&spa_val[r], key);
      const uint32_t bit = 1u << (r & 31);
      if (!(spa_occ[r >> 5] & bit)) atomicOr(&spa_occ[r >> 5], bit);
    }
  }
}

// Occupied-row count of each block's word range.
__global__ __launch_bounds__(kEmitBlock) void k_spa_count(const uint32_t* __restrict__ occ,
                                                          int64_t nwords,
                                                          int64_t* __restrict__ blk_count) {
  const int64_t w0 = blockIdx.x * (int64_t)kWordsPerBlock + threadIdx.x * kWordsPerThread;
  int c = 0;
#pragma unroll
  for (int i = 0; i < kWordsPerThread; ++i)
    if (w0 + i < nwords) c += __popc(occ[w0 + i]);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  __shared__ int s[kEmitBlock / 64];
  if (lane_id() == 0) s[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int x = 0; x < kEmitBlock / 64; ++x) t += s[x];
    blk_count[blockIdx.x] = t;
  }
}

// Exclusive scan of the block counts (one block); total -> counters[0].
__global__ void k_spa_scan(int64_t* __restrict__ blk_count, int64_t nblk,
                           unsigned long long* __restrict__ counters) {
  __shared__ long long s_carry;
  __shared__ long long s_w[4];
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nblk; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const long long v = i < nblk ? blk_count[i] : 0;
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
    if (i < nblk) blk_count[i] = carry + wb + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) counters[0] = (unsigned long long)s_carry;
}

// Bitmap scan: rows ascending with their SPA values; resets SPA entries.
__global__ __launch_bounds__(kEmitBlock) void k_spa_emit(
    uint32_t* __restrict__ occ, int64_t nwords, uint32_t* __restrict__ spa_val,
    const int64_t* __restrict__ blk_off, const unsigned long long* __restrict__ counters,
    int64_t capacity, int32_t* __restrict__ out_idx, int32_t* __restrict__ out_val) {
  const bool write = counters[0] <= (unsigned long long)capacity && counters[1] == 0ull;
  const int64_t w0 = blockIdx.x * (int64_t)kWordsPerBlock + threadIdx.x * kWordsPerThread;
  uint32_t words[kWordsPerThread];
  int c = 0;
#pragma unroll
  for (int i = 0; i < kWordsPerThread; ++i) {
    words[i] = (w0 + i < nwords) ? occ[w0 + i] : 0u;
    c += __popc(words[i]);
  }
  const long long incl = wave_incl_scan(c);
  __shared__ long long s_w[kEmitBlock / 64];
  const int wid = threadIdx.x >> 6;
  if (lane_id() == 63) s_w[wid] = incl;
  __syncthreads();
  long long wb = 0;
  for (int x = 0; x < wid; ++x) wb += s_w[x];
  long long pos = blk_off[blockIdx.x] + wb + incl - c;
#pragma unroll
  for (int i = 0; i < kWordsPerThread; ++i) {
    uint32_t bits = words[i];
    if (!bits) continue;
    const int64_t wbase = (w0 + i) << 5;
    while (bits) {
      const int b = __ffs(bits) - 1;
      bits &= bits - 1;
      const int64_t r = wbase + b;
      const uint32_t key = spa_val[r];
      spa_val[r] = 0xFFFFFFFFu;
      if (write) {
        out_idx[pos] = (int32_t)r;
        out_val[pos] = (int32_t)(key ^ 0x80000000u);
      }
      ++pos;
    }
    occ[w0 + i] = 0u;
  }
}

// Sort path: frontier entries and products it can hold in LDS.
constexpr int kSortBlock = 1024;
constexpr int kSortMaxF = 8192;
constexpr int kSortMaxP = 8192;

__device__ __forceinline__ int32_t dcsc_lookup(int32_t k, const int32_t* __restrict__ jc,
                                               const int32_t* __restrict__ aux, int shift) {
  const int64_t b = (int64_t)k >> shift;
  int32_t lo = aux[b], hi = aux[b + 1];
  const int32_t end = hi;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (jc[mid] < k) lo = mid + 1; else hi = mid;
  }
  return (lo < end && jc[lo] == k) ? lo : -1;
}

// Block-wide exclusive scan of one int per thread (kSortBlock threads).
__device__ __forceinline__ int sort_block_scan(int v, int* s_w, int& total) {
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  if (lane == 63) s_w[wid] = incl;
  __syncthreads();
  int base = 0;
  total = 0;
  for (int x = 0; x < kSortBlock / 64; ++x) {
    if (x < wid) base += s_w[x];
    total += s_w[x];
  }
  __syncthreads();
  return base + incl - v;
}

// counters[0] = output count, [1] = frontier error, [2] = product too large
// for LDS (the caller then runs the SPA path).
__global__ __launch_bounds__(kSortBlock) void k_spmspv_sort(
    int64_t fnnz, const int32_t* __restrict__ fidx, const int32_t* __restrict__ fval,
    int32_t ncols, const int32_t* __restrict__ jc, const int32_t* __restrict__ cp,
    const int32_t* __restrict__ ir, const int32_t* __restrict__ aux, int shift,
    unsigned long long* __restrict__ counters, int64_t capacity, int32_t* __restrict__ out_idx,
    int32_t* __restrict__ out_val) {
  __shared__ unsigned long long s_key[kSortMaxP];
  __shared__ int s_w[kSortBlock / 64];
  __shared__ int s_err;
  const int tid = threadIdx.x;
  constexpr int PER = kSortMaxF / kSortBlock;
  if (tid == 0) s_err = 0;
  __syncthreads();
  // lookup: thread t owns entries t*PER .. t*PER+PER-1 (contiguous, so the
  // product slots come out in frontier order); the PER lookups advance
  // together, one load each per step
  int32_t kk[PER], lo[PER], hi[PER], bend[PER];
  {
    const int64_t i0 = (int64_t)tid * PER;
    const int32_t prev = (i0 > 0 && i0 <= fnnz) ? fidx[i0 - 1] : -1;
#pragma unroll
    for (int j = 0; j < PER; ++j) kk[j] = (i0 + j < fnnz) ? fidx[i0 + j] : -1;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (i0 + j >= fnnz) continue;
      const int32_t before = j ? kk[j - 1] : prev;
      if (kk[j] < 0 || kk[j] >= ncols || (i0 + j > 0 && before >= kk[j])) bad = true;
    }
    if (bad) s_err = 1;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      lo[j] = hi[j] = bend[j] = 0;
      if (i0 + j < fnnz && kk[j] >= 0 && kk[j] < ncols) {
        const int64_t bk = (int64_t)kk[j] >> shift;
        lo[j] = aux[bk];
        hi[j] = bend[j] = aux[bk + 1];
      }
    }
    for (;;) {
      bool any = false;
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        if (lo[j] < hi[j]) {
          const int32_t mid = (lo[j] + hi[j]) >> 1;
          if (jc[mid] < kk[j]) lo[j] = mid + 1; else hi[j] = mid;
          any = true;
        }
      }
      if (!any) break;
    }
  }
  int32_t q0[PER], len[PER];
  int mine = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int64_t i = (int64_t)tid * PER + j;
    const bool found = i < fnnz && lo[j] < bend[j] && jc[lo[j]] == kk[j];
    q0[j] = found ? cp[lo[j]] : 0;
    len[j] = found ? cp[lo[j] + 1] - q0[j] : 0;
    mine += len[j];
  }
  __syncthreads();   // s_err complete
  int total = 0;
  int off = sort_block_scan(mine, s_w, total);
  if (s_err || total > kSortMaxP) {
    if (tid == 0) {
      if (s_err) counters[1] = 1ull;
      else counters[2] = 1ull;
    }
    return;
  }
  // expand: products as (row << 32) | order-preserving value; the first
  // product of every entry is loaded together
  {
    int32_t r0[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) r0[j] = len[j] > 0 ? ir[q0[j]] : 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int64_t i = (int64_t)tid * PER + j;
      if (len[j] == 0) continue;
      const uint32_t key = (uint32_t)(fval ? fval[i] : kk[j]) ^ 0x80000000u;
      s_key[off] = ((unsigned long long)(uint32_t)r0[j] << 32) | key;
      for (int32_t q = 1; q < len[j]; ++q)
        s_key[off + q] = ((unsigned long long)(uint32_t)ir[q0[j] + q] << 32) | key;
      off += len[j];
    }
  }
  // pad to a power of two with keys above every product
  int np2 = 1;
  while (np2 < total) np2 <<= 1;
  for (int i = total + tid; i < np2; i += kSortBlock) s_key[i] = ~0ull;
  __syncthreads();
  // bitonic sort, ascending
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < (np2 >> 1); i += kSortBlock) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & size) == 0;
        const unsigned long long a = s_key[lo], b = s_key[hi];
        if ((a > b) == up) {
          s_key[lo] = b;
          s_key[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  // first key of each row = its minimum value; rows come out ascending
  constexpr int PP = kSortMaxP / kSortBlock;
  int keep[PP];
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < PP; ++j) {
    const int i = tid * PP + j;
    keep[j] = (i < total && (i == 0 || (s_key[i] >> 32) != (s_key[i - 1] >> 32))) ? 1 : 0;
    cnt += keep[j];
  }
  int nout = 0;
  int pos = sort_block_scan(cnt, s_w, nout);
  const bool write = nout <= capacity;
#pragma unroll
  for (int j = 0; j < PP; ++j) {
    const int i = tid * PP + j;
    if (keep[j]) {
      if (write) {
        out_idx[pos] = (int32_t)(s_key[i] >> 32);
        out_val[pos] = (int32_t)((uint32_t)s_key[i] ^ 0x80000000u);
      }
      ++pos;
    }
  }
  if (tid == 0) counters[0] = (unsigned long long)nout;
}

}  // namespace

int dcsc_setup(bfs_graph* g, hipStream_t s, bool validate) {
  DcscDev& d = g->dcsc;
  if (validate) {
    int32_t* d_err = nullptr;
    BFS_HIP(hipMalloc(&d_err, 4));
    BFS_HIP(hipMemsetAsync(d_err, 0, 4, s));
    k_dcsc_validate<<<1024, 256, 0, s>>>(d.nrows, d.ncols, d.nzc, d.nnz, d.jc, d.cp, d.ir, d_err);
    int32_t h = 0;
    hipError_t e = hipMemcpyAsync(&h, d_err, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_err);
    if (e != hipSuccess) return hip_fail(e, "dcsc validation");
    if (h & 1) return fail(BFS_ERR_FORMAT, "DCSC column id out of [0, ncols)");
    if (h & 2) return fail(BFS_ERR_FORMAT, "DCSC JC must be strictly ascending");
    if (h & 4) return fail(BFS_ERR_FORMAT, "DCSC CP must be strictly increasing");
    if (h & 8) return fail(BFS_ERR_FORMAT, "DCSC CP must start at 0 and end at nnz");
    if (h & 16) return fail(BFS_ERR_FORMAT, "DCSC row id out of [0, nrows)");
  }
  // bucket width: about four stored columns per bucket on average
  int shift = 0;
  if (d.nzc > 0) {
    const double ratio = (double)d.ncols / (double)d.nzc;
    while ((double)(1ll << (shift + 1)) <= ratio * 4.0 && shift < 30) ++shift;
  }
  d.aux_shift = shift;
  d.naux = ((int64_t)std::max(d.ncols, 1) >> shift) + 2;
  BFS_HIP(hipMalloc(&d.aux, (size_t)d.naux * 4));
  k_build_aux<<<1024, 256, 0, s>>>(d.jc, d.nzc, shift, d.naux, d.aux);
  d.nwords = ((int64_t)d.nrows + 31) / 32;
  BFS_HIP(hipMalloc(&d.spa_val, (size_t)std::max(d.nrows, 1) * 4));
  BFS_HIP(hipMalloc(&d.spa_occ, (size_t)std::max<int64_t>(d.nwords, 1) * 4));
  k_fill_u32<<<1024, 256, 0, s>>>(d.spa_val, d.nrows, 0xFFFFFFFFu);
  BFS_HIP(hipMemsetAsync(d.spa_occ, 0, (size_t)std::max<int64_t>(d.nwords, 1) * 4, s));
  d.nblk = (d.nwords + kWordsPerBlock - 1) / kWordsPerBlock;
  BFS_HIP(hipMalloc(&d.blk_count, (size_t)std::max<int64_t>(d.nblk, 1) * 8));
  BFS_HIP(hipMalloc(&d.counters, 3 * sizeof(unsigned long long)));
  BFS_HIP(hipMemsetAsync(d.counters, 0, 3 * sizeof(unsigned long long), s));
  BFS_HIP(hipHostMalloc(&d.h_counters, 3 * sizeof(unsigned long long), hipHostMallocDefault));
  BFS_HIP(hipStreamSynchronize(s));
  g->device_bytes += d.naux * 4 + (int64_t)std::max(d.nrows, 1) * 4 +
                     std::max<int64_t>(d.nwords, 1) * 4 + std::max<int64_t>(d.nblk, 1) * 8 + 16;
  return BFS_OK;
}

void dcsc_free(bfs_graph* g) {
  DcscDev& d = g->dcsc;
  (void)hipFree(d.jc);
  (void)hipFree(d.cp);
  (void)hipFree(d.ir);
  (void)hipFree(d.aux);
  (void)hipFree(d.spa_val);
  (void)hipFree(d.spa_occ);
  (void)hipFree(d.blk_count);
  (void)hipFree(d.counters);
  if (d.h_counters) (void)hipHostFree(d.h_counters);
  d = DcscDev{};
}

int dcsc_spmspv(bfs_graph* g, const bfs_svec_t* f, bfs_svec_t* out, hipStream_t s) {
  DcscDev& d = g->dcsc;
  if (f->nnz < 0 || (f->nnz > 0 && !f->idx)) return fail(BFS_ERR_ARG, "bad frontier vector");
  if (f->nnz > (int64_t)d.ncols) return fail(BFS_ERR_ARG, "frontier longer than ncols");
  if (out->capacity < 0 || (out->capacity > 0 && (!out->idx || !out->val)))
    return fail(BFS_ERR_ARG, "bad output vector");
  BFS_HIP(hipMemsetAsync(d.counters, 0, 3 * sizeof(unsigned long long), s));
  // sort path for small frontiers (a product too large for LDS falls back)
  const int64_t sort_max = std::min<int64_t>(g->opt.spmspv_sort_max, kSortMaxF);
  if (f->nnz > 0 && f->nnz <= sort_max) {
    k_spmspv_sort<<<1, kSortBlock, 0, s>>>(f->nnz, f->idx, f->val, d.ncols, d.jc, d.cp, d.ir,
                                           d.aux, d.aux_shift, d.counters, out->capacity,
                                           out->idx, out->val);
    BFS_HIP(hipGetLastError());
    BFS_HIP(hipMemcpyAsync(d.h_counters, d.counters, 3 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    BFS_HIP(hipStreamSynchronize(s));
    if (!d.h_counters[2]) {
      const int64_t cnt = (int64_t)d.h_counters[0];
      if (d.h_counters[1]) {
        out->nnz = 0;
        return fail(BFS_ERR_ARG, "frontier indices must be strictly ascending and in [0, ncols)");
      }
      out->nnz = cnt;
      if (cnt > out->capacity) return fail(BFS_ERR_CAPACITY, "output capacity too small");
      return BFS_OK;
    }
    BFS_HIP(hipMemsetAsync(d.counters, 0, 3 * sizeof(unsigned long long), s));
  }
  if (f->nnz > 0) {
    const int blk = 256;
    const int64_t grid = std::min<int64_t>((f->nnz + blk - 1) / blk, 65536);
    k_spmspv_scatter<<<(int)grid, blk, 0, s>>>(f->nnz, f->idx, f->val, d.ncols, d.jc, d.cp,
                                                d.ir, d.aux, d.aux_shift, d.spa_val, d.spa_occ,
                                                d.counters);
  }
  if (d.nwords > 0) {
    k_spa_count<<<(int)d.nblk, kEmitBlock, 0, s>>>(d.spa_occ, d.nwords, d.blk_count);
    k_spa_scan<<<1, 256, 0, s>>>(d.blk_count, d.nblk, d.counters);
    k_spa_emit<<<(int)d.nblk, kEmitBlock, 0, s>>>(d.spa_occ, d.nwords, d.spa_val, d.blk_count,
                                                   d.counters, out->capacity, out->idx,
                                                   out->val);
  }
  BFS_HIP(hipGetLastError());
  BFS_HIP(hipMemcpyAsync(d.h_counters, d.counters, 2 * sizeof(unsigned long long),
                         hipMemcpyDeviceToHost, s));
  BFS_HIP(hipStreamSynchronize(s));
  const int64_t cnt = (int64_t)d.h_counters[0];
  if (d.h_counters[1]) {
    out->nnz = 0;
    return fail(BFS_ERR_ARG, "frontier indices must be strictly ascending and in [0, ncols)");
  }
  out->nnz = cnt;
  if (cnt > out->capacity) return fail(BFS_ERR_CAPACITY, "output capacity too small");
  return BFS_OK;
}

}  // namespace bfsi
