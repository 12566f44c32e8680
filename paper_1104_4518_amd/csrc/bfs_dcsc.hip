// Local sparse-matrix x sparse-vector product on one hypersparse 2D share
// stored as DCSC (section 4.1; Algorithm 3's SpMSV step, section 4.2).
//
// The product is the union of the columns A(:, k) for every k in the
// frontier, each row keeping the minimum selected value, emitted in
// ascending row order. Two branches, as in section 4.2's polyalgorithm:
//
//   binned accumulator (any frontier): the sparse accumulator of section 4.2
//            split by rows. k_spmspv_bin looks up each frontier index k in JC
//            (a bucket index over column ids, aux[b] = first p with JC[p] >=
//            b * width, then a short search; for scattered lookups a record
//            per bucket holds its columns and row ranges in one line),
//            expands the rows IR[CP[p] ..
//            CP[p+1]) edge-balanced and appends every (row, value) product to
//            the bin of its row (2^18 rows per bin); k_spmspv_reduce gives
//            every bin one workgroup, whose LDS holds the bin's accumulator
//            (a bitmap of the rows hit, ranked by a prefix over its words,
//            and the minimum value of each ranked row) and which emits its
//            rows ascending at the offset a chained scan over the bins gives.
//            No global atomic per product, and no pass over the whole row
//            space: the accumulator is cleared and scanned in LDS.
//   sort-based merge (very sparse frontiers, below a tuned size): one
//            workgroup looks up the columns, writes the products as packed
//            (row, value) keys into LDS, sorts them (bitonic) and keeps the
//            first key of each row.
#include "bfs_internal.h"

#include <algorithm>
#include <vector>

namespace bfsi {
namespace {

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

// Bucket records: bucket b's stored columns in one 64-byte line (16 words):
// [0] first position p, [1] count (bit 31: no record, use AUX/JC/CP),
// [2] cp[p], [3..6] the columns' offsets in the bucket (one byte each, up to
// kRecCols), [7..13] cp[p + i + 1] - cp[p] for each column i (16 bits each).
constexpr int kRecCols = 14;
__global__ void k_build_recs(const int32_t* __restrict__ jc, const int32_t* __restrict__ cp,
                             const int32_t* __restrict__ aux, int shift, int64_t nb,
                             uint4* __restrict__ recs) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += stride) {
    const int32_t lo = aux[b], cnt = aux[b + 1] - lo;
    const int32_t base = cp[lo];
    uint32_t w[16] = {0u};
    bool ok = cnt <= kRecCols;
    for (int i = 0; ok && i < cnt; ++i) {
      const uint32_t off = (uint32_t)((int64_t)jc[lo + i] - (b << shift));
      const int32_t cum = cp[lo + i + 1] - base;
      if (cum > 0xFFFF) {
        ok = false;
        break;
      }
      w[3 + (i >> 2)] |= off << (8 * (i & 3));
      w[7 + (i >> 1)] |= (uint32_t)cum << (16 * (i & 1));
    }
    w[0] = (uint32_t)lo;
    w[1] = (uint32_t)cnt | (ok ? 0u : 0x80000000u);
    w[2] = (uint32_t)base;
#pragma unroll
    for (int x = 0; x < 4; ++x)
      recs[b * 4 + x] = make_uint4(w[4 * x], w[4 * x + 1], w[4 * x + 2], w[4 * x + 3]);
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------- binned product
// The accumulator of section 4.2 split by rows. The output rows are cut into
// bins of 2^kBinShift consecutive rows; bin b owns the slice
// [bin_start[b], bin_start[b+1]) of a pair buffer, as long as the stored
// entries of the block in those rows (a bound on the products one call can
// put there, since every stored entry yields at most one product).
//
//   k_spmspv_bin     looks up the frontier's columns (bucket record, or
//                    bucket index + short search), expands them edge-balanced, and
//                    appends every product (row, value) to its row's bin:
//                    products are staged in LDS, counted per bin, and each
//                    workgroup reserves its slots of a bin with one atomic
//                    per non-empty bin and staging round
//   k_spmspv_reduce  one workgroup per bin: an LDS bitmap of the bin's rows
//                    marks the rows hit; a prefix over its words ranks them;
//                    the minimum of each row is taken in an LDS array indexed
//                    by rank; the rows are emitted ascending. The output
//                    offset of a bin is the number of rows hit by all bins
//                    before it, found by a chained scan over the bins in
//                    ascending order (each workgroup publishes its own count,
//                    then its inclusive prefix; bins are taken in order of a
//                    ticket counter, so a workgroup only waits for bins
//                    already running).
// Values travel order-preserving as (val ^ 0x80000000), so that an unsigned
// minimum is the signed one.
constexpr int kBinShift = 18;
constexpr int kBinRows = 1 << kBinShift;
constexpr int kBinWords = kBinRows / 32;
constexpr int kMaxBins = 8192;          // 2^31 rows
constexpr int kBinBlock = 1024;
constexpr int kStage = 4096;            // products staged in LDS between bin rounds
constexpr int kStagePer = kStage / kBinBlock;
// frontier entries looked up together per thread: 2 (two workgroups per CU
// fit, which hides more latency than more entries per thread in one), or 1
// for small frontiers so that more CUs take part
constexpr int kNarrowEntries = 2, kSingleEntries = 1;
constexpr int kProbe = 4;               // stored columns of a bucket read at once
constexpr int kReduceBlock = 1024;
constexpr int kHeld = 8;                // pairs per thread the reduction keeps in registers

// Workgroup barrier that orders LDS only: global loads and stores still in
// flight (prefetched frontier entries, pair stores) are not waited for. The
// kernels below use it wherever the threads of a workgroup exchange data
// through LDS alone.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
constexpr int kValCap = 16384;          // rows of one bin reduced in LDS; more use the SPA
// chained-scan flag word: epoch (30 bits) | status (2 bits) | count (32 bits)
constexpr uint64_t kFlagAgg = 1, kFlagIncl = 2;
constexpr long long kLookbackSpins = 1ll << 22;

struct BinArgs {
  int64_t fnnz;
  const int32_t* fidx;
  const int32_t* fval;
  int32_t ncols;
  const int32_t* jc;
  const int32_t* cp;
  const int32_t* ir;
  const int32_t* aux;
  const uint4* recs;        // bucket records, or null (buckets wider than 256 columns)
  int shift;
  int32_t nbins;
  const int64_t* bin_start;
  int32_t* cursor;
  unsigned long long* pairs;
  unsigned long long* counters;
  uint32_t epoch;
};

// EPT frontier entries per thread form a sub-chunk of kBinBlock * EPT
// consecutive entries; their lookups advance together (one load each per
// step), then the sub-chunk's products are expanded edge-balanced into the
// LDS stage, which is binned whenever it fills.
template <int EPT>
__global__ __launch_bounds__(kBinBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_spmspv_bin(BinArgs a) {
  // the bucket probe pays for scattered lookups only (with two entries per
  // thread, i.e. dense frontiers, the binary search measured faster)
  constexpr bool PROBE = EPT == 1;
  constexpr int WAVES = kBinBlock / 64;
  constexpr int SUB = kBinBlock * EPT;
  __shared__ int32_t s_pre[SUB];            // product prefix of the sub-chunk's entries
  __shared__ int32_t s_q0[SUB];             // first stored entry of the entry's column
  __shared__ uint32_t s_fv[SUB];            // the entries' values (order-preserving key)
  __shared__ int32_t s_row[kStage];         // staged products
  __shared__ uint32_t s_kst[kStage];
  __shared__ int s_w[WAVES];
  extern __shared__ long long s_dyn[];
  long long* s_base = s_dyn;                // pair slot of the round's first product, or -1
  int32_t* s_hist = reinterpret_cast<int32_t*>(s_dyn + a.nbins);   // products per bin (kept zero)
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;
  for (int b = tid; b < a.nbins; b += kBinBlock) s_hist[b] = 0;
  int staged = 0;   // products in the stage (the same in every thread)
  bool bad = false;

  // bins the staged products: per-bin ranks in LDS, one global reservation
  // per non-empty bin, then the pairs written to their bins' slices
  auto flush = [&](int S) {
    lds_barrier();
    int rk[kStagePer];
#pragma unroll
    for (int i = 0; i < kStagePer; ++i) {
      const int j = tid + i * kBinBlock;
      rk[i] = j < S ? atomicAdd(&s_hist[s_row[j] >> kBinShift], 1) : 0;
    }
    lds_barrier();
    for (int b = tid; b < a.nbins; b += kBinBlock) {
      const int h = s_hist[b];
      if (h) {
        // a valid frontier never exceeds a bin's slice (each stored entry
        // gives at most one product); a repeated column could
        const int64_t pos = a.bin_start[b] + atomicAdd(&a.cursor[b], h);
        s_base[b] = pos + h <= a.bin_start[b + 1] ? pos : -1;
        s_hist[b] = 0;
      }
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < kStagePer; ++i) {
      const int j = tid + i * kBinBlock;
      if (j < S) {
        const int32_t row = s_row[j];
        const long long base = s_base[row >> kBinShift];
        if (base >= 0)
          a.pairs[base + rk[i]] = ((unsigned long long)(uint32_t)(row & (kBinRows - 1)) << 32) | s_kst[j];
        else
          bad = true;
      }
    }
    lds_barrier();
  };

  const int64_t nsub = (a.fnnz + SUB - 1) / SUB;
  // the frontier entries of a sub-chunk (thread t owns entries t*EPT ..
  // t*EPT + EPT - 1) and the entry before them; the next sub-chunk's are
  // loaded while the current one is expanded
  // (loaded unconditionally at clamped indices, so that no load waits
  // before the entries are used; the entries past the frontier are dropped
  // there)
  int32_t nk[EPT], nv[EPT], nprev = -1;
  auto load_entries = [&](int64_t c) {
    const int64_t i0 = c * SUB + (int64_t)tid * EPT;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int64_t i = min(i0 + j, a.fnnz - 1);
      nk[j] = a.fidx[i];
      nv[j] = a.fval ? a.fval[i] : 0;
    }
    nprev = a.fidx[max(min(i0, a.fnnz) - 1, (int64_t)0)];
  };
  load_entries(blockIdx.x);
  for (int64_t c = blockIdx.x; c < nsub; c += gridDim.x) {
    const int64_t c0 = c * SUB;
    const int nE = (int)min((int64_t)SUB, a.fnnz - c0);
    // lookup; every step issues the loads of all the thread's entries before
    // it uses any of them (entries without a column read index 0 and drop it)
    int32_t kk[EPT], kv[EPT];
    {
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        kk[j] = tid * EPT + j < nE ? nk[j] : -1;
        kv[j] = a.fval ? nv[j] : nk[j];
      }
      const int32_t prev = c0 + (int64_t)tid * EPT > 0 ? nprev : -1;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        if (tid * EPT + j >= nE) continue;
        const int32_t before = j ? kk[j - 1] : prev;
        if (kk[j] < 0 || kk[j] >= a.ncols || before >= kk[j]) {
          bad = true;
          kk[j] = -1;
        }
      }
    }
    // column positions. With one entry per thread (small frontiers, whose
    // lookups are scattered) the entry's bucket record, one 64-byte line,
    // holds the bucket's columns and their row ranges and so decides the
    // lookup in one load. Other entries (larger frontiers, and buckets
    // without a record) read AUX, then a bucket of JC (its first kProbe
    // columns together for one entry per thread, else, and past them, a
    // binary search), then CP.
    int32_t q0[EPT], len[EPT];
    bool slow[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      q0[j] = 0;
      len[j] = 0;
      slow[j] = kk[j] >= 0;
    }
    if constexpr (PROBE) {
      if (a.recs) {
        uint4 r[EPT][4];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const int64_t bk = kk[j] >= 0 ? ((int64_t)kk[j] >> a.shift) : 0;
#pragma unroll
          for (int x = 0; x < 4; ++x) r[j][x] = a.recs[bk * 4 + x];
        }
        // (an empty use of every loaded word, so that the compiler cannot
        // load the count alone and the rest only under a branch on it)
#pragma unroll
        for (int j = 0; j < EPT; ++j)
#pragma unroll
          for (int x = 0; x < 4; ++x)
            asm volatile("" ::"v"(r[j][x].x), "v"(r[j][x].y), "v"(r[j][x].z), "v"(r[j][x].w));
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const uint32_t w[16] = {r[j][0].x, r[j][0].y, r[j][0].z, r[j][0].w,
                                  r[j][1].x, r[j][1].y, r[j][1].z, r[j][1].w,
                                  r[j][2].x, r[j][2].y, r[j][2].z, r[j][2].w,
                                  r[j][3].x, r[j][3].y, r[j][3].z, r[j][3].w};
          if (kk[j] < 0 || (w[1] >> 31)) continue;
          slow[j] = false;
          const uint32_t off = (uint32_t)kk[j] & ((1u << a.shift) - 1u);
#pragma unroll
          for (int i = 0; i < kRecCols; ++i) {
            const uint32_t col = (w[3 + (i >> 2)] >> (8 * (i & 3))) & 0xFFu;
            const uint32_t c1 = (w[7 + (i >> 1)] >> (16 * (i & 1))) & 0xFFFFu;
            const uint32_t c0 = i ? (w[7 + ((i - 1) >> 1)] >> (16 * ((i - 1) & 1))) & 0xFFFFu : 0u;
            if ((uint32_t)i < w[1] && col == off) {
              q0[j] = (int32_t)(w[2] + c0);
              len[j] = (int32_t)(c1 - c0);
            }
          }
        }
      }
    }
    bool any_slow = false;
#pragma unroll
    for (int j = 0; j < EPT; ++j) any_slow |= slow[j];
    if (__any(any_slow)) {
      int32_t ks[EPT], lo[EPT], hi[EPT], bend[EPT], qp[EPT];
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        ks[j] = slow[j] ? kk[j] : -1;
        qp[j] = -1;
      }
      int32_t a0[EPT], a1[EPT];
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int64_t bk = ks[j] >= 0 ? ((int64_t)ks[j] >> a.shift) : 0;
        a0[j] = a.aux[bk];
        a1[j] = a.aux[bk + 1];
      }
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        lo[j] = ks[j] >= 0 ? a0[j] : 0;
        hi[j] = bend[j] = ks[j] >= 0 ? a1[j] : 0;
      }
      if constexpr (PROBE) {
        int32_t w[EPT][kProbe];
#pragma unroll
        for (int j = 0; j < EPT; ++j)
#pragma unroll
          for (int i = 0; i < kProbe; ++i) w[j][i] = a.jc[lo[j] + i < hi[j] ? lo[j] + i : 0];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          int c = 0;
#pragma unroll
          for (int i = 0; i < kProbe; ++i) c += lo[j] + i < hi[j] && w[j][i] < ks[j];
          int32_t at = INT32_MAX;
#pragma unroll
          for (int i = kProbe - 1; i >= 0; --i)
            if (i == c && lo[j] + i < hi[j]) at = w[j][i];
          if (ks[j] >= 0 && c < kProbe && at == ks[j]) qp[j] = lo[j] + c;
          if (ks[j] >= 0 && c == kProbe && lo[j] + kProbe < hi[j]) lo[j] += kProbe;
          else lo[j] = hi[j];
        }
      }
      for (;;) {
        bool any = false;
        int32_t mid[EPT], vm[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          mid[j] = (lo[j] + hi[j]) >> 1;
          vm[j] = a.jc[lo[j] < hi[j] ? mid[j] : 0];
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (lo[j] < hi[j]) {
            if (vm[j] < ks[j]) lo[j] = mid[j] + 1; else hi[j] = mid[j];
            any = true;
          }
        if (!any) break;
      }
      {
        int32_t vl[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const bool open = qp[j] < 0 && ks[j] >= 0 && lo[j] < bend[j];
          vl[j] = a.jc[open ? lo[j] : 0];
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (qp[j] < 0 && ks[j] >= 0 && lo[j] < bend[j] && vl[j] == ks[j]) qp[j] = lo[j];
      }
      {
        int32_t c0[EPT], c1[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          const int32_t p = qp[j] >= 0 ? qp[j] : 0;
          c0[j] = a.cp[p];
          c1[j] = a.cp[p + 1];
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (slow[j] && qp[j] >= 0) {
            len[j] = c1[j] - c0[j];
            q0[j] = c0[j];
          }
      }
    }
    int mine = 0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) mine += len[j];
    load_entries(c + gridDim.x);
    // exclusive product prefix over the sub-chunk's entries (entry order)
    const int incl = (int)wave_incl_scan((long long)mine);
    if (lane == 63) s_w[wid] = incl;
    lds_barrier();
    int wb = 0, P = 0;
#pragma unroll
    for (int x = 0; x < WAVES; ++x) {
      if (x < wid) wb += s_w[x];
      P += s_w[x];
    }
    {
      int ex = wb + incl - mine;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = tid * EPT + j;
        if (e < nE) {
          s_pre[e] = ex;
          s_q0[e] = q0[j];
          s_fv[e] = (uint32_t)kv[j] ^ 0x80000000u;
        }
        ex += len[j];
      }
    }
    lds_barrier();
    // expand: product jj belongs to the last entry whose prefix is <= jj
    // (entries without products share their successor's prefix)
    for (int done = 0; done < P;) {
      const int take = min(P - done, kStage - staged);
      for (int j = tid; j < take; j += kBinBlock) {
        const int jj = done + j;
        int l = 0, h = nE - 1;
        while (l < h) {
          const int mid = (l + h + 1) >> 1;
          if (s_pre[mid] <= jj) l = mid; else h = mid - 1;
        }
        s_row[staged + j] = a.ir[s_q0[l] + (jj - s_pre[l])];
        s_kst[staged + j] = s_fv[l];
      }
      staged += take;
      done += take;
      if (staged == kStage) {
        flush(staged);
        staged = 0;
      }
    }
    lds_barrier();   // s_pre / s_q0 are rewritten by the next sub-chunk
  }
  if (staged > 0) flush(staged);
  if (__any(bad) && lane == 0) a.counters[1] = a.epoch;
}

struct ReduceArgs {
  int32_t nbins;
  const int64_t* bin_start;
  int32_t* cursor;
  const unsigned long long* pairs;
  unsigned long long* chain;
  uint32_t* ticket;         // bin tickets taken by all calls so far (wraps)
  uint32_t ticket_base;     // the counter's value when this call's reduction starts
  uint32_t* spa_val;        // nrows, all ones between calls (bins over kValCap rows)
  unsigned long long* counters;
  unsigned long long* host;  // pinned host words the results are written to
  uint32_t epoch;
  int64_t capacity;
  int32_t* out_idx;
  int32_t* out_val;
};

__device__ __forceinline__ unsigned long long chain_word(uint32_t epoch, uint64_t status,
                                                         uint32_t count) {
  return ((unsigned long long)epoch << 34) | (status << 32) | count;
}

__global__ __launch_bounds__(kReduceBlock) void k_spmspv_reduce(ReduceArgs a) {
  constexpr int WAVES = kReduceBlock / 64;
  constexpr int WPT = kBinWords / kReduceBlock;   // bitmap words per thread
  __shared__ uint32_t s_bits[kBinWords];
  __shared__ int32_t s_wpre[kBinWords];
  __shared__ uint32_t s_val[kValCap];
  __shared__ int s_w[WAVES];
  __shared__ uint32_t s_b;
  __shared__ long long s_excl;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;
  // The bin comes from the ticket counter: bins are taken in the order
  // workgroups start, so a workgroup's chained-scan waits are only for
  // workgroups already running.
  if (tid == 0) s_b = atomicAdd(a.ticket, 1u) - a.ticket_base;
  // the thread's first kHeld pairs, all loaded before any is used and kept
  // for the second pass; a bin with more pairs reads the rest in place
  unsigned long long pr[kHeld];
  int64_t st;
  int cnt;
  bool err;
  auto read_bin = [&](int bin) {
    st = a.bin_start[bin];
    cnt = (int)min((int64_t)__hip_atomic_load(&a.cursor[bin], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT),
                   a.bin_start[bin + 1] - st);
    err = a.counters[1] == a.epoch;
#pragma unroll
    for (int i = 0; i < kHeld; ++i) {
      const int j = tid + i * kReduceBlock;
      pr[i] = (!err && j < cnt) ? a.pairs[st + j] : 0ull;
    }
  };
  for (int w = tid; w < kBinWords; w += kReduceBlock) s_bits[w] = 0u;
  lds_barrier();
  const uint32_t ub = s_b;
  if (ub >= (uint32_t)a.nbins) {   // tickets out of step with the grid: report, touch nothing
    if (tid == 0) a.host[3] = a.epoch;
    return;
  }
  const int b = (int)ub;
  read_bin(b);
  if (!err) {
#pragma unroll
    for (int i = 0; i < kHeld; ++i) {
      const uint32_t r = (uint32_t)(pr[i] >> 32);
      if (tid + i * kReduceBlock < cnt) atomicOr(&s_bits[r >> 5], 1u << (r & 31));
    }
    for (int j = tid + kHeld * kReduceBlock; j < cnt; j += kReduceBlock) {
      const uint32_t r = (uint32_t)(a.pairs[st + j] >> 32);
      atomicOr(&s_bits[r >> 5], 1u << (r & 31));
    }
  }
  lds_barrier();
  // rank of the first hit row of every word (block prefix over popcounts)
  int c = 0;
#pragma unroll
  for (int i = 0; i < WPT; ++i) c += __popc(s_bits[tid * WPT + i]);
  const int incl = (int)wave_incl_scan((long long)c);
  if (lane == 63) s_w[wid] = incl;
  lds_barrier();
  int wb = 0, U = 0;
#pragma unroll
  for (int x = 0; x < WAVES; ++x) {
    if (x < wid) wb += s_w[x];
    U += s_w[x];
  }
  {
    int r = wb + incl - c;
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      s_wpre[tid * WPT + i] = r;
      r += __popc(s_bits[tid * WPT + i]);
    }
  }
  // chained scan: publish this bin's count, then find the rows of all bins
  // before it (wave 0 reads back 256 bins at a time, four words per lane,
  // all issued before any is examined)
  if (!err && wid == 0) {
    if (lane == 0)
      __hip_atomic_store(&a.chain[b], chain_word(a.epoch, kFlagAgg, (uint32_t)U),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    constexpr int R = 4;
    long long excl = 0;
    int j = b - 1;
    long long spins = 0;
    while (j >= 0) {
      unsigned long long f[R];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int idx = j - lane - 64 * k;
        f[k] = idx >= 0 ? __hip_atomic_load(&a.chain[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                        : chain_word(a.epoch, kFlagIncl, 0u);   // before bin 0: nothing
      }
      bool done = false, wait = false;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const uint32_t fe = (uint32_t)(f[k] >> 34);
        const int status = fe == a.epoch ? (int)((f[k] >> 32) & 3u) : 0;
        const unsigned long long nr = wave_ballot(status == 0);
        const unsigned long long inc = wave_ballot(status == 2);
        const int first_nr = nr ? __ffsll((long long)nr) - 1 : 64;
        const int first_inc = inc ? __ffsll((long long)inc) - 1 : 64;
        if (first_nr < first_inc) {
          // a bin not published yet: take the counts before it and wait
          long long v = lane < first_nr ? (long long)(uint32_t)f[k] : 0;
#pragma unroll
          for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
          excl += v;
          j -= first_nr;
          wait = true;
          break;
        }
        long long v = lane <= first_inc ? (long long)(uint32_t)f[k] : 0;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        excl += v;
        if (first_inc < 64) {
          done = true;
          break;
        }
        j -= 64;
      }
      if (done) break;
      if (wait) {
        if (++spins > kLookbackSpins) {
          if (lane == 0) a.host[3] = a.epoch;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (lane == 0) {
      __hip_atomic_store(&a.chain[b], chain_word(a.epoch, kFlagIncl, (uint32_t)(excl + U)),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_excl = excl;
    }
  }
  lds_barrier();
  if (!err) {
    const long long excl = s_excl;
    const int64_t row0 = (int64_t)b << kBinShift;
    if (U <= kValCap) {
      for (int i = tid; i < U; i += kReduceBlock) s_val[i] = 0xFFFFFFFFu;
      lds_barrier();
      auto take = [&](unsigned long long p) {
        const uint32_t r = (uint32_t)(p >> 32);
        const int w = (int)(r >> 5);
        const int rank = s_wpre[w] + __popc(s_bits[w] & ((1u << (r & 31)) - 1u));
        atomicMin(&s_val[rank], (uint32_t)p);
      };
#pragma unroll
      for (int i = 0; i < kHeld; ++i)
        if (tid + i * kReduceBlock < cnt) take(pr[i]);
      for (int j = tid + kHeld * kReduceBlock; j < cnt; j += kReduceBlock) take(a.pairs[st + j]);
      lds_barrier();
      for (int i = 0; i < WPT; ++i) {
        const int w = i * kReduceBlock + tid;
        uint32_t bits = s_bits[w];
        int r = s_wpre[w];
        while (bits) {
          const int bit = __ffs(bits) - 1;
          bits &= bits - 1;
          const long long pos = excl + r;
          if (pos < a.capacity) {
            a.out_idx[pos] = (int32_t)(row0 + w * 32 + bit);
            a.out_val[pos] = (int32_t)(s_val[r] ^ 0x80000000u);
          }
          ++r;
        }
      }
    } else {
      // more rows than the LDS array holds: the minimum goes through the
      // block-wide SPA (all ones between calls), reset as it is emitted
      for (int j = tid; j < cnt; j += kReduceBlock) {
        const unsigned long long p = a.pairs[st + j];
        atomicMin(&a.spa_val[row0 + (uint32_t)(p >> 32)], (uint32_t)p);
      }
      __threadfence();
      __syncthreads();
      for (int i = 0; i < WPT; ++i) {
        const int w = i * kReduceBlock + tid;
        uint32_t bits = s_bits[w];
        int r = s_wpre[w];
        while (bits) {
          const int bit = __ffs(bits) - 1;
          bits &= bits - 1;
          const int64_t row = row0 + w * 32 + bit;
          const uint32_t v =
              __hip_atomic_load(&a.spa_val[row], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          a.spa_val[row] = 0xFFFFFFFFu;
          const long long pos = excl + r;
          if (pos < a.capacity) {
            a.out_idx[pos] = (int32_t)row;
            a.out_val[pos] = (int32_t)(v ^ 0x80000000u);
          }
          ++r;
        }
      }
    }
  }
  if (tid == 0) {
    a.cursor[b] = 0;   // the bin's slice is empty for the next call
    // the last bin's workgroup hands the call's results to the host (read
    // once the stream has drained): output count, frontier error, and the
    // epoch as the mark that the call completed
    if (b == a.nbins - 1) {
      a.host[0] = err ? 0ull : (unsigned long long)(s_excl + U);
      a.host[1] = err ? a.epoch : 0ull;
      a.host[2] = a.epoch;
    }
  }
}

// Stored entries per bin of rows (setup): LDS histogram per workgroup.
__global__ void k_bin_count(int64_t nnz, const int32_t* __restrict__ ir, int32_t nbins,
                            unsigned long long* __restrict__ counts) {
  __shared__ unsigned int s_h[kMaxBins];
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) s_h[b] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += stride)
    atomicAdd(&s_h[ir[q] >> kBinShift], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x)
    if (s_h[b]) atomicAdd(&counts[b], (unsigned long long)s_h[b]);
}

// Sort path: frontier entries and products it can hold in LDS.
constexpr int kSortBlock = 1024;
constexpr int kSortMaxF = 8192;
constexpr int kSortMaxP = 8192;


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
// for LDS (the caller then runs the binned path).
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
  // bucket records (one byte per column offset: buckets of at most 256 columns)
  d.recs = nullptr;
  if (shift <= 8) {
    BFS_HIP(hipMalloc(&d.recs, (size_t)(d.naux - 1) * 64));
    k_build_recs<<<1024, 256, 0, s>>>(d.jc, d.cp, d.aux, shift, d.naux - 1,
                                      reinterpret_cast<uint4*>(d.recs));
  }
  // row bins: each owns a slice of the pair buffer as long as its stored entries
  d.nbins = (int32_t)(((int64_t)std::max(d.nrows, 1) + kBinRows - 1) >> kBinShift);
  BFS_HIP(hipMalloc(&d.bin_start, (size_t)(d.nbins + 1) * 8));
  {
    unsigned long long* cnt = nullptr;
    BFS_HIP(hipMalloc(&cnt, (size_t)d.nbins * 8));
    BFS_HIP(hipMemsetAsync(cnt, 0, (size_t)d.nbins * 8, s));
    if (d.nnz > 0) k_bin_count<<<1024, 256, 0, s>>>(d.nnz, d.ir, d.nbins, cnt);
    std::vector<unsigned long long> h((size_t)d.nbins);
    hipError_t e = hipMemcpyAsync(h.data(), cnt, h.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(cnt);
    if (e != hipSuccess) return hip_fail(e, "dcsc bin counts");
    std::vector<int64_t> start((size_t)d.nbins + 1, 0);
    for (int32_t b = 0; b < d.nbins; ++b) start[(size_t)b + 1] = start[(size_t)b] + (int64_t)h[(size_t)b];
    BFS_HIP(hipMemcpy(d.bin_start, start.data(), start.size() * 8, hipMemcpyHostToDevice));
  }
  BFS_HIP(hipMalloc(&d.cursor, (size_t)d.nbins * 4));
  BFS_HIP(hipMemsetAsync(d.cursor, 0, (size_t)d.nbins * 4, s));
  BFS_HIP(hipMalloc(&d.chain, (size_t)d.nbins * 8));
  BFS_HIP(hipMemsetAsync(d.chain, 0, (size_t)d.nbins * 8, s));
  BFS_HIP(hipMalloc(&d.ticket, 4));
  BFS_HIP(hipMemsetAsync(d.ticket, 0, 4, s));
  d.ticket_base = 0;
  BFS_HIP(hipMalloc(&d.pairs, (size_t)std::max<int64_t>(d.nnz, 1) * 8));
  BFS_HIP(hipMalloc(&d.spa_val, (size_t)std::max(d.nrows, 1) * 4));
  k_fill_u32<<<1024, 256, 0, s>>>(d.spa_val, d.nrows, 0xFFFFFFFFu);
  BFS_HIP(hipMalloc(&d.counters, 4 * sizeof(unsigned long long)));
  BFS_HIP(hipMemsetAsync(d.counters, 0, 4 * sizeof(unsigned long long), s));
  BFS_HIP(hipHostMalloc(&d.h_counters, 4 * sizeof(unsigned long long), hipHostMallocDefault));
  for (int i = 0; i < 4; ++i) d.h_counters[i] = 0ull;   // no epoch matches before a call
  BFS_HIP(hipHostGetDevicePointer((void**)&d.h_counters_dev, d.h_counters, 0));
  BFS_HIP(hipStreamSynchronize(s));
  // the binning kernel's per-bin counters live in dynamic LDS (12 B per bin)
  (void)hipFuncSetAttribute((const void*)k_spmspv_bin<kNarrowEntries>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxBins * 12);
  (void)hipFuncSetAttribute((const void*)k_spmspv_bin<kSingleEntries>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, kMaxBins * 12);
  (void)hipGetLastError();
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device) !=
          hipSuccess || cus <= 0)
    cus = 256;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_spmspv_bin<kNarrowEntries>,
                                                   kBinBlock, (size_t)d.nbins * 12) !=
          hipSuccess || occ <= 0)
    occ = 1;
  (void)hipGetLastError();
  d.grid_bin = cus * occ;   // co-resident workgroups of the binning kernel
  d.epoch = 1;
  g->device_bytes += d.naux * 4 + (d.recs ? (d.naux - 1) * 64 : 0) +
                     (int64_t)std::max(d.nrows, 1) * 4 +
                     (int64_t)(d.nbins + 1) * 8 + (int64_t)d.nbins * 12 + 4 +
                     std::max<int64_t>(d.nnz, 1) * 8 + 32;
  return BFS_OK;
}

void dcsc_free(bfs_graph* g) {
  DcscDev& d = g->dcsc;
  (void)hipFree(d.jc);
  (void)hipFree(d.cp);
  (void)hipFree(d.ir);
  (void)hipFree(d.aux);
  if (d.recs) (void)hipFree(d.recs);
  (void)hipFree(d.spa_val);
  (void)hipFree(d.bin_start);
  (void)hipFree(d.cursor);
  (void)hipFree(d.chain);
  (void)hipFree(d.ticket);
  (void)hipFree(d.pairs);
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
  if (f->nnz == 0) {   // the empty product: nothing to look up or emit
    out->nnz = 0;
    return BFS_OK;
  }
  // sort path for small frontiers (a product too large for LDS falls back)
  const int64_t sort_max = std::min<int64_t>(g->opt.spmspv_sort_max, kSortMaxF);
  if (f->nnz <= sort_max) {
    BFS_HIP(hipMemsetAsync(d.counters, 0, 3 * sizeof(unsigned long long), s));
    k_spmspv_sort<<<1, kSortBlock, 0, s>>>(f->nnz, f->idx, f->val, d.ncols, d.jc, d.cp, d.ir,
                                           d.aux, d.aux_shift, d.counters, out->capacity,
                                           out->idx, out->val);
    BFS_HIP(hipGetLastError());
    BFS_HIP(hipMemcpyAsync(d.h_counters, d.counters, 3 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    BFS_HIP(wait_stream(s));
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
  }
  // binned path; every call has its own epoch, so the flags of earlier calls
  // (chained scan, error words) need no clearing between calls
  // (epochs start at 2: the sort path writes 0 or 1 into the error word)
  if (++d.epoch >= (1u << 30)) {
    BFS_HIP(hipMemsetAsync(d.chain, 0, (size_t)d.nbins * 8, s));
    BFS_HIP(hipMemsetAsync(d.counters, 0, 4 * sizeof(unsigned long long), s));
    BFS_HIP(hipMemsetAsync(d.ticket, 0, 4, s));
    d.ticket_base = 0;
    d.epoch = 2;
  }
  BinArgs ba;
  ba.fnnz = f->nnz;
  ba.fidx = f->idx;
  ba.fval = f->val;
  ba.ncols = d.ncols;
  ba.jc = d.jc;
  ba.cp = d.cp;
  ba.ir = d.ir;
  ba.aux = d.aux;
  ba.recs = reinterpret_cast<const uint4*>(d.recs);
  ba.shift = d.aux_shift;
  ba.nbins = d.nbins;
  ba.bin_start = d.bin_start;
  ba.cursor = d.cursor;
  ba.pairs = d.pairs;
  ba.counters = d.counters;
  ba.epoch = d.epoch;
  const size_t dyn = (size_t)d.nbins * 12;
  auto nsub = [&](int ept) { return (f->nnz + kBinBlock * ept - 1) / (kBinBlock * ept); };
  if (nsub(kNarrowEntries) >= d.grid_bin) {
    k_spmspv_bin<kNarrowEntries><<<d.grid_bin, kBinBlock, dyn, s>>>(ba);
  } else {
    k_spmspv_bin<kSingleEntries>
        <<<(int)std::min<int64_t>(nsub(kSingleEntries), d.grid_bin), kBinBlock, dyn, s>>>(ba);
  }
  ReduceArgs ra;
  ra.nbins = d.nbins;
  ra.bin_start = d.bin_start;
  ra.cursor = d.cursor;
  ra.pairs = d.pairs;
  ra.chain = d.chain;
  ra.ticket = d.ticket;
  ra.ticket_base = d.ticket_base;
  ra.spa_val = d.spa_val;
  ra.counters = d.counters;
  ra.host = d.h_counters_dev;
  ra.epoch = d.epoch;
  ra.capacity = out->capacity;
  ra.out_idx = out->idx;
  ra.out_val = out->val;
  k_spmspv_reduce<<<d.nbins, kReduceBlock, 0, s>>>(ra);
  BFS_HIP(hipGetLastError());
  d.ticket_base += (uint32_t)d.nbins;   // one ticket per workgroup
  BFS_HIP(wait_stream(s));
  const volatile unsigned long long* h = d.h_counters;
  if (h[2] != d.epoch || h[3] == d.epoch) {
    // the tickets may be out of step with the calls: start them again
    BFS_HIP(hipMemsetAsync(d.ticket, 0, 4, s));
    d.ticket_base = 0;
    BFS_HIP(wait_stream(s));
    return fail(BFS_ERR_DEVICE, h[2] != d.epoch
                                    ? "spmspv: the reduction over the row bins did not complete"
                                    : "spmspv: chained scan over the row bins did not complete");
  }
  if (h[1] == d.epoch) {
    out->nnz = 0;
    return fail(BFS_ERR_ARG, "frontier indices must be strictly ascending and in [0, ncols)");
  }
  const int64_t cnt = (int64_t)h[0];
  out->nnz = cnt;
  if (cnt > out->capacity) return fail(BFS_ERR_CAPACITY, "output capacity too small");
  return BFS_OK;
}

}  // namespace bfsi
