// Seeded synthetic inputs: R-MAT and Erdos-Renyi edge lists turned into
// symmetric CSR, 2D lattices, uniform hypersparse DCSC blocks, sparse
// frontier samples and BFS roots.
//
// This module builds inputs only. It holds none of the traversal or
// sparse-product arithmetic: it is shared by the CPU oracle and the GPU
// library, and both see exactly the same bytes.
//
// Randomness is counter based, so every value depends only on (seed, index)
// and not on thread count or scheduling: SplitMix64 (Steele, Lea, Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014), used as
// out(i) = mix(key + (i + 1) * golden).
//
// Graph recipe (R-MAT of Chakrabarti, Zhan, Faloutsos 2004, with the
// parameters of the paper's experimental section):
//   * every edge picks one quadrant per bit level with probabilities
//     a, b, c, d, given as 32-bit integer thresholds, no noise;
//   * vertex ids are relabelled with a seeded bijection of [0, 2^scale)
//     (the paper relabels vertices at random for load balance);
//   * the edge list is symmetrised, self-loops are dropped, duplicate
//     adjacencies are removed and each adjacency list is sorted ascending.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <omp.h>
#include <parallel/algorithm>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGolden); }

// Purpose-separated keys so that edge, permutation and root streams of one
// seed never overlap.
inline uint64_t stream_key(uint64_t seed, uint64_t purpose) {
  return mix64(seed * 0xD1342543DE82EF95ull + purpose * kGolden + 0x632BE59BD9B4E019ull);
}

enum : uint64_t { kEdges = 1, kPerm = 2, kRoots = 3, kSample = 4, kBlock = 5 };

// Seeded bijection of [0, 2^bits): rounds of odd multiply, xor-shift and
// add, each invertible modulo 2^bits.
struct Perm {
  uint64_t k[4];
  uint64_t mask;
  int sh;
  Perm(int bits, uint64_t key) {
    mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1);
    sh = (bits + 1) / 2;
    for (int r = 0; r < 4; ++r) k[r] = draw(key, (uint64_t)r);
  }
  uint64_t operator()(uint64_t x) const {
    if (mask == 0) return 0;
    for (int r = 0; r < 4; ++r) {
      x = (x * (k[r] | 1ull)) & mask;
      x ^= (x >> sh);
      x = (x + (k[r] >> 17)) & mask;
    }
    return x;
  }
};

inline uint64_t perm_bits(uint64_t x, int bits, uint64_t key) {
  if (bits <= 0) return 0;
  return Perm(bits, key)(x);
}

struct EdgeSpec {
  int kind;        // 0 = R-MAT, 1 = uniform endpoints
  int scale;       // n = 2^scale
  int64_t m;       // generated edges
  uint32_t ta, tab, tabc;  // cumulative quadrant thresholds (x 2^32)
  uint64_t ekey;
  Perm perm;
  int permute;
};

inline void gen_edge(const EdgeSpec& s, int64_t e, uint64_t* pu, uint64_t* pv) {
  uint64_t u = 0, v = 0;
  const uint64_t mask = (1ull << s.scale) - 1;
  if (s.kind == 1) {
    const uint64_t r0 = draw(s.ekey, (uint64_t)e * 2);
    const uint64_t r1 = draw(s.ekey, (uint64_t)e * 2 + 1);
    u = r0 & mask;
    v = r1 & mask;
  } else {
    for (int i = 0; i < s.scale; i += 2) {
      const uint64_t r = draw(s.ekey, (uint64_t)e * 32 + (uint64_t)(i / 2));
      for (int h = 0; h < 2 && i + h < s.scale; ++h) {
        const uint32_t x = (uint32_t)(h ? (r >> 32) : r);
        // quadrants in order a (0,0), b (0,1), c (1,0), d (1,1)
        const uint64_t ge_a = x >= s.ta, ge_ab = x >= s.tab, ge_abc = x >= s.tabc;
        const uint64_t ub = ge_ab;
        const uint64_t vb = ge_a ^ ge_ab ^ ge_abc;
        u = (u << 1) | ub;
        v = (v << 1) | vb;
      }
    }
  }
  if (s.permute) {
    u = s.perm(u);
    v = s.perm(v);
  }
  *pu = u;
  *pv = v;
}

EdgeSpec make_spec(int kind, int scale, int64_t m, uint32_t ta, uint32_t tab, uint32_t tabc,
                   uint64_t seed, int permute) {
  EdgeSpec s{0, 0, 0, 0, 0, 0, 0, Perm(scale, stream_key(seed, kPerm)), 0};
  s.kind = kind;
  s.scale = scale;
  s.m = m;
  s.ta = ta;
  s.tab = tab;
  s.tabc = tabc;
  s.ekey = stream_key(seed, kEdges);
  s.permute = permute;
  return s;
}

}  // namespace

extern "C" {

uint64_t gg_mix64(uint64_t x) { return mix64(x); }
uint64_t gg_draw(uint64_t key, uint64_t i) { return draw(key, i); }
uint64_t gg_stream_key(uint64_t seed, uint64_t purpose) { return stream_key(seed, purpose); }
uint64_t gg_perm(uint64_t x, int bits, uint64_t seed) {
  return perm_bits(x, bits, stream_key(seed, kPerm));
}

void gg_edge_list(int kind, int scale, int64_t m, uint32_t ta, uint32_t tab, uint32_t tabc,
                  uint64_t seed, int permute, int64_t* us, int64_t* vs) {
  const EdgeSpec s = make_spec(kind, scale, m, ta, tab, tabc, seed, permute);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t u, v;
    gen_edge(s, e, &u, &v);
    us[e] = (int64_t)u;
    vs[e] = (int64_t)v;
  }
}

// Pass 1: raw adjacency counts (both directions, self-loops dropped) as an
// exclusive prefix in off_raw[0..n]. Returns off_raw[n].
int64_t gg_edges_count(int kind, int scale, int64_t m, uint32_t ta, uint32_t tab, uint32_t tabc,
                       uint64_t seed, int permute, int64_t* off_raw) {
  const EdgeSpec s = make_spec(kind, scale, m, ta, tab, tabc, seed, permute);
  const int64_t n = (int64_t)1 << scale;
  std::atomic<int64_t>* deg = reinterpret_cast<std::atomic<int64_t>*>(off_raw);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i <= n; ++i) off_raw[i] = 0;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t u, v;
    gen_edge(s, e, &u, &v);
    if (u == v) continue;
    deg[u + 1].fetch_add(1, std::memory_order_relaxed);
    deg[v + 1].fetch_add(1, std::memory_order_relaxed);
  }
  for (int64_t i = 0; i < n; ++i) off_raw[i + 1] += off_raw[i];
  return off_raw[n];
}

// Pass 2: scatter both directions into col_raw, sort each row, drop
// duplicates in place; deg_unique[v] receives the deduplicated degree.
// Returns the total deduplicated adjacency count.
int64_t gg_edges_fill(int kind, int scale, int64_t m, uint32_t ta, uint32_t tab, uint32_t tabc,
                      uint64_t seed, int permute, const int64_t* off_raw, int32_t* col_raw,
                      int64_t* deg_unique) {
  const EdgeSpec s = make_spec(kind, scale, m, ta, tab, tabc, seed, permute);
  const int64_t n = (int64_t)1 << scale;
  std::atomic<int64_t>* cur = reinterpret_cast<std::atomic<int64_t>*>(deg_unique);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) deg_unique[i] = off_raw[i];
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint64_t u, v;
    gen_edge(s, e, &u, &v);
    if (u == v) continue;
    col_raw[cur[u].fetch_add(1, std::memory_order_relaxed)] = (int32_t)v;
    col_raw[cur[v].fetch_add(1, std::memory_order_relaxed)] = (int32_t)u;
  }
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : total)
  for (int64_t i = 0; i < n; ++i) {
    int32_t* b = col_raw + off_raw[i];
    int32_t* e = col_raw + off_raw[i + 1];
    std::sort(b, e);
    const int64_t k = std::unique(b, e) - b;
    deg_unique[i] = k;
    total += k;
  }
  return total;
}

// Rows of col_raw (first deg_unique[v] entries of each) packed into the
// final CSR arrays.
void gg_compact(int64_t n, const int64_t* off_raw, const int32_t* col_raw,
                const int64_t* deg_unique, int64_t* off, int32_t* col) {
  off[0] = 0;
  for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + deg_unique[i];
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i)
    std::memcpy(col + off[i], col_raw + off_raw[i], (size_t)deg_unique[i] * sizeof(int32_t));
}

// W x H 4-neighbour lattice, row-major ids, adjacency ascending.
int64_t gg_grid_count(int64_t w, int64_t h) { return 2 * ((w - 1) * h + (h - 1) * w); }

void gg_grid(int64_t w, int64_t h, int64_t* off, int32_t* col) {
  const int64_t n = w * h;
  off[0] = 0;
  for (int64_t id = 0; id < n; ++id) {
    const int64_t i = id / w, j = id % w;
    off[id + 1] = off[id] + (i > 0) + (j > 0) + (j < w - 1) + (i < h - 1);
  }
#pragma omp parallel for schedule(static)
  for (int64_t id = 0; id < n; ++id) {
    const int64_t i = id / w, j = id % w;
    int64_t p = off[id];
    if (i > 0) col[p++] = (int32_t)(id - w);
    if (j > 0) col[p++] = (int32_t)(id - 1);
    if (j < w - 1) col[p++] = (int32_t)(id + 1);
    if (i < h - 1) col[p++] = (int32_t)(id + w);
  }
}

// Uniform (row, col) pairs in a 2^log_n x 2^log_n block, packed as
// (col << 32 | row), sorted and deduplicated. Returns the unique count.
int64_t gg_block_keys(int log_n, int64_t nnz, uint64_t seed, uint64_t* keys) {
  const uint64_t key = stream_key(seed, kBlock);
  const uint64_t mask = (1ull << log_n) - 1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nnz; ++e) {
    const uint64_t r = draw(key, (uint64_t)e);
    const uint64_t row = r & mask;
    const uint64_t colv = (r >> 32) & mask;
    keys[e] = (colv << 32) | row;
  }
  __gnu_parallel::sort(keys, keys + nnz);
  return std::unique(keys, keys + nnz) - keys;
}

// DCSC arrays from sorted unique keys: jc (column ids), cp (nzc + 1
// pointers), ir (row ids). jc and cp must hold cnt + 1 entries. Returns nzc.
int64_t gg_dcsc_from_keys(const uint64_t* keys, int64_t cnt, int32_t* jc, int32_t* cp,
                          int32_t* ir) {
  int64_t nzc = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    const uint32_t c = (uint32_t)(keys[i] >> 32);
    if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != c) {
      jc[nzc] = (int32_t)c;
      cp[nzc] = (int32_t)i;
      ++nzc;
    }
    ir[i] = (int32_t)(keys[i] & 0xFFFFFFFFull);
  }
  cp[nzc] = (int32_t)cnt;
  return nzc;
}

// k distinct indices of [0, 2^log_n), sorted ascending: images of 0..k-1
// under a seeded bijection.
void gg_sample(int log_n, int64_t k, uint64_t seed, int32_t* out) {
  const Perm pm(log_n, stream_key(seed, kSample));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < k; ++i) out[i] = (int32_t)pm((uint64_t)i);
  __gnu_parallel::sort(out, out + k);
}

// Up to `count` distinct roots with degree >= 1: v = draw(seed, t) mod n for
// t = 0, 1, ..., rejecting degree-0 vertices and repeats. Returns how many
// were found (fewer only if the graph has fewer non-isolated vertices).
int64_t gg_roots(int64_t n, const int64_t* off, int64_t count, uint64_t seed, int32_t* out) {
  const uint64_t key = stream_key(seed, kRoots);
  int64_t got = 0;
  const int64_t max_tries = 64 * n + 4096;
  for (int64_t t = 0; t < max_tries && got < count; ++t) {
    const int64_t v = (int64_t)(draw(key, (uint64_t)t) % (uint64_t)n);
    if (off[v + 1] - off[v] < 1) continue;
    bool dup = false;
    for (int64_t j = 0; j < got; ++j)
      if (out[j] == v) { dup = true; break; }
    if (!dup) out[got++] = (int32_t)v;
  }
  return got;
}

// Order-fixed hash of a byte array (independent of thread count).
uint64_t gg_hash_bytes(const void* data, int64_t nbytes) {
  const uint8_t* p = static_cast<const uint8_t*>(data);
  const int64_t chunk = 1 << 20;
  const int64_t nchunks = (nbytes + chunk - 1) / chunk;
  std::vector<uint64_t> hs((size_t)std::max<int64_t>(nchunks, 1), 0);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nchunks; ++c) {
    const int64_t b = c * chunk, e = std::min(nbytes, b + chunk);
    uint64_t h = 0x84222325CBF29CE4ull ^ (uint64_t)c;
    int64_t i = b;
    for (; i + 8 <= e; i += 8) {
      uint64_t w;
      std::memcpy(&w, p + i, 8);
      h = mix64(h ^ w) + kGolden;
    }
    for (; i < e; ++i) h = mix64(h ^ p[i]) + kGolden;
    hs[(size_t)c] = h;
  }
  uint64_t h = mix64((uint64_t)nbytes);
  for (int64_t c = 0; c < nchunks; ++c) h = mix64(h ^ hs[(size_t)c]) + kGolden;
  return h;
}

}  // extern "C"
