/*
 * Host builder of the seeded synthetic graphs (OpenMP).
 *
 * Produces a symmetric CSR with int64 offsets and int32 neighbour IDs: each
 * undirected edge is stored as two directed entries, self-loops and duplicate
 * edges are removed and every adjacency list is sorted by ascending ID.  The
 * result is a pure function of the generator parameters and the seed; the
 * thread count only changes how fast it is built.
 *
 * Graph families:
 *   - Kronecker / R-MAT (gg_kronecker): edgefactor * 2^scale generated edges,
 *     quadrant probabilities A, B, C (D = 1-A-B-C), seeded vertex relabelling.
 *   - Chung-Lu power law with path tails (gg_chung_lu): expected-degree
 *     weights w_i = c (i0 + i)^(-1/(gamma-1)), both endpoints of every edge
 *     drawn proportionally to w through a Walker/Vose alias table, seeded
 *     relabelling of the core vertices, plus path tails of new vertices that
 *     hang off random core vertices of degree >= 1.
 *
 * Nothing here performs a breadth-first search.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include <omp.h>

#include "gg_chunglu.h"
#include "gg_rng.h"

namespace {

struct Csr {
  int64_t n = 0, m = 0;
  int64_t* offsets = nullptr;
  int32_t* indices = nullptr;
};

template <class T>
T* alloc_array(int64_t count) {
  if (count <= 0) count = 1;
  return static_cast<T*>(std::malloc(sizeof(T) * (size_t)count));
}

/* Exclusive prefix sum of cnt[0..n) into out[0..n], parallel in blocks. */
void exclusive_scan(const int64_t* cnt, int64_t* out, int64_t n) {
  const int nt = omp_get_max_threads();
  std::vector<int64_t> part(nt + 1, 0);
#pragma omp parallel num_threads(nt)
  {
    const int t = omp_get_thread_num();
    const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += cnt[i];
    part[t + 1] = s;
#pragma omp barrier
#pragma omp single
    for (int i = 0; i < nt; ++i) part[i + 1] += part[i];
    int64_t run = part[t];
    for (int64_t i = lo; i < hi; ++i) {
      out[i] = run;
      run += cnt[i];
    }
  }
  out[n] = part[nt];
}

/* Edge list -> cleaned symmetric CSR.  `edge(k, u, v)` yields generated edge
   k of `count`; it may be called twice per k (count pass, fill pass). */
template <class EdgeFn>
int build_csr(int64_t n, int64_t count, const EdgeFn& edge, Csr* out) {
  int64_t* deg = alloc_array<int64_t>(n);
  if (!deg) return -3;
  std::memset(deg, 0, sizeof(int64_t) * (size_t)n);

#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) {
    uint32_t u, v;
    edge(k, u, v);
    if (u == v) continue;
    __atomic_fetch_add(&deg[u], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&deg[v], 1, __ATOMIC_RELAXED);
  }

  int64_t* off_dup = alloc_array<int64_t>(n + 1);
  if (!off_dup) { std::free(deg); return -3; }
  exclusive_scan(deg, off_dup, n);
  const int64_t m_dup = off_dup[n];
  int32_t* idx_dup = alloc_array<int32_t>(m_dup);
  if (!idx_dup) { std::free(deg); std::free(off_dup); return -3; }

  /* Reuse deg as the per-row fill cursor. */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) deg[i] = off_dup[i];

#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) {
    uint32_t u, v;
    edge(k, u, v);
    if (u == v) continue;
    const int64_t pu = __atomic_fetch_add(&deg[u], 1, __ATOMIC_RELAXED);
    const int64_t pv = __atomic_fetch_add(&deg[v], 1, __ATOMIC_RELAXED);
    idx_dup[pu] = (int32_t)v;
    idx_dup[pv] = (int32_t)u;
  }

  /* Sort and de-duplicate every row in place; deg[] becomes the unique count. */
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i) {
    int32_t* b = idx_dup + off_dup[i];
    int32_t* e = idx_dup + off_dup[i + 1];
    std::sort(b, e);
    deg[i] = std::unique(b, e) - b;
  }

  int64_t* offsets = alloc_array<int64_t>(n + 1);
  if (!offsets) { std::free(deg); std::free(off_dup); std::free(idx_dup); return -3; }
  exclusive_scan(deg, offsets, n);
  const int64_t m = offsets[n];
  int32_t* indices = alloc_array<int32_t>(m);
  if (!indices) {
    std::free(deg); std::free(off_dup); std::free(idx_dup); std::free(offsets);
    return -3;
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < n; ++i)
    std::memcpy(indices + offsets[i], idx_dup + off_dup[i], sizeof(int32_t) * (size_t)deg[i]);

  std::free(deg);
  std::free(off_dup);
  std::free(idx_dup);
  out->n = n;
  out->m = m;
  out->offsets = offsets;
  out->indices = indices;
  return 0;
}

gg_rmat_t rmat_thresholds(double a, double b, double c) {
  const double s = 4294967296.0;
  gg_rmat_t t;
  t.a = (uint32_t)std::floor(a * s);
  t.ab = (uint32_t)std::floor((a + b) * s);
  t.abc = (uint32_t)std::floor((a + b + c) * s);
  return t;
}

/* Keyed bijection of [0, n) for arbitrary n >= 1 (cycle walking over the
   power-of-two Feistel permutation). */
}  // namespace

extern "C" {

typedef struct gg_csr_s {
  int64_t n, m;
  int64_t* offsets;
  int32_t* indices;
} gg_csr;

void gg_set_threads(int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
}

/* Thresholds as used by both builders (so the device builder can take them). */
void gg_rmat_thresholds(double a, double b, double c, uint32_t out[3]) {
  const gg_rmat_t t = rmat_thresholds(a, b, c);
  out[0] = t.a;
  out[1] = t.ab;
  out[2] = t.abc;
}

/* Raw generated edge k (after relabelling when permute != 0); for tests. */
void gg_kronecker_edges(int scale, uint64_t seed, double a, double b, double c, int permute,
                        int64_t first, int64_t count, uint32_t* u_out, uint32_t* v_out) {
  const uint64_t key = gg_stream_key(seed, GG_STREAM_EDGES);
  const uint64_t pkey = gg_stream_key(seed, GG_STREAM_PERM);
  const gg_rmat_t t = rmat_thresholds(a, b, c);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) {
    uint32_t u, v;
    gg_rmat_edge(key, scale, t, (uint64_t)(first + i), &u, &v);
    if (permute) {
      u = gg_permute(pkey, scale, u);
      v = gg_permute(pkey, scale, v);
    }
    u_out[i] = u;
    v_out[i] = v;
  }
}

uint32_t gg_permute_value(uint64_t seed, int scale, uint32_t x) {
  return gg_permute(gg_stream_key(seed, GG_STREAM_PERM), scale, x);
}

/* Kronecker graph: n = 2^scale vertices, edgefactor * n generated edges. */
gg_csr* gg_kronecker(int scale, int edgefactor, uint64_t seed, double a, double b, double c,
                     int permute, int* status) {
  *status = -1;
  if (scale < 1 || scale > 31 || edgefactor < 1) return nullptr;
  const int64_t n = (int64_t)1 << scale;
  const int64_t count = (int64_t)edgefactor << scale;
  const uint64_t key = gg_stream_key(seed, GG_STREAM_EDGES);
  const uint64_t pkey = gg_stream_key(seed, GG_STREAM_PERM);
  const gg_rmat_t t = rmat_thresholds(a, b, c);
  auto edge = [&](int64_t k, uint32_t& u, uint32_t& v) {
    gg_rmat_edge(key, scale, t, (uint64_t)k, &u, &v);
    if (permute) {
      u = gg_permute(pkey, scale, u);
      v = gg_permute(pkey, scale, v);
    }
  };
  Csr csr;
  *status = build_csr(n, count, edge, &csr);
  if (*status) return nullptr;
  gg_csr* g = new (std::nothrow) gg_csr{csr.n, csr.m, csr.offsets, csr.indices};
  if (!g) *status = -3;
  return g;
}

/* Expected-degree weights of the Chung-Lu family (gg_chunglu.h). */
int gg_chung_lu_weights(int64_t n, double gamma, double avg_deg, double max_deg, double* i0_out,
                        double* c_out) {
  return gg_cl_weights(n, gamma, avg_deg, max_deg, i0_out, c_out);
}

/* Chung-Lu core of n_core vertices plus n_tails path tails of tail_len new
   vertices each.  Vertex IDs: core [0, n_core) (seeded relabelling), tail t
   vertex j is n_core + t*tail_len + j.  The core has round(n_core*avg_deg/2)
   generated edges. */
gg_csr* gg_chung_lu(int64_t n_core, double gamma, double avg_deg, double max_deg, int32_t n_tails,
                    int32_t tail_len, uint64_t seed, int* status) {
  *status = -1;
  if (n_core < 2 || n_tails < 0 || tail_len < 0) return nullptr;
  const int64_t n = n_core + (int64_t)n_tails * tail_len;
  if (n > 2147483647LL) return nullptr;
  double i0, c;
  if (gg_cl_weights(n_core, gamma, avg_deg, max_deg, &i0, &c)) return nullptr;
  std::vector<uint32_t> thr;
  std::vector<int32_t> alias;
  gg_cl_alias(n_core, i0, c, 1.0 / (gamma - 1.0), thr, alias);
  gg_cl_core_t t;
  t.key = gg_stream_key(seed, GG_STREAM_CL_EDGES);
  t.pkey = gg_stream_key(seed, GG_STREAM_PERM);
  t.n_core = n_core;
  t.pbits = gg_bits_for((uint64_t)n_core);
  t.pad = 0;
  t.thr = thr.data();
  t.alias = alias.data();
  const int64_t m_core = (int64_t)std::llround((double)n_core * avg_deg / 2.0);

  /* Tail anchors: uniform core vertices of degree >= 1 in the core graph
     (degree counted before de-duplication: a non-loop edge survives it). */
  std::vector<uint32_t> anchor((size_t)std::max<int32_t>(n_tails, 1));
  if (n_tails > 0 && tail_len > 0) {
    std::vector<uint8_t> has_edge((size_t)n_core, 0);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m_core; ++k) {
      uint32_t u, v;
      gg_cl_core_edge(t, k, &u, &v);
      if (u != v) {
        __atomic_store_n(&has_edge[u], (uint8_t)1, __ATOMIC_RELAXED);
        __atomic_store_n(&has_edge[v], (uint8_t)1, __ATOMIC_RELAXED);
      }
    }
    if (gg_cl_anchors(n_core, seed, n_tails, has_edge.data(), anchor.data())) {
      *status = -2;
      return nullptr;
    }
  }
  const uint32_t* anchor_p = anchor.data();
  const int64_t per_tail = tail_len;
  const int64_t count = m_core + (tail_len > 0 ? (int64_t)n_tails * per_tail : 0);
  auto edge = [&](int64_t k, uint32_t& u, uint32_t& v) { gg_cl_edge(t, m_core, anchor_p, per_tail, k, &u, &v); };
  Csr csr;
  *status = build_csr(n, count, edge, &csr);
  if (*status) return nullptr;
  gg_csr* g = new (std::nothrow) gg_csr{csr.n, csr.m, csr.offsets, csr.indices};
  if (!g) *status = -3;
  return g;
}

/* CSR from an explicit edge list (self-loops and duplicates removed,
   symmetrised); for small hand-made graphs. */
gg_csr* gg_from_edges(int64_t n, int64_t count, const int64_t* src, const int64_t* dst, int* status) {
  *status = -1;
  if (n < 1 || n > 2147483647LL || count < 0) return nullptr;
  for (int64_t k = 0; k < count; ++k)
    if (src[k] < 0 || src[k] >= n || dst[k] < 0 || dst[k] >= n) return nullptr;
  auto edge = [&](int64_t k, uint32_t& u, uint32_t& v) {
    u = (uint32_t)src[k];
    v = (uint32_t)dst[k];
  };
  Csr csr;
  *status = build_csr(n, count, edge, &csr);
  if (*status) return nullptr;
  gg_csr* g = new (std::nothrow) gg_csr{csr.n, csr.m, csr.offsets, csr.indices};
  if (!g) *status = -3;
  return g;
}

void gg_csr_free(gg_csr* g) {
  if (!g) return;
  std::free(g->offsets);
  std::free(g->indices);
  delete g;
}

/* The candidate sequence behind gg_sample_roots: out[i] = candidate number
   first+i, uniform in [0, n). */
void gg_root_candidates(int64_t n, uint64_t seed, int64_t first, int64_t count, int64_t* out) {
  const uint64_t key = gg_stream_key(seed, GG_STREAM_ROOTS);
  for (int64_t i = 0; i < count; ++i) out[i] = (int64_t)gg_below(gg_draw(key, (uint64_t)(first + i)), (uint64_t)n);
}

/* `count` distinct roots, uniform over the vertices of degree >= 1, drawn in
   order from the ROOTS stream of `seed`.  Returns the number found. */
int64_t gg_sample_roots(const int64_t* offsets, int64_t n, uint64_t seed, int64_t count, int64_t* out) {
  const uint64_t key = gg_stream_key(seed, GG_STREAM_ROOTS);
  int64_t found = 0;
  const uint64_t limit = (uint64_t)n * 64ull + 4096ull;
  for (uint64_t ctr = 0; found < count && ctr < limit; ++ctr) {
    const int64_t cand = (int64_t)gg_below(gg_draw(key, ctr), (uint64_t)n);
    if (offsets[cand + 1] - offsets[cand] < 1) continue;
    bool dup = false;
    for (int64_t i = 0; i < found; ++i) dup |= (out[i] == cand);
    if (!dup) out[found++] = cand;
  }
  return found;
}

}  // extern "C"
