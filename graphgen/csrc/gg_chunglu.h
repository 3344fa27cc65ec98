/*
 * The Chung-Lu power-law family with path tails, shared by the host and the
 * device builders so that both produce the same graph bit for bit:
 *
 *   - expected-degree weights w_i = c (i0 + i)^(-p), p = 1/(gamma-1), with
 *     i0 and c solved so that w_0 = max_deg and the mean weight is avg_deg;
 *   - a Walker/Vose alias table over the weights (built once, sequentially,
 *     on the host; thresholds quantised to 32 bits), through which both
 *     endpoints of each of round(n_core*avg_deg/2) core edges are drawn,
 *     then relabelled by a seeded bijection of [0, n_core);
 *   - n_tails path tails of tail_len new vertices, tail t's first vertex
 *     linked to an anchor: a uniform core vertex with at least one non-loop
 *     generated edge.
 *
 * Nothing here performs a breadth-first search.
 */
#ifndef GG_CHUNGLU_H
#define GG_CHUNGLU_H

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "gg_rng.h"

/* Weight constants (i0, c) for n vertices; 0 on success. */
static inline int gg_cl_weights(int64_t n, double gamma, double avg_deg, double max_deg, double* i0_out,
                                double* c_out) {
  if (n < 2 || gamma <= 1.0 || avg_deg <= 0 || max_deg <= avg_deg) return -1;
  const double p = 1.0 / (gamma - 1.0);
  /* mean(i0) = (max_deg * i0^p / n) * sum_i (i0+i)^(-p), increasing in i0.
     The sum is exact over its first K terms and the midpoint-rule integral
     beyond (relative error far below 1e-9 for K = 1e5). */
  const int64_t K = std::min<int64_t>(n, 100000);
  auto mean_for = [&](double i0) {
    double s = 0.0;
    for (int64_t i = 0; i < K; ++i) s += std::pow(i0 + (double)i, -p);
    if (K < n) {
      const double a = i0 + (double)K - 0.5, b = i0 + (double)n - 0.5;
      s += (std::pow(b, 1.0 - p) - std::pow(a, 1.0 - p)) / (1.0 - p);
    }
    return max_deg * std::pow(i0, p) * s / (double)n;
  };
  double lo = 1e-9, hi = 1.0;
  while (mean_for(hi) < avg_deg) {
    hi *= 2.0;
    if (hi > 1e18) return -2;
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mean_for(mid) < avg_deg) lo = mid; else hi = mid;
    if (hi - lo <= 1e-12 * hi) break;
  }
  *i0_out = 0.5 * (lo + hi);
  *c_out = max_deg * std::pow(*i0_out, p);
  return 0;
}

/* Walker/Vose alias table over w_i = c (i0+i)^(-p), i < n_core: slot s
   keeps s when the 32-bit coin is below thr[s], else takes alias[s]. */
static inline void gg_cl_alias(int64_t n_core, double i0, double c, double p, std::vector<uint32_t>& thr,
                               std::vector<int32_t>& alias) {
  std::vector<double> w((size_t)n_core);
  double total = 0.0;
  for (int64_t i = 0; i < n_core; ++i) {
    w[(size_t)i] = c * std::pow(i0 + (double)i, -p);
    total += w[(size_t)i];
  }
  thr.assign((size_t)n_core, 0u);
  alias.assign((size_t)n_core, 0);
  std::vector<double> q((size_t)n_core);
  std::vector<int64_t> small, large;
  small.reserve((size_t)n_core);
  large.reserve((size_t)n_core);
  for (int64_t i = 0; i < n_core; ++i) {
    q[(size_t)i] = w[(size_t)i] * (double)n_core / total;
    (q[(size_t)i] < 1.0 ? small : large).push_back(i);
  }
  while (!small.empty() && !large.empty()) {
    const int64_t s = small.back(); small.pop_back();
    const int64_t l = large.back();
    const double qs = q[(size_t)s];
    thr[(size_t)s] = (uint32_t)std::min(4294967295.0, std::floor(qs * 4294967296.0));
    alias[(size_t)s] = (int32_t)l;
    q[(size_t)l] = (q[(size_t)l] + qs) - 1.0;
    if (q[(size_t)l] < 1.0) { large.pop_back(); small.push_back(l); }
  }
  for (int64_t i : large) { thr[(size_t)i] = 0xFFFFFFFFu; alias[(size_t)i] = (int32_t)i; }
  for (int64_t i : small) { thr[(size_t)i] = 0xFFFFFFFFu; alias[(size_t)i] = (int32_t)i; }
}

/* Everything that fixes the core edges. */
typedef struct {
  uint64_t key, pkey;   /* CL_EDGES and PERM sub-stream keys */
  int64_t n_core;
  int32_t pbits;        /* gg_bits_for(n_core) */
  int32_t pad;
  const uint32_t* thr;  /* alias table (host or device memory, as the caller runs) */
  const int32_t* alias;
} gg_cl_core_t;

GG_FN uint32_t gg_cl_endpoint(const gg_cl_core_t& t, uint64_t x_slot, uint64_t x_coin) {
  const uint64_t s = gg_below(x_slot, (uint64_t)t.n_core);
  const uint32_t pick = ((uint32_t)x_coin < t.thr[s]) ? (uint32_t)s : (uint32_t)t.alias[s];
  return gg_permute_n(t.pkey, t.pbits, (uint64_t)t.n_core, pick);
}

/* Endpoints of core edge number k: draws 4k .. 4k+3 of the edge stream. */
GG_FN void gg_cl_core_edge(const gg_cl_core_t& t, int64_t k, uint32_t* u, uint32_t* v) {
  const uint64_t base = (uint64_t)k * 4ull;
  *u = gg_cl_endpoint(t, gg_draw(t.key, base + 0), gg_draw(t.key, base + 1));
  *v = gg_cl_endpoint(t, gg_draw(t.key, base + 2), gg_draw(t.key, base + 3));
}

/* Tail anchors from the marks of core vertices with a non-loop generated
   edge: candidates drawn in order from the CL_TAILS sub-stream, first
   marked one per tail.  0 on success. */
static inline int gg_cl_anchors(int64_t n_core, uint64_t seed, int32_t n_tails, const uint8_t* has_edge,
                                uint32_t* anchor) {
  const uint64_t tkey = gg_stream_key(seed, GG_STREAM_CL_TAILS);
  uint64_t ctr = 0;
  for (int32_t t = 0; t < n_tails; ++t) {
    for (;;) {
      const uint64_t cand = gg_below(gg_draw(tkey, ctr++), (uint64_t)n_core);
      if (has_edge[(size_t)cand]) { anchor[t] = (uint32_t)cand; break; }
      if (ctr > (uint64_t)n_core * 64ull + 4096ull) return -2;
    }
  }
  return 0;
}

/* Edge k of the whole stream: core edges first, then each tail's anchor
   link and chain (tail t vertex j is n_core + t*tail_len + j). */
GG_FN void gg_cl_edge(const gg_cl_core_t& t, int64_t m_core, const uint32_t* anchor, int64_t tail_len, int64_t k,
                      uint32_t* u, uint32_t* v) {
  if (k < m_core) {
    gg_cl_core_edge(t, k, u, v);
    return;
  }
  const int64_t r = k - m_core;
  const int64_t tt = r / tail_len, j = r % tail_len;
  const uint32_t first = (uint32_t)(t.n_core + tt * tail_len);
  if (j == 0) { *u = anchor[tt]; *v = first; }
  else { *u = first + (uint32_t)(j - 1); *v = first + (uint32_t)j; }
}

#endif /* GG_CHUNGLU_H */
