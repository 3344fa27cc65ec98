/*
 * Seeded, counter-based building blocks of the synthetic graph inputs.
 *
 * Everything here is a pure function of (seed, counter), so the host builder
 * and the device builder produce bit-identical edge streams whatever the
 * thread count, chunking or launch shape.  Nothing in this file performs a
 * breadth-first search: it only describes which edges a synthetic graph has.
 *
 *   - gg_mix64 / gg_draw: the SplitMix64 generator of Steele, Lea and Flood
 *     ("Fast splittable pseudorandom number generators", OOPSLA 2014): a Weyl
 *     sequence with increment 0x9E3779B97F4A7C15 passed through its 64-bit
 *     finaliser.  gg_draw(key, c) is output number c of the generator whose
 *     state starts at key, so any output can be computed directly.
 *   - gg_rmat_edge: the recursive-matrix (R-MAT / Kronecker) edge model used
 *     by Graph500-style synthetic graphs: at each of `scale` bit levels one
 *     quadrant of the adjacency matrix is chosen with probabilities A, B, C,
 *     D = 1-A-B-C.  Quadrant thresholds are fixed 32-bit integers so both
 *     builders compare identical integers.
 *   - gg_permute: a keyed bijection of [0, 2^scale) (a 4-round balanced
 *     Feistel network on 2*ceil(scale/2) bits with cycle walking), used as
 *     the seeded random vertex relabelling that hides the R-MAT structure in
 *     the vertex IDs.
 */
#ifndef GG_RNG_H
#define GG_RNG_H

#include <stdint.h>

#if defined(__HIPCC__)
#define GG_FN __host__ __device__ static inline
#else
#define GG_FN static inline
#endif

#define GG_GOLDEN 0x9E3779B97F4A7C15ull

/* Independent sub-streams of one seed. */
enum { GG_STREAM_EDGES = 1, GG_STREAM_PERM = 2, GG_STREAM_ROOTS = 3,
       GG_STREAM_CL_EDGES = 4, GG_STREAM_CL_TAILS = 5 };

GG_FN uint64_t gg_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Output number `ctr` of the SplitMix64 sequence whose state starts at key. */
GG_FN uint64_t gg_draw(uint64_t key, uint64_t ctr) {
  return gg_mix64(key + (ctr + 1ull) * GG_GOLDEN);
}

/* Key of sub-stream `stream` of `seed`. */
GG_FN uint64_t gg_stream_key(uint64_t seed, uint64_t stream) {
  return gg_mix64(seed ^ gg_mix64((stream + 1ull) * GG_GOLDEN));
}

/* Uniform integer in [0, n) from a 64-bit draw (multiply-high). */
GG_FN uint64_t gg_below(uint64_t x, uint64_t n) {
  return (uint64_t)(((unsigned __int128)x * (unsigned __int128)n) >> 64);
}

/* Cumulative quadrant thresholds over 2^32: x < a -> A, x < ab -> B,
   x < abc -> C, otherwise D. */
typedef struct { uint32_t a, ab, abc; } gg_rmat_t;

/* Endpoints (before relabelling) of R-MAT edge number k at the given scale
   (1 <= scale <= 31).  Level b (0 = most significant bit) uses 32-bit
   uniform number b of the edge: draws 2j and 2j+1 are the low and high
   halves of gg_draw(key, 16k + j). */
GG_FN void gg_rmat_edge(uint64_t key, int scale, gg_rmat_t t, uint64_t k,
                        uint32_t* u_out, uint32_t* v_out) {
  uint32_t u = 0, v = 0;
  const int words = (scale + 1) >> 1;
  for (int j = 0; j < words; ++j) {
    const uint64_t r = gg_draw(key, k * 16ull + (uint64_t)j);
    for (int h = 0; h < 2; ++h) {
      if (2 * j + h >= scale) break;
      const uint32_t x = (uint32_t)(r >> (32 * h));
      const uint32_t ubit = (x >= t.ab) ? 1u : 0u;                      /* C or D */
      const uint32_t vbit = ((x >= t.a && x < t.ab) || x >= t.abc) ? 1u : 0u; /* B or D */
      u = (u << 1) | ubit;
      v = (v << 1) | vbit;
    }
  }
  *u_out = u;
  *v_out = v;
}

/* One pass of the 4-round Feistel network on 2*hbits bits (hbits <= 16). */
GG_FN uint32_t gg_feistel(uint64_t key, int hbits, uint32_t x) {
  const uint32_t mask = (hbits >= 32) ? 0xFFFFFFFFu : ((1u << hbits) - 1u);
  uint32_t l = (x >> hbits) & mask, r = x & mask;
  for (uint64_t round = 0; round < 4; ++round) {
    const uint32_t f = (uint32_t)gg_draw(key, (round << 32) | (uint64_t)r) & mask;
    const uint32_t nl = r;
    r = l ^ f;
    l = nl;
  }
  return (l << hbits) | r;
}

/* Keyed bijection of [0, 2^scale), 1 <= scale <= 31. */
GG_FN uint32_t gg_permute(uint64_t key, int scale, uint32_t x) {
  const int h = (scale + 1) >> 1;
  uint32_t y = gg_feistel(key, h, x);
  while ((uint64_t)y >> scale) y = gg_feistel(key, h, y);
  return y;
}

/* Keyed bijection of [0, n) for n <= 2^bits (bits = gg_bits_for(n)): the
   Feistel network of gg_permute on 2*ceil(bits/2) bits, cycle-walked into
   [0, n). */
GG_FN uint32_t gg_permute_n(uint64_t key, int bits, uint64_t n, uint32_t x) {
  const int h = (bits + 1) >> 1;
  uint32_t y = gg_feistel(key, h, x);
  while ((uint64_t)y >= n) y = gg_feistel(key, h, y);
  return y;
}

/* Smallest b >= 1 with 2^b >= n. */
GG_FN int gg_bits_for(uint64_t n) {
  int b = 1;
  while ((1ull << b) < n) ++b;
  return b;
}

#endif /* GG_RNG_H */
