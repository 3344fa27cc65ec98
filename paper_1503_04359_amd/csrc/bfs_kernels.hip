/*
 * Level kernels of direction-optimized BFS for gfx950 (wave64).
 *
 * One level L expands the frontier F_L (vertices of depth L) into F_{L+1}:
 *   top-down  (Algorithm 1, top-down branch): every vertex u of the queue
 *             Q_L examines each neighbour v; an unvisited v is claimed with an
 *             atomic OR on its visited bit, so exactly one u becomes its
 *             parent (the algorithm's check-then-set, made race-free);
 *   bottom-up (Algorithm 1, bottom-up branch): every unvisited vertex v
 *             scans its adjacency list in order and stops at the first
 *             neighbour u in F_L (a frontier-bitmap test), with u as parent.
 *             The frontier tested is F_L, not the visited set.
 * After each level the last workgroup to finish applies the switching rule
 * (Section 3.3) to on-device counters, so no level needs the host.
 *
 * Mapping to the hardware:
 *   - bottom-up: lane i of a wavefront owns vertex 64w+i of each 64-vertex
 *     visited word w it takes.  Fully visited words are skipped
 *     wave-uniformly, the new frontier word is the wave's ballot and
 *     visited |= ballot is one plain store: bottom-up needs no atomics.
 *     Round 0 (each vertex's first neighbour) runs for four words at a time
 *     with all their loads in flight together; the vertices that miss are
 *     searched in a second pass over the same words, in rounds of growing
 *     per-vertex quotas (at most max(64, bu_heavy_cut) per round) laid end
 *     to end over the 64 lanes, so work inside a word is balanced across
 *     lanes (see bottom_up).  Probes of the hub region of the frontier read
 *     an LDS copy.
 *   - top-down: degree-binned (the virtual-warp idea of Section 2.1 on
 *     64-wide wavefronts): a lane per vertex up to td_wave_cut, a wavefront
 *     per vertex up to td_huge_cut, and above that the vertex's edges are
 *     cut into kHugeChunk-edge tasks spread over all wavefronts by the aux
 *     kernel.
 *   - frontier representations: a level produces the next frontier as a
 *     bitmap (top-down sets bits with atomic OR, bottom-up writes whole
 *     words).  Before a large top-down level the aux kernel turns that
 *     bitmap into a queue with one atomic per workgroup, and clears the
 *     other bitmap buffer, which the top-down level then fills.  A small
 *     top-down level also appends its claims to a direct queue that the
 *     next top-down level reads as is.  Bitmap buffer F[L%2] holds F_L.
 */
#include <hip/hip_runtime.h>

#include "dobfs_internal.h"
#include "device_common.h"

namespace dobfs {
namespace {

__device__ __forceinline__ int random_dir(uint64_t seed, int32_t level) {
  uint64_t z = seed + (uint64_t)(level + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (int)(z & 1ull);
}

/* End of level L (all of its edges examined): log it, apply the switching
   rule and set up level L+1.  Runs in one thread. */
__device__ void decide(const GView& g, const WView& w, const KParams& kp) {
  Ctl* c = w.ctl;
  const int32_t L = c->level;
  const int32_t dir = c->dir;
  const int64_t nfn = ld_agent(&c->nf_next);
  const int64_t mfn = ld_agent(&c->mf_next);
  const int64_t chk = ld_agent(&c->checked);
  const int64_t scn = ld_agent(&c->scanned);
  const int64_t mu = c->m_u;
  if (c->log_len < w.log_cap) {
    dobfs_level_rec r;
    r.level = L;
    r.dir = dir;
    r.n_f = c->n_f;
    r.m_f = c->m_f;
    r.m_u = mu;
    r.scanned = scn;
    r.checked = chk;
    r.found = nfn;
    r.found_deg = mfn;
    r.t_end = wall_clock64();
    r.kernel_ms = 0.f;
    r.reserved = 0;
    w.log[c->log_len] = r;
    c->log_len = c->log_len + 1;
  }
  c->reached += nfn;
  c->reached_deg += mfn;
  c->checked_total += chk;
  const int64_t mu_next = mu - mfn;
  int next = dir;
  int32_t bu_run = (dir == kDirBU) ? c->bu_run + 1 : 0;
  if (nfn == 0) {
    c->done = 1;
    c->levels = L + 1;
  } else {
    switch (kp.policy) {
      case DOBFS_POLICY_EDGE:
        if (dir == kDirTD) next = (mfn * (int64_t)kp.alpha > mu_next) ? kDirBU : kDirTD;
        else next = (nfn < c->n_f && nfn * (int64_t)kp.beta < g.n) ? kDirTD : kDirBU;
        break;
      case DOBFS_POLICY_PAPER:
        if (dir == kDirTD)
          next = (c->bu_phases == 0 && mfn * (int64_t)kp.paper_pct > (g.n / kp.paper_div) * 100) ? kDirBU : kDirTD;
        else
          next = (bu_run >= kp.paper_bu_steps) ? kDirTD : kDirBU;
        break;
      case DOBFS_POLICY_COST: {
        const int64_t unvisited = g.n_nonisolated - (c->reached + nfn);
        if (dir == kDirTD) next = (mfn * 1000 > (int64_t)kp.kappa_x1000 * unvisited) ? kDirBU : kDirTD;
        else next = (nfn < c->n_f && nfn * (int64_t)kp.beta < g.n) ? kDirTD : kDirBU;
        break;
      }
      case DOBFS_POLICY_FORCED_TD: next = kDirTD; break;
      case DOBFS_POLICY_FORCED_BU: next = kDirBU; break;
      default: next = random_dir(kp.seed, L + 1); break;
    }
  }
  if (dir == kDirTD && next == kDirBU) c->bu_phases = c->bu_phases + 1;
  /* a top-down level that appended its claims hands its queue on as is;
     otherwise the next top-down level's queue is built from the bitmap */
  const bool appended = dir == kDirTD && c->q_append;
  const bool next_td = !c->done && next == kDirTD;
  c->aux = (next_td && !appended) ? kAuxToQueue : kAuxNone;
  c->q_direct = (next_td && appended) ? 1 : 0;
  c->q_append = (next_td && mfn <= (int64_t)kDirectCap) ? 1 : 0;
  c->qd_fill = 0ull;
  c->bu_run = bu_run;
  c->n_f = nfn;
  c->m_f = mfn;
  c->m_u = mu_next;
  c->dir = next;
  c->level = L + 1;
  c->nf_next = 0;
  c->mf_next = 0;
  c->checked = 0;
  c->scanned = 0;
  c->huge_pack = 0ull;
  c->q_fill = 0;
}

/* Writes the labels of a newly reached vertex: the caller's depth/parent
   arrays, or (relabelled graphs) one packed (parent << 32 | depth) word in
   internal labels that the finalize kernel maps back.  When the parent's
   caller ID pc is already at hand (pc >= 0) it is stored instead, flagged
   by kCallerParent in the depth field, and the finalize kernel uses it as
   is. */
constexpr uint32_t kCallerParent = 0x80000000u;

__device__ __forceinline__ void store_labels(const WView& w, int32_t v, int32_t d, int32_t p, int32_t pc = -1) {
  if (w.packed) {
    const uint64_t pf = (uint64_t)(uint32_t)(pc >= 0 ? pc : p);
    const uint64_t df = (uint64_t)((uint32_t)d | (pc >= 0 ? kCallerParent : 0u));
    w.packed[v] = (int64_t)((pf << 32) | df);
  } else {
    w.depth[v] = d;
    w.parent[v] = p;
  }
}

/* Bookkeeping of a vertex v claimed from u (caller ID uc, or -1) at level L:
   labels, next-frontier bit and the degree sum that feeds the switching
   rule. */
__device__ __forceinline__ void claimed(const GView& g, const WView& w, uint64_t* f_nxt, int32_t* q_app, int32_t v,
                                        int32_t u, int32_t uc, int32_t L, Acc& a) {
  store_labels(w, v, L + 1, u, uc);
  atomicOr(reinterpret_cast<unsigned long long*>(f_nxt + (v >> 6)), 1ull << (v & 63));
  if (q_app) q_app[atomicAdd(&w.ctl->qd_fill, 1ull)] = v;
  a.found += 1;
  a.found_deg += g.off[v + 1] - g.off[v];
}

/* Claims for J neighbour IDs of one lane (v[j] < 0: none), all from
   frontier vertex u (caller ID uc): each step (visited words, claim
   atomics, the winners' row bounds) is issued for all J before any result
   is used, so a lane has J independent accesses in flight instead of J
   dependent chains in a row.  Lanes with nothing to load read index 0 (in
   bounds) and are masked. */
template <int J>
__device__ __forceinline__ void claim_batch(const GView& g, const WView& w, uint64_t* f_nxt, int32_t* q_app,
                                            const int32_t (&v)[J], int32_t u, int32_t uc, int32_t L, Acc& a) {
  uint32_t* vis32 = reinterpret_cast<uint32_t*>(w.vis);
  const uint32_t* off_lo = reinterpret_cast<const uint32_t*>(g.off);
  uint32_t vw[J], old[J];
#pragma unroll
  for (int j = 0; j < J; ++j) vw[j] = vis32[v[j] >= 0 ? (uint32_t)v[j] >> 5 : 0u];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    old[j] = ~0u;
    const uint32_t bit = 1u << (v[j] & 31);
    if (v[j] >= 0 && !(vw[j] & bit)) old[j] = atomicOr(vis32 + ((uint32_t)v[j] >> 5), bit);
  }
  uint32_t won = 0u;
#pragma unroll
  for (int j = 0; j < J; ++j)
    if (!(old[j] & (1u << (v[j] & 31)))) won |= 1u << j;
  uint32_t ob[J], oe[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const uint32_t x = ((won >> j) & 1u) ? (uint32_t)v[j] : 0u;
    ob[j] = off_lo[2 * (uint64_t)x];
    oe[j] = off_lo[2 * (uint64_t)x + 2];
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    if ((won >> j) & 1u) {
      store_labels(w, v[j], L + 1, u, uc);
      atomicOr(reinterpret_cast<uint32_t*>(f_nxt) + ((uint32_t)v[j] >> 5), 1u << (v[j] & 31));
      if (q_app) q_app[atomicAdd(&w.ctl->qd_fill, 1ull)] = v[j];
      a.found += 1;
      a.found_deg += (int32_t)(oe[j] - ob[j]);  /* degrees fit in 31 bits */
    }
  }
}

/* Top-down level L, as workgroup vb of the nblocks workgroups that share its
   queue. */
__device__ void top_down(const GView& g, const WView& w, const KParams& kp, int32_t L, uint32_t vb, uint32_t nblocks,
                         Acc& a) {
  Ctl* c = w.ctl;
  /* control fields may have been written by this workgroup's own previous
     level (see level_body): read them from L2 */
  const int64_t nf = ld_agent(&c->n_f);
  const int32_t* q_cur = ld_agent(&c->q_direct) ? ((L & 1) ? w.qd1 : w.qd0) : w.q0;
  uint64_t* f_cur = (L & 1) ? w.fr1 : w.fr0;
  uint64_t* f_nxt = (L & 1) ? w.fr0 : w.fr1;
  /* a small level appends its claims to the next queue and clears its own
     frontier bits, leaving that buffer empty for the next level to fill */
  const bool append = ld_agent(&c->q_append) != 0;
  int32_t* q_app = append ? ((L & 1) ? w.qd0 : w.qd1) : nullptr;
  const int lane = lane_id();
  const int64_t wave = ((int64_t)vb * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)nblocks * blockDim.x) / kWave;
  const int64_t wave_cut = kp.td_wave_cut, huge_cut = kp.td_huge_cut;

  for (int64_t base = wave * kWave; base < nf; base += nwaves * kWave) {
    const int64_t i = base + lane;
    const bool valid = i < nf;
    int32_t u = 0, uc = -1;
    int64_t beg = 0, deg = 0;
    if (valid) {
      u = q_cur[i];
      beg = g.off[u];
      deg = g.off[u + 1] - beg;
      if (g.new2old) uc = g.new2old[u]; /* one lookup per frontier vertex, not per claim */
      if (append) atomicAnd(reinterpret_cast<unsigned long long*>(f_cur + (u >> 6)), ~(1ull << (u & 63)));
    }
    a.checked += deg;
    const bool huge = valid && deg > huge_cut;
    const bool med = !huge && deg > wave_cut;

    /* lane per vertex */
    const int64_t sdeg = (valid && !huge && !med) ? deg : 0;
    constexpr int JS = 2;  /* two at a time: the kernel's register budget allows no more */
    for (int64_t j0 = 0; j0 < sdeg; j0 += JS) {
      int32_t v[JS];
#pragma unroll
      for (int j = 0; j < JS; ++j) {
        v[j] = g.idx[beg + min(j0 + j, sdeg - 1)];  /* in the row */
        if (j0 + j >= sdeg) v[j] = -1;
      }
      claim_batch<JS>(g, w, f_nxt, q_app, v, u, uc, L, a);
    }

    /* wavefront per vertex */
    uint64_t mm = __ballot(med);
    while (mm) {
      const int src = __ffsll((unsigned long long)mm) - 1;
      mm &= mm - 1;
      const int32_t uu = __shfl(u, src), uuc = __shfl(uc, src);
      const int64_t bb = __shfl(beg, src);
      const int64_t dd = __shfl(deg, src);
      for (int64_t k = lane; k < dd; k += kWave) {
        const int32_t v = g.idx[bb + k];
        if (try_claim(w.vis, v)) claimed(g, w, f_nxt, q_app, v, uu, uuc, L, a);
      }
    }

    /* split vertices: defer to the aux kernel.  One atomic per wavefront
       reserves consecutive list entries and consecutive chunk numbers, so
       chunk bases increase with the entry index. */
    const uint64_t hm = __ballot(huge);
    if (hm) {
      const int nch = huge ? (int)((deg + kHugeChunk - 1) / kHugeChunk) : 0;
      const int incl = wave_incl_scan(nch, lane);
      const int tot = __shfl(incl, kWave - 1);
      unsigned long long old = 0;
      if (lane == 0)
        old = atomicAdd(reinterpret_cast<unsigned long long*>(&c->huge_pack),
                        ((unsigned long long)__popcll(hm) << 32) | (unsigned long long)tot);
      old = __shfl(old, 0);
      if (huge) {
        const uint32_t slot = (uint32_t)(old >> 32) + (uint32_t)__builtin_amdgcn_mbcnt_hi(
            (uint32_t)(hm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)hm, 0));
        w.huge_u[slot] = u;
        w.huge_base[slot] = (uint32_t)(old & 0xFFFFFFFFull) + (uint32_t)(incl - nch);
      }
    }
  }
}

/* One 64-entry chunk [c0, c0+64) of a bottom-up round: this lane's slice of
   it is [max(excl,c0), min(incl,c0+64)); H marks the entries that hit the
   frontier.  Records the first hit of the slice as the lane's parent. */
__device__ __forceinline__ void resolve_chunk(uint64_t H, int c0, int excl, int incl, int take, int32_t u,
                                              bool& found, int32_t& par, int32_t& checked) {
  const int lane = lane_id();
  const int sa = max(excl, c0) - c0, sb = min(incl, c0 + kWave) - c0;
  int src = lane;
  bool got = false;
  if (take > 0 && sa < sb && !found) {
    const uint64_t span = (sb - sa >= 64) ? ~0ull : (((1ull << (sb - sa)) - 1ull) << sa);
    const uint64_t h = H & span;
    if (h) {
      src = __ffsll((unsigned long long)h) - 1;
      got = true;
      checked += src - sa + 1;
    } else {
      checked += sb - sa;
    }
  }
  const int32_t pu = __shfl(u, src);
  if (got) {
    found = true;
    par = pu;
  }
}

/* Frontier bit of u: from the workgroup's LDS copy of the bitmap's first
   kBuHot32 words when u falls there, else from the bitmap.  Both loads are
   issued (the other one at a shared, in-bounds address) so that no load sits
   under a branch. */
__device__ __forceinline__ uint32_t frontier_word(const uint32_t* hot, const uint32_t* f32, uint32_t u) {
  const uint32_t wi = u >> 5;
  const bool in_hot = wi < (uint32_t)kBuHot32;
  const uint32_t h = hot[in_hot ? wi : 0u];
  const uint32_t gw = f32[in_hot ? 0u : wi];
  return in_hot ? h : gw;
}

/* Rounds after round 0 for one word of a bottom-up level: each vertex still
   searching contributes its next min(2^(r+1), remaining) neighbours (at
   most max_quota), the contributions are laid end to end and cut into
   64-entry chunks (two chunks in flight at a time), and each lane tests one
   neighbour.  Every
   lane does useful work even when degrees differ inside the word, one
   vertex's neighbour IDs are read contiguously, and a vertex stops at the
   round in which it meets its first frontier neighbour (its parent: the
   first hit in adjacency order). */
__device__ __forceinline__ void bu_rounds(const GView& g, const uint32_t* hot, const uint32_t* f32, int max_quota,
                                          int64_t pos, int64_t end, bool& found, int32_t& par, int32_t& n_checked) {
  const int lane = lane_id();
  int quota = 4;  /* measured: 4 beats 2 and 8 on sparse frontiers of scale-free graphs */
  while (__ballot(!found && pos < end)) {
    const int take = (!found && pos < end) ? (int)min(end - pos, (int64_t)quota) : 0;
    const int incl = wave_incl_scan(take, lane);
    const int excl = incl - take;
    const int total = __shfl(incl, kWave - 1);
    for (int c0 = 0; c0 < total; c0 += 2 * kWave) {
      const int p1 = c0 + lane, p2 = c0 + kWave + lane;
      const int o1 = owner_of(incl, p1), o2 = owner_of(incl, p2);
      const int64_t e1 = __shfl(pos, o1) + (p1 - __shfl(excl, o1));
      const int64_t e2 = __shfl(pos, o2) + (p2 - __shfl(excl, o2));
      int32_t u1 = 0, u2 = 0;
      if (p1 < total) u1 = g.idx[e1];
      if (p2 < total) u2 = g.idx[e2];
      const bool h1 = p1 < total && ((frontier_word(hot, f32, (uint32_t)u1) >> (u1 & 31)) & 1u);
      const bool h2 = p2 < total && ((frontier_word(hot, f32, (uint32_t)u2) >> (u2 & 31)) & 1u);
      const uint64_t H1 = __ballot(h1), H2 = __ballot(h2);
      resolve_chunk(H1, c0, excl, incl, take, u1, found, par, n_checked);
      resolve_chunk(H2, c0 + kWave, excl, incl, take, u2, found, par, n_checked);
    }
    pos += take;
    if (quota < max_quota) quota <<= 1;
  }
}

/* Bottom-up level, in two passes over the same words, each wavefront
   keeping its own words in both (so the second pass reads only what the
   same wavefront wrote in the first).

   Pass 1 takes kBuWords consecutive 64-vertex words at a time; lane i owns
   vertex 64w+i of each.  Round 0 of all of them is issued together, so that
   their dependent loads (visited word, row bounds and first neighbour,
   frontier bit, the parent's caller ID) overlap instead of following one
   another word by word: every unvisited vertex tests its first neighbour
   (its highest-degree one on a relabelled graph), read from the
   first-neighbour column in one coalesced load.  A word whose vertices all
   settle here is finished at once; for a word with vertices left to search,
   the round-0 hits and the searching vertices are recorded as two masks in
   the queue buffer, which bottom-up levels do not otherwise use.

   Pass 2 runs the later rounds (bu_rounds) for the recorded words, one
   word at a time, and finishes them.  Splitting the passes keeps each within
   64 registers: round 0 of several words and the rounds' own state are
   never live together. */
__device__ void bottom_up(const GView& g, const WView& w, const KParams& kp, int32_t L, Acc& a) {
  constexpr int K = kBuWords;
  const uint64_t* f_cur = (L & 1) ? w.fr1 : w.fr0;
  uint64_t* f_nxt = (L & 1) ? w.fr0 : w.fr1;
  uint64_t* rec = reinterpret_cast<uint64_t*>(w.q0);  /* word wd: [2wd] hits, [2wd+1] searching */
  const int lane = lane_id();
  const int64_t wave = wave_index();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int max_quota = kp.bu_heavy_cut < kWave ? kWave : kp.bu_heavy_cut;
  const int64_t W = g.words_active;
  /* per-lane counts in 32 bits (a lane sees far fewer than 2^31 entries per
     level); they join the 64-bit accumulators once at the end */
  int32_t n_scanned = 0, n_checked = 0, n_found = 0;
  /* The start of the frontier bitmap is staged in LDS: on a relabelled
     graph it holds the highest-degree vertices, which most probes hit (a
     vertex's neighbours are scanned highest degree first), and an LDS read
     spares the vector cache a scattered line access.  Words past the active
     range read as zero; no probe reaches them (isolated vertices are no
     one's neighbours). */
  __shared__ uint32_t hot[kBuHot32];
  const uint32_t* f32 = reinterpret_cast<const uint32_t*>(f_cur);
  for (int i = threadIdx.x; i < kBuHot32; i += blockDim.x) hot[i] = i < 2 * W ? f32[i] : 0u;
  __syncthreads();

  /* A wavefront's word groups are wb = (wave + j * nwaves) * K, j = 0, 1, ...
     Both passes take G of them per step, one word per lane (lane = g * K + k:
     word k of the step's group g), so a level with most vertices already
     visited costs one load and one store per lane for G groups instead of a
     step per group. */
  constexpr int G = kWave / K;
  static_assert(kWave % K == 0, "a wavefront holds whole word groups");
  /* the lane's word is the step's first word (wave-uniform) plus my_off */
  const uint32_t my_off = (uint32_t)((lane / K) * nwaves * K + (lane % K));

  /* ---- pass 1: round 0 ---- */
  for (int64_t j0 = 0; (wave + j0 * nwaves) * K < W; j0 += G) {
    const int64_t sb = (wave + j0 * nwaves) * K;
    const bool my_ok = (int64_t)my_off < W - sb;
    const uint64_t my_vis = my_ok ? w.vis[sb + my_off] : ~0ull;
    const uint64_t busy = __ballot(my_vis != ~0ull);
    /* every vertex of the lane's group visited: nothing reached, nothing to search */
    if (my_ok && !((busy >> (lane & ~(K - 1))) & ((1ull << K) - 1ull))) {
      (f_nxt + sb)[my_off] = 0ull;
      (rec + 2 * sb)[2 * my_off + 1] = 0ull;
    }
    uint64_t todo = busy;
    while (todo) {
      const int gsel = (__ffsll((unsigned long long)todo) - 1) / K;
      todo &= ~(((1ull << K) - 1ull) << (gsel * K));
      const int64_t wb = (wave + (j0 + gsel) * nwaves) * K;
      /* lanes 0..K-1: word wb+lane (~0 past the end) */
      const uint64_t vis_mine = __shfl(my_vis, gsel * K + (lane & (K - 1)));
      /* Every load is issued before any is used, and none sits under a
         branch (lanes with nothing to load read entry 0 of the word group,
         which is in bounds), so the compiler can wait for each one alone
         instead of for everything outstanding.  Addresses are a wave-uniform
         base plus a 32-bit lane offset. */
      const int64_t v0 = wb * kWave;
      const uint32_t* off_lo = reinterpret_cast<const uint32_t*>(g.off + v0);
      const int32_t* first = g.first + v0;
      uint32_t b[K], e[K], fw[K];
      int32_t u0[K], pcr[K];
      bool unv[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint64_t vw = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(vis_mine >> 32), k) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)vis_mine, k);
        unv[k] = ((vw >> lane) & 1ull) == 0ull;  /* bits >= n are set */
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int i = unv[k] ? k * kWave + lane : 0;
        /* degrees fit in 31 bits, so the low words of the row bounds give
           the degree */
        b[k] = off_lo[2 * i];
        e[k] = off_lo[2 * i + 2];
        u0[k] = first[i];
        /* the first neighbour's caller ID, in case it is the parent: loaded
           with the rest rather than after the frontier test */
        pcr[k] = g.first_caller ? g.first_caller[v0 + i] : -1;
      }
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (!unv[k]) e[k] = b[k];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t u = e[k] != b[k] ? (uint32_t)u0[k] : 0u;
        fw[k] = frontier_word(hot, f32, u);
      }
      uint32_t hit = 0u;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int32_t deg = (int32_t)(e[k] - b[k]);
        if (deg > 0 && ((fw[k] >> (u0[k] & 31)) & 1u)) hit |= 1u << k;
        n_scanned += unv[k] ? 1 : 0;
        n_checked += deg > 0 ? 1 : 0;
      }
      uint64_t my_hit = 0ull, my_srch = 0ull;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int32_t deg = (int32_t)(e[k] - b[k]);
        const bool h = (hit >> k) & 1u;
        if (h) {
          store_labels(w, (int32_t)(v0 + k * kWave + lane), L + 1, u0[k], pcr[k]);
          a.found_deg += deg;
          n_found += 1;
        }
        const uint64_t hm = __ballot(h), sm = __ballot(!h && deg > 1);
        if (lane == k) {
          my_hit = hm;
          my_srch = sm;
        }
      }
      if (lane < K && wb + lane < W) {
        const int64_t wd = wb + lane;
        rec[2 * wd + 1] = my_srch;
        if (my_srch) {
          rec[2 * wd] = my_hit;  /* finished in pass 2 */
        } else {
          f_nxt[wd] = my_hit;
          if (my_hit) w.vis[wd] = vis_mine | my_hit;
        }
      }
    }
  }
  /* pass 2 reads what other lanes of this wavefront stored in pass 1 */
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  /* ---- pass 2: later rounds of the recorded words ---- */
  for (int64_t j0 = 0; (wave + j0 * nwaves) * K < W; j0 += G) {
    const int64_t sb = (wave + j0 * nwaves) * K;
    const uint64_t my_srch = (int64_t)my_off < W - sb ? (rec + 2 * sb)[2 * my_off + 1] : 0ull;
    uint64_t todo = __ballot(my_srch != 0ull);
#pragma unroll 1
    while (todo) {
      const int li = __ffsll((unsigned long long)todo) - 1;
      todo &= todo - 1ull;
      const uint64_t sm = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(my_srch >> 32), li) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)my_srch, li);
      const int64_t wd = (wave + (j0 + li / K) * nwaves) * K + (li % K);
      const int32_t v = (int32_t)(wd * kWave + lane);
      const bool s = (sm >> lane) & 1ull;
      int64_t pos = 0, end = 0;
      if (s) {
        pos = g.off[v] + 1;  /* round 0 tested the first entry */
        end = g.off[v + 1];
      }
      bool found = !s;  /* only searching lanes take part */
      int32_t par = -1;
      bu_rounds(g, hot, f32, max_quota, pos, end, found, par, n_checked);
      const bool got = s && found;
      if (got) {
        store_labels(w, v, L + 1, par);
        a.found_deg += end - (pos - 1);
        n_found += 1;
      }
      const uint64_t fm = __ballot(got);
      if (lane == 0) {
        const uint64_t all = rec[2 * wd] | fm;
        f_nxt[wd] = all;
        if (all) w.vis[wd] |= all;
      }
    }
  }
  a.scanned += n_scanned;
  a.checked += n_checked;
  a.found += n_found;
}

/* The level kernels: top-down and bottom-up are separate kernels, both
   launched for every level, so that each gets its own register allocation;
   the one whose direction is not the level's returns at once.

   Completion protocol.  Every workgroup of the grid that finds the level in
   its direction reports to the completion count, also a top-down workgroup
   with no queue entries of its own (a top-down level needs only one queue
   entry per thread, i.e. ceil(n_f / kBlock) workgroups, and the others
   report empty counters).  The control state therefore cannot change
   before every workgroup of the launch has read it: a workgroup dispatched
   late, when other kernels hold the compute units, still sees the level
   the launch was enqueued for, and no ticket is left over for a later
   launch.

   The workgroup that closes a top-down level goes straight on to the next
   one when that level is again top-down, has its queue handed on directly
   and fits one workgroup: it runs it alone, as workgroup 0 of a
   one-workgroup level, since every other workgroup of the launch has
   already reported and left.  Long chains of tiny levels (path-like tails)
   cost a barrier each instead of a launch sequence each. */
template <int BT>
__device__ __forceinline__ void level_body(const GView& g, const WView& w, const KParams& kp, int32_t want_dir) {
  Ctl* c = w.ctl;
  if (ld_agent(&c->done) || ld_agent(&c->aux) != kAuxNone || ld_agent(&c->dir) != want_dir) return;
  for (bool alone = false;; alone = true) {
    const int32_t L = ld_agent(&c->level);
    const uint32_t vb = alone ? 0u : blockIdx.x;
    uint32_t nb = alone ? 1u : gridDim.x;
    if (want_dir == kDirTD) {
      const int64_t need = (ld_agent(&c->n_f) + kBlock - 1) / kBlock;
      if (need < (int64_t)nb) nb = need < 1 ? 1u : (uint32_t)need;
    }
    Acc a = {0, 0, 0, 0};
    if (vb < nb) {
      if (want_dir == kDirTD) top_down(g, w, kp, L, vb, nb, a);
      else bottom_up(g, w, kp, L, a);
    }
    if (!finish_block_all<BT>(c, a, alone ? 1u : 0u)) return;
    if (threadIdx.x == 0) {
      if (want_dir == kDirTD && ld_agent(&c->huge_pack) != 0ull) {
        c->aux = kAuxHuge;
      } else {
        decide(g, w, kp);
      }
    }
    if (want_dir != kDirTD) return;
    /* make thread 0's control writes and every workgroup's labels, bits and
       queue entries of this level visible to the whole workgroup */
    __threadfence();
    __syncthreads();
    __threadfence();
    if (ld_agent(&c->done) || ld_agent(&c->aux) != kAuxNone || ld_agent(&c->dir) != kDirTD ||
        !ld_agent(&c->q_direct) || ld_agent(&c->n_f) > (int64_t)kBlock)
      return;
  }
}

__global__ void __launch_bounds__(kBlock, 8) k_level_td(GView g, WView w, KParams kp) {
  level_body<kBlock>(g, w, kp, kDirTD);
}

/* Larger workgroups at the same occupancy (two per CU): each keeps a
   larger part of the frontier bitmap in LDS. */
__global__ void __launch_bounds__(kBuBlock, 8) k_level_bu(GView g, WView w, KParams kp) {
  level_body<kBuBlock>(g, w, kp, kDirBU);
}

/* Exclusive prefix sum over the workgroup; *total gets the sum. */
__device__ int64_t block_excl_scan(int64_t x, int64_t* total) {
  __shared__ int64_t wsum[kBlock / kWave];
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  int64_t incl = x;
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) wsum[wv] = incl;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int j = 0; j < kBlock / kWave; ++j) {
    if (j < wv) before += wsum[j];
    all += wsum[j];
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

/* Expands the split top-down vertices (kAuxHuge) or turns the frontier
   bitmap of a level about to run top-down into its queue (kAuxToQueue). */
/* Not held to 8 waves per SIMD: claiming eight split-row entries per lane at
   a time needs more registers than that allows, and measured faster at 7. */
__global__ void __launch_bounds__(kBlock) k_aux(GView g, WView w, KParams kp) {
  Ctl* c = w.ctl;
  if (c->done) return;
  const int aux = c->aux;
  if (aux == kAuxNone) return;
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int32_t L = c->level;

  if (aux == kAuxHuge) {
    Acc a = {0, 0, 0, 0};
    const unsigned long long pack = c->huge_pack;
    const int64_t nent = (int64_t)(pack >> 32);
    const int64_t nchunks = (int64_t)(pack & 0xFFFFFFFFull);
    uint64_t* f_nxt = (L & 1) ? w.fr0 : w.fr1;
    /* each wavefront takes a contiguous range of chunks: one search for
       the first chunk's entry, then a forward walk */
    const int64_t per = (nchunks + nwaves - 1) / nwaves;
    const int64_t c0 = min(nchunks, wave * per), c1 = min(nchunks, c0 + per);
    int64_t lo = 0;
    if (c0 < c1) {
      int64_t hi = nent - 1;  /* last entry with base <= c0 */
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)w.huge_base[mid] <= c0) lo = mid; else hi = mid - 1;
      }
    }
    for (int64_t ch = c0; ch < c1; ++ch) {
      while (lo + 1 < nent && (int64_t)w.huge_base[lo + 1] <= ch) ++lo;
      const int32_t u = w.huge_u[lo];
      const int32_t uc = g.new2old ? g.new2old[u] : -1;
      int32_t* q_app = c->q_append ? ((L & 1) ? w.qd0 : w.qd1) : nullptr;
      const int64_t rb = g.off[u], re = g.off[u + 1];
      const int64_t beg = rb + (ch - (int64_t)w.huge_base[lo]) * kHugeChunk;
      const int64_t end = min(re, beg + (int64_t)kHugeChunk);
      /* A lane's entries of the chunk go through each step J at a time
         (neighbour IDs, visited words, claims, then the winners' labels
         and degrees), so a lane has J independent accesses in flight per
         step instead of walking dependent chains one after another.  Lanes
         without an entry use index 0 (in bounds) and are masked. */
      constexpr int J = kHugeBatch;
      for (int64_t k0 = beg + lane; k0 < end; k0 += (int64_t)J * kWave) {
        int32_t v[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const int64_t k = k0 + (int64_t)j * kWave;
          v[j] = g.idx[k < end ? k : beg];
          if (k >= end) v[j] = -1;
        }
        claim_batch<J>(g, w, f_nxt, q_app, v, u, uc, L, a);
      }
    }
    if (finish_block(c, a)) {
      c->aux = kAuxNone;
      decide(g, w, kp);
    }
    return;
  }

  /* kAuxToQueue: level L runs top-down.  Each workgroup owns a contiguous
     range of frontier words: it counts their bits, reserves its queue slice
     with one atomic, then writes the vertices; the other bitmap buffer
     (read by level L-1 or already clear) is zeroed for level L to fill. */
  const uint64_t* f_cur = (L & 1) ? w.fr1 : w.fr0;
  uint64_t* f_old = (L & 1) ? w.fr0 : w.fr1;
  int32_t* q = w.q0;
  const int64_t W = g.words_active;
  const int64_t per = (W + gridDim.x - 1) / gridDim.x;
  const int64_t w0 = min(W, (int64_t)blockIdx.x * per), w1 = min(W, w0 + per);
  int64_t cnt = 0;
  for (int64_t wd = w0 + threadIdx.x; wd < w1; wd += blockDim.x) {
    cnt += __popcll(f_cur[wd]);
    f_old[wd] = 0ull;
  }
  int64_t blk_total = 0;
  (void)block_excl_scan(cnt, &blk_total);
  __shared__ int64_t s_base;
  if (threadIdx.x == 0)
    s_base = blk_total ? (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(&c->q_fill),
                                            (unsigned long long)blk_total)
                       : 0;
  __syncthreads();
  int64_t run = s_base;
  if (blk_total) {
    for (int64_t b = w0; b < w1; b += blockDim.x) {
      const int64_t wd = b + threadIdx.x;
      uint64_t word = wd < w1 ? f_cur[wd] : 0ull;
      int64_t chunk_total = 0;
      int64_t pos = run + block_excl_scan(__popcll(word), &chunk_total);
      while (word) {
        const int bit = __ffsll((unsigned long long)word) - 1;
        word &= word - 1;
        q[pos++] = (int32_t)(wd * kWave + bit);
      }
      run += chunk_total;
    }
  }
  const Acc none = {0, 0, 0, 0};
  if (finish_block(c, none)) c->aux = kAuxNone;
}

__global__ void __launch_bounds__(kBlock) k_init_fill(GView g, WView w) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  if (!w.packed) {  /* relabelled graphs: the finalize kernel reads the visited bitmap instead */
    for (int64_t i = tid; i < g.n; i += nth) {
      w.depth[i] = -1;
      w.parent[i] = -1;
    }
  }
  for (int64_t i = tid; i < g.words; i += nth) {
    w.vis[i] = g.iso[i];
    w.fr0[i] = 0ull;
    w.fr1[i] = 0ull;
  }
}

/* Seeds the traversal from one or more roots (caller IDs): roots[i] for
   i < nroots, or root0 when roots is NULL.  A root given twice is seeded
   once.  One workgroup. */
__global__ void __launch_bounds__(kBlock) k_init_roots(GView g, WView w, const int32_t* roots, int32_t nroots,
                                                     int32_t root0, int32_t first_dir) {
  __shared__ int32_t s_cnt;
  __shared__ int64_t s_deg[kBlock / kWave];
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  int64_t dsum = 0;
  for (int32_t i = threadIdx.x; i < nroots; i += blockDim.x) {
    const int32_t rc = roots ? roots[i] : root0;
    const int32_t v = g.old2new ? g.old2new[rc] : rc;
    const unsigned long long bit = 1ull << (v & 63);
    if (atomicOr(reinterpret_cast<unsigned long long*>(w.fr0 + (v >> 6)), bit) & bit) continue;
    atomicOr(reinterpret_cast<unsigned long long*>(w.vis + (v >> 6)), bit);
    store_labels(w, v, 0, v);
    w.q0[atomicAdd(&s_cnt, 1)] = v;
    dsum += g.off[v + 1] - g.off[v];
  }
  dsum = wave_sum(dsum);
  if (lane_id() == 0) s_deg[threadIdx.x / kWave] = dsum;
  reset_groups(w.ctl);
  __syncthreads();
  if (threadIdx.x != 0) return;
  int64_t dr = 0;
  for (int j = 0; j < kBlock / kWave; ++j) dr += s_deg[j];
  Ctl* c = w.ctl;
  c->level = 0;
  c->dir = first_dir;
  c->done = 0;
  c->aux = kAuxNone;
  c->bu_run = 0;
  c->bu_phases = first_dir == kDirBU ? 1 : 0;
  c->levels = 0;
  c->log_len = 0;
  c->n_f = s_cnt;
  c->m_f = dr;
  c->m_u = g.m - dr;
  c->nf_next = 0;
  c->mf_next = 0;
  c->checked = 0;
  c->scanned = 0;
  c->huge_pack = 0ull;
  c->q_fill = 0;
  c->q_direct = 0;
  c->q_append = (first_dir == kDirTD && dr <= (int64_t)kDirectCap) ? 1 : 0;
  c->qd_fill = 0ull;
  c->reached = s_cnt;
  c->reached_deg = dr;
  c->checked_total = 0;
  c->t_begin = wall_clock64();
}

/* Relabelled multi-root runs: every root's own labels (a degree-0 root is
   not covered by the finalize kernel's single-root rule). */
__global__ void k_fix_roots(WView w, const int32_t* roots, int32_t nroots) {
  for (int32_t i = threadIdx.x; i < nroots; i += blockDim.x) {
    const int32_t rc = roots[i];
    w.depth[rc] = 0;
    if (w.parent) w.parent[rc] = rc;
  }
}

/* Relabelled graphs: caller-label outputs from the packed internal words.
   Caller vertex x has internal label v = old2new[x]; v was reached exactly
   when it is the root or its visited bit is set and v < n_nonisolated
   (degree-0 vertices start visited but are never reached).  Parents are
   mapped back through new2old.  Each thread takes kFinUnroll caller IDs a
   workgroup apart and issues each round of loads for all of them before
   using any, so every lane keeps several independent gathers in flight;
   the streamed arrays (old2new, the outputs) bypass the caches' retention. */
constexpr int kFinUnroll = 8;

__global__ void __launch_bounds__(kBlock) k_finalize(GView g, WView w, int32_t root_caller) {
  /* Workgroups are dealt to the kXcds dies round-robin.  Each die sweeps
     its own contiguous eighth of the caller range, so the runs of
     consecutive internal IDs that a range gathers from stay in one die's
     L2 while its workgroups move along them. */
  const int64_t nn = g.n_nonisolated;
  const int xcd = (int)(blockIdx.x % kXcds);
  const int64_t per_xcd = (int64_t)(gridDim.x / kXcds);
  const int64_t local = (int64_t)(blockIdx.x / kXcds);
  const int64_t span = (int64_t)blockDim.x * kFinUnroll;
  const int64_t part = ((g.n + kXcds - 1) / kXcds + span - 1) / span * span;
  const int64_t lo = (int64_t)xcd * part, hi = min(g.n, lo + part);
  for (int64_t base = lo + local * span + threadIdx.x; base < hi; base += per_xcd * span) {
    int32_t v[kFinUnroll];
#pragma unroll
    for (int j = 0; j < kFinUnroll; ++j) {
      const int64_t x = base + (int64_t)j * blockDim.x;
      v[j] = x < hi ? __builtin_nontemporal_load(g.old2new + x) : 0x7FFFFFFF;
    }
    uint64_t word[kFinUnroll], rec[kFinUnroll];
#pragma unroll
    for (int j = 0; j < kFinUnroll; ++j) {
      const bool in = (int64_t)v[j] < nn;
      word[j] = in ? w.vis[v[j] >> 6] : 0ull;
      rec[j] = in ? (uint64_t)w.packed[v[j]] : 0ull;
    }
    int32_t d[kFinUnroll], p[kFinUnroll];
    const bool want_parent = w.parent != nullptr; /* parents are mapped only when asked for */
#pragma unroll
    for (int j = 0; j < kFinUnroll; ++j) {
      const bool hit = (word[j] >> (v[j] & 63)) & 1ull;
      const uint32_t df = (uint32_t)(rec[j] & 0xFFFFFFFFull), pf = (uint32_t)(rec[j] >> 32);
      d[j] = hit ? (int32_t)(df & ~kCallerParent) : -1;
      p[j] = (hit && want_parent) ? ((df & kCallerParent) ? (int32_t)pf : g.new2old[(int32_t)pf]) : -1;
    }
#pragma unroll
    for (int j = 0; j < kFinUnroll; ++j) {
      const int64_t x = base + (int64_t)j * blockDim.x;
      if (x >= hi) continue;
      if (x == root_caller) {
        d[j] = 0;
        p[j] = root_caller;
      }
      __builtin_nontemporal_store(d[j], w.depth + x);
      if (w.parent) __builtin_nontemporal_store(p[j], w.parent + x);
    }
  }
}

}  // namespace

hipError_t level_grid(int* grid) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_level_bu), kBuBlock, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  *grid = cus * per_cu * (kBuBlock / kBlock);  /* in kBlock-thread workgroups */
  return hipSuccess;
}

hipError_t launch_init(const GView& g, const WView& w, const int32_t* roots, int32_t nroots, int64_t root0,
                       int32_t first_dir, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_init_fill, dim3(grid), dim3(kBlock), 0, s, g, w);
  hipLaunchKernelGGL(k_init_roots, dim3(1), dim3(kBlock), 0, s, g, w, roots, nroots, (int32_t)root0, first_dir);
  return hipGetLastError();
}

hipError_t launch_fix_roots(const WView& w, const int32_t* roots, int32_t nroots, hipStream_t s) {
  hipLaunchKernelGGL(k_fix_roots, dim3(1), dim3(kBlock), 0, s, w, roots, nroots);
  return hipGetLastError();
}

hipError_t launch_level_td(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_level_td, dim3(grid), dim3(kBlock), 0, s, g, w, kp);
  return hipGetLastError();
}

hipError_t launch_level_bu(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_level_bu, dim3((grid + kBuBlock / kBlock - 1) / (kBuBlock / kBlock)), dim3(kBuBlock), 0, s,
                     g, w, kp);
  return hipGetLastError();
}

hipError_t launch_level(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s) {
  /* a top-down level that ends by deciding bottom-up lets the next level
     run in the same slot */
  const hipError_t e = launch_level_td(g, w, kp, grid, s);
  if (e != hipSuccess) return e;
  return launch_level_bu(g, w, kp, grid, s);
}

hipError_t launch_finalize(const GView& g, const WView& w, int64_t root, int grid, hipStream_t s) {
  const int64_t blocks = grid < kXcds ? kXcds : grid / kXcds * kXcds; /* whole workgroups per die */
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)blocks), dim3(kBlock), 0, s, g, w, (int32_t)root);
  return hipGetLastError();
}

hipError_t launch_aux(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_aux, dim3(grid), dim3(kBlock), 0, s, g, w, kp);
  return hipGetLastError();
}

}  // namespace dobfs
