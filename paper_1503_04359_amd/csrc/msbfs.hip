/*
 * Batched traversal: up to 64 single-source BFS of one graph at once, bit
 * b of a per-vertex 64-bit mask standing for root slot b (the bit-parallel
 * multi-source BFS idea applied to the same level-synchronous,
 * direction-optimized step of Algorithm 1).
 *
 * Per vertex: visit (slots that reached it), cur[2] (slots for which it is
 * in the current / next frontier) and nxt (accumulator).  Each slot has its
 * own direction in every level (the pull mask):
 *   push (top-down) slots: every vertex v with such slots in cur[v] ORs
 *     them, minus visit[u], into nxt[u] of each neighbour u (atomic OR);
 *   pull (bottom-up) slots: every vertex still missing some of them ORs
 *     cur[u] over its neighbours in adjacency order and stops as soon as
 *     every missing pull slot is covered.
 * Rows longer than one wavefront should take go to a split list, whose
 * 512-edge chunks are spread over the whole grid by the second kernel of
 * the level (push chunks OR into the neighbours' nxt, pull chunks into the
 * vertex's own nxt).  A dense pass then folds nxt into the frontier:
 * new = nxt & ~visit.  Depth of slot b at v = the level at which bit b
 * first appears at v.  Each slot switches direction by the edge rule of
 * single-source runs, on its own (estimated) counts.
 */
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "dobfs_internal.h"

namespace dobfs {
namespace {

constexpr uint32_t kPullEntry = 0x80000000u;  /* split-list entry of a pull vertex */

/* Depth d of vertex v for one slot b.  Outputs are slot-major, so lanes
   holding consecutive vertices write consecutive addresses. */
__device__ __forceinline__ void ms_put(const GView& g, const MsView& m, int64_t v, int b, int32_t d) {
  if (m.session) d -= m.slot_start[b];
  if (m.internal) m.internal[(int64_t)b * g.n_nonisolated + v] = d;
  else if (m.session) m.slot_out[b][v] = d;
  else m.out[(int64_t)b * g.n + v] = d;
}

/* Per-workgroup per-slot accumulators (new vertices, estimated edges). */
struct SlotLds {
  unsigned long long* nf;
  unsigned long long* mf;
};

__device__ __forceinline__ SlotLds slot_lds() {
  __shared__ unsigned long long s_nf[64];
  __shared__ unsigned long long s_mf[64];
  return {s_nf, s_mf};
}

__device__ __forceinline__ void slot_lds_clear() {
  const SlotLds s = slot_lds();
  if (threadIdx.x < 64) {
    s.nf[threadIdx.x] = 0ull;
    s.mf[threadIdx.x] = 0ull;
  }
  __syncthreads();
}

__device__ __forceinline__ void slot_lds_flush(Ctl* c) {
  __syncthreads();
  const SlotLds s = slot_lds();
  if (threadIdx.x < 64 && s.nf[threadIdx.x]) {
    atomicAdd(&c->slot[threadIdx.x].nf_next, s.nf[threadIdx.x]);
    atomicAdd(&c->slot[threadIdx.x].mf_next, s.mf[threadIdx.x]);
  }
}

/* Depth d for every slot in each lane's nw, the whole wavefront at once:
   one store per slot present anywhere in the wavefront, so each store
   covers the wavefront's consecutive vertices; the slot's counters get the
   number of new vertices times their mean degree.  Every lane must call
   it. */
__device__ __forceinline__ void ms_store_wave(const GView& g, const MsView& m, int64_t v, uint64_t nw, int64_t deg,
                                              int32_t d) {
  unsigned long long any = nw;
  for (int o = 32; o > 0; o >>= 1) any |= __shfl_xor(any, o);
  if (!any) return;
  const int lane = lane_id();
  const int nv = __popcll(__ballot(nw != 0ull));
  const int64_t mean = wave_sum(nw ? deg : 0) / nv;
  const SlotLds s = slot_lds();
  while (any) {
    const int b = __ffsll(any) - 1;
    any &= any - 1;
    const bool mine = (nw >> b) & 1ull;
    const unsigned long long who = __ballot(mine);
    if (mine) ms_put(g, m, v, b, d);
    if (lane == 0) {
      const unsigned long long cnt = (unsigned long long)__popcll(who);
      atomicAdd(&s.nf[b], cnt);
      atomicAdd(&s.mf[b], cnt * (unsigned long long)mean);
    }
  }
}

/* Vertices whose row is too long for one wavefront go to the split list:
   one atomic per wavefront reserves consecutive entries and consecutive
   chunk numbers (kHugeChunk edges each), so chunk bases increase with the
   entry index.  Every lane must call it. */
__device__ __forceinline__ void ms_defer(const MsView& m, bool split, int64_t deg, int32_t v, uint32_t kind) {
  const unsigned long long sm = __ballot(split);
  if (!sm) return;
  const int lane = lane_id();
  const int nch = split ? (int)((deg + kHugeChunk - 1) / kHugeChunk) : 0;
  const int incl = wave_incl_scan(nch, lane);
  const int tot = __shfl(incl, kWave - 1);
  unsigned long long old = 0;
  if (lane == 0)
    old = atomicAdd(reinterpret_cast<unsigned long long*>(&m.ctl->huge_pack),
                    ((unsigned long long)__popcll(sm) << 32) | (unsigned long long)tot);
  old = __shfl(old, 0);
  if (split) {
    const uint32_t slot = (uint32_t)(old >> 32) + (uint32_t)__builtin_amdgcn_mbcnt_hi(
        (uint32_t)(sm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)sm, 0));
    m.split_u[slot] = (int32_t)((uint32_t)v | kind);
    m.split_base[slot] = (uint32_t)(old & 0xFFFFFFFFull) + (uint32_t)(incl - nch);
  }
}

__device__ __forceinline__ uint64_t ms_mix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Resets a slot's counters for a new root of degree deg. */
__device__ __forceinline__ void slot_start_counts(Ctl* c, int b, int64_t deg, int64_t m) {
  SlotStat& st = c->slot[b];
  st.nf = 1;
  st.mf = deg;
  st.mu = m - deg;
  st.nf_next = 0ull;
  st.mf_next = 0ull;
}

/* End of a level (thread 0 of the last workgroup): log, totals, the
   slots still alive, and each slot's direction for the next level. */
__device__ void ms_decide(const GView& g, const MsView& m, const KParams& kp) {
  Ctl* c = m.ctl;
  const int32_t L = c->level;
  const int64_t nfn = ld_agent(&c->nf_next);
  const int64_t mfn = ld_agent(&c->mf_next);
  const int64_t chk = ld_agent(&c->checked);
  const int64_t scn = ld_agent(&c->scanned);
  const uint64_t live_now = m.full & c->live;
  const uint64_t pulled = live_now & c->pull_mask;
  const int32_t dir = pulled == 0ull ? kDirTD : (pulled == live_now ? kDirBU : 2);
  if (c->log_len < m.log_cap) {
    dobfs_level_rec r;
    r.level = L;
    r.dir = dir;
    r.n_f = c->n_f;
    r.m_f = c->m_f;
    r.m_u = c->m_u;
    r.scanned = scn;
    r.checked = chk;
    r.found = nfn;
    r.found_deg = mfn;
    r.t_end = wall_clock64();
    r.kernel_ms = 0.f;
    r.reserved = 0;
    m.log[c->log_len] = r;
    c->log_len = c->log_len + 1;
  }
  c->reached += nfn;
  c->reached_deg += mfn;
  c->checked_total += chk;
  const uint64_t live_next = ld_agent(&c->live_next);
  c->live = live_next;
  c->live_next = 0ull;
  unsigned long long pull = c->pull_mask;
  for (int b = 0; b < 64; ++b) {
    SlotStat& st = c->slot[b];
    const int64_t nf = (int64_t)ld_agent(&st.nf_next), mf = (int64_t)ld_agent(&st.mf_next);
    st.nf_next = 0ull;
    st.mf_next = 0ull;
    if (!((m.full >> b) & 1ull)) continue;
    const unsigned long long bit = 1ull << b;
    st.mu -= mf;
    if (kp.policy == DOBFS_POLICY_FORCED_TD) pull &= ~bit;
    else if (kp.policy == DOBFS_POLICY_FORCED_BU) pull |= bit;
    else if (kp.policy != DOBFS_POLICY_RANDOM) {
      if (!(pull & bit)) {
        if (mf * (int64_t)kp.alpha > st.mu) pull |= bit;
      } else if (nf < st.nf && nf * (int64_t)kp.beta < g.n) {
        pull &= ~bit;
      }
    }
    st.nf = nf;
    st.mf = mf;
  }
  if (kp.policy == DOBFS_POLICY_RANDOM) pull = ms_mix(kp.seed ^ ms_mix((uint64_t)L + 1));
  if (nfn == 0) {
    c->done = 1;
    c->levels = L + 1;
  }
  c->pull_mask = pull;
  c->dir = (pull & live_next) == 0ull ? kDirTD : kDirBU;
  c->aux = kAuxNone;
  c->n_f = nfn;
  c->m_f = mfn;
  c->m_u = c->m_u - mfn;
  c->level = L + 1;
  c->nf_next = 0;
  c->mf_next = 0;
  c->checked = 0;
  c->scanned = 0;
}

/* Push slots: all neighbours of every vertex with such slots in its
   frontier mask, rows laid end to end over the lanes in chunks of at most
   kMsTake entries per row and round. */
__device__ void ms_push(const GView& g, const MsView& m, const uint64_t* cur_in, uint64_t pushb, Acc& a) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t wd = wave; wd < g.words_active; wd += nwaves) {
    const int64_t v = wd * kWave + lane;
    const uint64_t cv = v < g.n ? (cur_in[v] & pushb) : 0ull;
    if (__ballot(cv != 0ull) == 0ull) continue;
    int64_t pos = 0, end = 0;
    if (cv) {
      pos = g.off[v];
      end = g.off[v + 1];
    }
    const bool split = end - pos > kMsPushSplit;
    ms_defer(m, split, end - pos, (int32_t)v, 0u);
    if (split) pos = end; /* its chunks run in the aux kernel */
    a.checked += end - pos;
    while (__ballot(pos < end)) {
      const int take = pos < end ? (int)min(end - pos, (int64_t)kMsTake) : 0;
      const int incl = wave_incl_scan(take, lane);
      const int excl = incl - take;
      const int total = __shfl(incl, kWave - 1);
      for (int c0 = 0; c0 < total; c0 += kWave) {
        const int p = c0 + lane;
        const int o = owner_of(incl, p);
        const int64_t e = __shfl(pos, o) + (p - __shfl(excl, o));
        const uint64_t mo = __shfl(cv, o);
        if (p < total) {
          const int32_t u = g.idx[e];
          const uint64_t x = mo & ~m.visit[u];
          if (x) atomicOr(reinterpret_cast<unsigned long long*>(m.nxt + u), (unsigned long long)x);
        }
      }
      pos += take;
    }
  }
}

/* Pull slots: each vertex still missing some of them ORs its neighbours'
   frontier masks until every missing pull slot is covered.  Writes the
   new frontier of every vertex in the active words (pull slots only). */
__device__ void ms_pull(const GView& g, const MsView& m, const uint64_t* cur_in, uint64_t* cur_out, uint64_t pullb,
                        int32_t L, const KParams& kp, Acc& a) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int max_quota = kp.bu_heavy_cut < kWave ? kWave : kp.bu_heavy_cut;
  for (int64_t wd = wave; wd < g.words_active; wd += nwaves) {
    const int64_t v = wd * kWave + lane;
    const uint64_t vis = v < g.n ? m.visit[v] : ~0ull;
    const uint64_t need = pullb & ~vis;
    if (__ballot(need != 0ull) == 0ull) {
      if (v < g.n) cur_out[v] = 0ull;
      continue;
    }
    int64_t pos = 0, end = 0;
    if (need) {
      pos = g.off[v];
      end = g.off[v + 1];
    }
    const int64_t deg = end - pos;
    a.scanned += need ? 1 : 0;
    /* a long row is searched here only up to its first kMsPullProbe
       entries; if slots are still missing then, the rest goes to the split
       list */
    const bool longrow = deg > kMsPullSplit;
    const int64_t full_end = end;
    if (longrow) end = pos + kMsPullProbe;
    uint64_t acc = 0ull;
    if (pos < end) { /* round 0: own first neighbour, from the first-neighbour column */
      acc = cur_in[g.first[v]];
      a.checked += 1;
      ++pos;
    }
    int quota = 2;
    while (__ballot((need & ~acc) != 0ull && pos < end)) {
      const int take = ((need & ~acc) != 0ull && pos < end) ? (int)min(end - pos, (int64_t)quota) : 0;
      const int incl = wave_incl_scan(take, lane);
      const int excl = incl - take;
      const int total = __shfl(incl, kWave - 1);
      for (int c0 = 0; c0 < total; c0 += kWave) {
        const int p = c0 + lane;
        const int o = owner_of(incl, p);
        const int oexcl = __shfl(excl, o);
        const int64_t e = __shfl(pos, o) + (p - oexcl);
        uint64_t x = 0ull;
        if (p < total) x = cur_in[g.idx[e]];
        /* segmented inclusive OR over the owners' slices of this chunk */
        bool f = (lane == 0) || (p == oexcl);
        for (int d = 1; d < kWave; d <<= 1) {
          const uint64_t y = __shfl_up(x, d);
          const bool gf = __shfl_up((int)f, d) != 0;
          if (lane >= d && !f) {
            x |= y;
            f = gf;
          }
        }
        const int sa = max(excl, c0) - c0, sb = min(incl, c0 + kWave) - c0;
        const bool mine = take > 0 && sa < sb;
        const uint64_t slice = __shfl(x, mine ? sb - 1 : lane);
        if (mine) {
          acc |= slice;
          a.checked += sb - sa;
        }
      }
      pos += take;
      if (quota < max_quota) quota <<= 1;
    }
    const bool split = longrow && (need & ~acc) != 0ull;
    ms_defer(m, split, full_end - pos, (int32_t)v, kPullEntry);
    if (split) {
      /* the probe's finds wait in nxt; the fold settles the vertex */
      if (acc & need) atomicOr(reinterpret_cast<unsigned long long*>(m.nxt + v), (unsigned long long)(acc & need));
      acc = 0ull;
    }
    const uint64_t nw = acc & need;
    if (v < g.n) {
      if (nw) m.visit[v] = vis | nw;
      cur_out[v] = nw;
    }
    ms_store_wave(g, m, v, nw, deg, L + 1);
    if (nw) {
      const int cnt = __popcll(nw);
      a.found += cnt;
      a.found_deg += (int64_t)cnt * deg;
      a.bits |= nw;
    }
  }
}

/* First kernel of a level. */
__global__ void __launch_bounds__(kBlock, 8) k_ms_level(GView g, MsView m, KParams kp) {
  Ctl* c = m.ctl;
  if (c->done || c->aux != kAuxNone) return;
  const int32_t L = c->level;
  const uint64_t* cur_in = (L & 1) ? m.cur1 : m.cur0;
  uint64_t* cur_out = (L & 1) ? m.cur0 : m.cur1;
  /* a slot with an empty frontier cannot reach anything new */
  const uint64_t live = m.full & c->live;
  const uint64_t pullb = live & c->pull_mask, pushb = live & ~c->pull_mask;
  slot_lds_clear();
  Acc a = {0, 0, 0, 0};
  if (pushb) ms_push(g, m, cur_in, pushb, a);
  if (pullb) ms_pull(g, m, cur_in, cur_out, pullb, L, kp, a);
  slot_lds_flush(c);
  if (finish_block(c, a)) {
    if (ld_agent(&c->huge_pack) != 0ull) c->aux = kAuxMsSplit;
    else if (pushb) c->aux = kAuxMsUpdate;
    else ms_decide(g, m, kp);
  }
}

/* Fold nxt into the frontier: new = nxt & ~visit for every vertex; the
   pull slots' part of the frontier, already written by the level kernel,
   is kept. */
__device__ void ms_update(const GView& g, const MsView& m, const KParams& kp) {
  Ctl* c = m.ctl;
  const int32_t L = c->level;
  uint64_t* cur_out = (L & 1) ? m.cur0 : m.cur1;
  const bool keep = (m.full & c->live & c->pull_mask) != 0ull;
  slot_lds_clear();
  Acc a = {0, 0, 0, 0};
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int lane = lane_id();
  const int64_t lim = g.words_active * kWave < g.n ? g.words_active * kWave : g.n;
  /* the loop bound is per wavefront, so all lanes reach ms_store_wave */
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; base < lim; base += nth) {
    const int64_t v = base + lane;
    const uint64_t x = v < lim ? m.nxt[v] : 0ull;
    uint64_t nw = 0ull;
    int64_t deg = 0;
    if (x) {
      m.nxt[v] = 0ull;
      const uint64_t vis = m.visit[v];
      nw = x & ~vis;
      if (nw) {
        m.visit[v] = vis | nw;
        deg = g.off[v + 1] - g.off[v];
        const int cnt = __popcll(nw);
        a.found += cnt;
        a.found_deg += (int64_t)cnt * deg;
        a.bits |= nw;
      }
    }
    ms_store_wave(g, m, v, nw, deg, L + 1);
    if (v < lim) cur_out[v] = keep ? (cur_out[v] | nw) : nw;
  }
  slot_lds_flush(c);
  if (finish_block(c, a)) {
    c->huge_pack = 0ull;
    ms_decide(g, m, kp);
  }
}

/* Chunks of split vertices, each wavefront a contiguous range of chunk
   numbers.  Push entry: OR the vertex's push slots into nxt of each
   neighbour.  Pull entry: OR the frontier masks of the chunk's neighbours
   into the vertex's own nxt word, skipping chunks once its missing pull
   slots are all covered. */
__device__ void ms_split(const GView& g, const MsView& m) {
  Ctl* c = m.ctl;
  const int32_t L = c->level;
  const uint64_t* cur_in = (L & 1) ? m.cur1 : m.cur0;
  const uint64_t live = m.full & c->live;
  const uint64_t pullb = live & c->pull_mask, pushb = live & ~c->pull_mask;
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const unsigned long long pack = c->huge_pack;
  const int64_t nent = (int64_t)(pack >> 32);
  const int64_t nchunks = (int64_t)(pack & 0xFFFFFFFFull);
  const int64_t per = (nchunks + nwaves - 1) / nwaves;
  const int64_t c0 = min(nchunks, wave * per), c1 = min(nchunks, c0 + per);
  Acc a = {0, 0, 0, 0};
  int64_t lo = 0;
  if (c0 < c1) {
    int64_t hi = nent - 1; /* last entry whose first chunk is <= c0 */
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if ((int64_t)m.split_base[mid] <= c0) lo = mid; else hi = mid - 1;
    }
  }
  for (int64_t ch = c0; ch < c1; ++ch) {
    while (lo + 1 < nent && (int64_t)m.split_base[lo + 1] <= ch) ++lo;
    const uint32_t ent = (uint32_t)m.split_u[lo];
    const int32_t v = (int32_t)(ent & ~kPullEntry);
    /* pull entries start after the probe */
    const int64_t rb = g.off[v] + ((ent & kPullEntry) ? kMsPullProbe : 0), re = g.off[v + 1];
    const int64_t beg = rb + (ch - (int64_t)m.split_base[lo]) * kHugeChunk;
    const int64_t end = min(re, beg + (int64_t)kHugeChunk);
    if (!(ent & kPullEntry)) {
      const uint64_t cv = cur_in[v] & pushb;
      for (int64_t k = beg + lane; k < end; k += kWave) {
        const int32_t u = g.idx[k];
        const uint64_t x = cv & ~m.visit[u];
        if (x) atomicOr(reinterpret_cast<unsigned long long*>(m.nxt + u), (unsigned long long)x);
        a.checked += 1;
      }
    } else {
      const uint64_t need = pullb & ~m.visit[v];
      if ((need & ~ld_agent(m.nxt + v)) == 0ull) continue;
      unsigned long long acc = 0ull;
      for (int64_t k = beg + lane; k < end; k += kWave) {
        acc |= cur_in[g.idx[k]];
        a.checked += 1;
      }
      for (int o = 32; o > 0; o >>= 1) acc |= __shfl_xor(acc, o);
      acc &= need;
      if (lane == 0 && acc) atomicOr(reinterpret_cast<unsigned long long*>(m.nxt + v), acc);
    }
  }
  if (finish_block(c, a)) {
    c->huge_pack = 0ull;
    c->aux = kAuxMsUpdate;
  }
}

/* Second launch of a level: the split chunks, or the fold. */
__global__ void __launch_bounds__(kBlock) k_ms_aux(GView g, MsView m, KParams kp) {
  Ctl* c = m.ctl;
  if (c->done) return;
  const int aux = c->aux;
  if (aux == kAuxMsSplit) ms_split(g, m);
  else if (aux == kAuxMsUpdate) ms_update(g, m, kp);
}

/* Third launch of a level: the fold after split chunks. */
__global__ void __launch_bounds__(kBlock) k_ms_fin(GView g, MsView m, KParams kp) {
  Ctl* c = m.ctl;
  if (c->done) return;
  if (c->aux == kAuxMsUpdate) ms_update(g, m, kp);
}

__global__ void __launch_bounds__(kBlock) k_ms_init_fill(GView g, MsView m) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = tid; v < g.n; v += nth) {
    m.visit[v] = ((g.iso[v >> 6] >> (v & 63)) & 1ull) ? ~0ull : 0ull;
    m.cur0[v] = 0ull;
    m.cur1[v] = 0ull;
    m.nxt[v] = 0ull;
  }
  /* relabelled graphs: internal depths are only read where the slot's
     visit bit is set, so they need no fill */
  if (m.session || m.internal) return;
  const int64_t cells = g.n * m.k;
  for (int64_t i = tid; i < cells; i += nth) m.out[i] = -1;
}

__device__ void ctl_reset(Ctl* c) {
  c->level = 0;
  c->dir = kDirTD;
  c->done = 0;
  c->aux = kAuxNone;
  c->bu_run = 0;
  c->bu_phases = 0;
  c->levels = 0;
  c->log_len = 0;
  c->n_f = 0;
  c->m_f = 0;
  c->m_u = 0;
  c->nf_next = 0;
  c->mf_next = 0;
  c->checked = 0;
  c->scanned = 0;
  c->huge_pack = 0ull;
  c->q_fill = 0;
  c->reached = 0;
  c->reached_deg = 0;
  c->checked_total = 0;
  c->live_next = 0ull;
  c->live = 0ull;
  c->active_slots = 0;
  c->pull_mask = 0ull;
  c->t_begin = wall_clock64();
}

/* One wavefront, lane b seeds slot b (roots may repeat, hence atomics). */
__global__ void k_ms_init_roots(GView g, MsView m, MsRoots roots, int32_t first_pull) {
  const int b = threadIdx.x;
  Ctl* c = m.ctl;
  int64_t deg = 0;
  if (b < m.k) {
    const int32_t rc = roots.r[b];
    const int32_t v = g.old2new ? g.old2new[rc] : rc;
    const unsigned long long bit = 1ull << b;
    atomicOr(reinterpret_cast<unsigned long long*>(m.visit + v), bit);
    atomicOr(reinterpret_cast<unsigned long long*>(m.cur0 + v), bit);
    if (!m.internal || (int64_t)v < g.n_nonisolated) ms_put(g, m, v, b, 0);
    deg = g.off[v + 1] - g.off[v];
  }
  if (b < 64) slot_start_counts(c, b, deg, g.m);
  reset_groups(c);
  const int64_t deg_sum = wave_sum(deg);
  if (b != 0) return;
  ctl_reset(c);
  c->n_f = m.k;
  c->m_f = deg_sum;
  c->m_u = g.m * (int64_t)m.k - deg_sum;
  c->reached = m.k;
  c->reached_deg = deg_sum;
  c->live = m.full;
  c->active_slots = m.k;
  c->pull_mask = first_pull ? m.full : 0ull;
  c->dir = first_pull ? kDirBU : kDirTD;
}

/* Session admission, part 1: forget slots about to be reused (their bits in
   every mask; degree-0 vertices keep all bits set). */
__global__ void __launch_bounds__(kBlock) k_ms_session_clear(GView g, MsView m, unsigned long long clear) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n; v += nth) {
    m.visit[v] = ((g.iso[v >> 6] >> (v & 63)) & 1ull) ? ~0ull : (m.visit[v] & ~clear);
    m.cur0[v] &= ~clear;
    m.cur1[v] &= ~clear;
    m.nxt[v] &= ~clear;
  }
}

/* Session admission, part 2: new slots join at the current level with their
   root in the current frontier, pushing first (pulling under the forced
   bottom-up policy). */
__global__ void k_ms_session_seed(GView g, MsView m, MsRoots roots, SlotOuts outs, unsigned long long bits,
                                  int32_t first_pull) {
  const int b = threadIdx.x;
  Ctl* c = m.ctl;
  const bool done = c->done != 0;
  const int32_t L = c->level;
  uint64_t* cur_in = (L & 1) ? m.cur1 : m.cur0;
  const bool mine = b < 64 && ((bits >> b) & 1ull);
  int64_t deg = 0;
  if (mine) {
    const int32_t rc = roots.r[b];
    const int32_t v = g.old2new ? g.old2new[rc] : rc;
    const unsigned long long bit = 1ull << b;
    atomicOr(reinterpret_cast<unsigned long long*>(m.visit + v), bit);
    atomicOr(reinterpret_cast<unsigned long long*>(cur_in + v), bit);
    m.slot_out[b] = outs.p[b];
    m.slot_start[b] = L;
    if (m.internal) {
      if ((int64_t)v < g.n_nonisolated) m.internal[(int64_t)b * g.n_nonisolated + v] = 0;
    } else {
      outs.p[b][rc] = 0;
    }
    deg = g.off[v + 1] - g.off[v];
    slot_start_counts(c, b, deg, g.m);
  }
  const int64_t dsum = wave_sum(deg);
  if (b != 0) return;
  if (done) { /* idle: restart the level loop */
    c->done = 0;
    c->aux = kAuxNone;
    c->n_f = 0;
    c->m_f = 0;
  }
  c->n_f += __popcll(bits);
  c->m_f += dsum;
  c->live |= bits;
  c->pull_mask = first_pull ? (c->pull_mask | bits) : (c->pull_mask & ~bits);
  c->active_slots = __popcll(m.full);
}

__global__ void k_ms_session_ctl(MsView m) {
  reset_groups(m.ctl);
  if (threadIdx.x != 0) return;
  Ctl* c = m.ctl;
  ctl_reset(c);
  c->done = 1;
  for (int b = 0; b < 64; ++b) slot_start_counts(c, b, 0, 0);
}

/* Session, relabelled graphs: each ended slot b gets
   outs.p[b][x] = internal[b][old2new[x]] where it reached the vertex, else
   -1 (its root: 0).  Ended slots keep their visit bits until reused. */
__global__ void __launch_bounds__(kBlock) k_ms_session_finalize(GView g, MsView m, MsRoots roots, SlotOuts outs,
                                                               unsigned long long ended) {
  constexpr int kPer = 8;
  const int64_t span = (int64_t)kBlock * kPer;
  const int64_t nn = g.n_nonisolated;
  for (int64_t x0 = (int64_t)blockIdx.x * span; x0 < g.n; x0 += (int64_t)gridDim.x * span) {
    int32_t v[kPer];
    uint64_t vis[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int64_t x = x0 + (int64_t)j * kBlock + threadIdx.x;
      v[j] = x < g.n ? __builtin_nontemporal_load(g.old2new + x) : -1;
      vis[j] = (v[j] >= 0 && (int64_t)v[j] < nn) ? m.visit[v[j]] : 0ull;
    }
    for (unsigned long long left = ended; left; left &= left - 1) {
      const int b = __ffsll(left) - 1;
      const int32_t rb = roots.r[b];
      int32_t* ob = outs.p[b];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int64_t x = x0 + (int64_t)j * kBlock + threadIdx.x;
        if (x >= g.n) continue;
        int32_t d;
        if ((int64_t)v[j] < nn) d = ((vis[j] >> b) & 1ull) ? m.internal[(int64_t)b * nn + v[j]] : -1;
        else d = (rb == (int32_t)x) ? 0 : -1;
        __builtin_nontemporal_store(d, ob + x);
      }
    }
  }
}

/* Relabelled graphs: out[b][x] = internal[b][old2new[x]] where slot b
   reached the vertex, else -1; degree-0 vertices are unreached except as
   their own slot's root.  A workgroup takes kFinPer * kBlock consecutive
   caller IDs and writes them slot by slot: within a degree class internal
   IDs follow caller order, so each slot's reads for the range are a few
   runs of consecutive IDs, while the writes stay coalesced. */
constexpr int kFinPer = 16;

__global__ void __launch_bounds__(kBlock) k_ms_finalize(GView g, MsView m, MsRoots roots) {
  const int64_t span = (int64_t)kBlock * kFinPer;
  const int64_t nn = g.n_nonisolated;
  for (int64_t x0 = (int64_t)blockIdx.x * span; x0 < g.n; x0 += (int64_t)gridDim.x * span) {
    int32_t v[kFinPer];
    uint64_t vis[kFinPer];
#pragma unroll
    for (int j = 0; j < kFinPer; ++j) {
      const int64_t x = x0 + (int64_t)j * kBlock + threadIdx.x;
      v[j] = x < g.n ? __builtin_nontemporal_load(g.old2new + x) : -1;
      vis[j] = (v[j] >= 0 && (int64_t)v[j] < nn) ? m.visit[v[j]] : 0ull;
    }
    for (int b = 0; b < m.k; ++b) {
      const int32_t rb = roots.r[b];
#pragma unroll
      for (int j = 0; j < kFinPer; ++j) {
        const int64_t x = x0 + (int64_t)j * kBlock + threadIdx.x;
        if (x >= g.n) continue;
        int32_t d;
        if ((int64_t)v[j] < nn) d = ((vis[j] >> b) & 1ull) ? m.internal[(int64_t)b * nn + v[j]] : -1;
        else d = (rb == (int32_t)x) ? 0 : -1;
        __builtin_nontemporal_store(d, m.out + (int64_t)b * g.n + x);
      }
    }
  }
}

}  // namespace

hipError_t launch_ms_init(const GView& g, const MsView& m, const MsRoots& r, int first_pull, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_init_fill, dim3(grid), dim3(kBlock), 0, s, g, m);
  hipLaunchKernelGGL(k_ms_init_roots, dim3(1), dim3(kWave), 0, s, g, m, r, first_pull);
  return hipGetLastError();
}

hipError_t launch_ms_level(const GView& g, const MsView& m, const KParams& kp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_level, dim3(grid), dim3(kBlock), 0, s, g, m, kp);
  hipLaunchKernelGGL(k_ms_aux, dim3(grid), dim3(kBlock), 0, s, g, m, kp);
  hipLaunchKernelGGL(k_ms_fin, dim3(grid), dim3(kBlock), 0, s, g, m, kp);
  return hipGetLastError();
}

hipError_t launch_ms_session_start(const GView& g, const MsView& m, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_init_fill, dim3(grid), dim3(kBlock), 0, s, g, m);
  hipLaunchKernelGGL(k_ms_session_ctl, dim3(1), dim3(kWave), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_ms_session_admit(const GView& g, const MsView& m, unsigned long long clear_bits, const MsRoots& r,
                                   const SlotOuts& outs, unsigned long long new_bits, int first_pull, int grid,
                                   hipStream_t s) {
  if (clear_bits) hipLaunchKernelGGL(k_ms_session_clear, dim3(grid), dim3(kBlock), 0, s, g, m, clear_bits);
  hipLaunchKernelGGL(k_ms_session_seed, dim3(1), dim3(kWave), 0, s, g, m, r, outs, new_bits, first_pull);
  return hipGetLastError();
}

hipError_t launch_ms_session_finalize(const GView& g, const MsView& m, const MsRoots& r, const SlotOuts& outs,
                                      unsigned long long ended, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_session_finalize, dim3(grid), dim3(kBlock), 0, s, g, m, r, outs, ended);
  return hipGetLastError();
}

hipError_t launch_ms_finalize(const GView& g, const MsView& m, const MsRoots& r, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_finalize, dim3(grid), dim3(kBlock), 0, s, g, m, r);
  return hipGetLastError();
}

}  // namespace dobfs
