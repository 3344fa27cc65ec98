/*
 * Batched traversal: up to 64 single-source BFS of one graph at once, bit
 * b of a per-vertex 64-bit mask standing for root slot b (the bit-parallel
 * multi-source BFS idea applied to the same level-synchronous,
 * direction-optimized step of Algorithm 1).
 *
 * Per vertex: visit (slots that reached it), cur[2] (slots for which it is
 * in the current / next frontier) and nxt (push accumulator).
 *   push (top-down) level: every vertex v with cur[v] != 0 ORs
 *     cur[v] & ~visit[u] into nxt[u] of each neighbour u (atomic OR); the
 *     aux kernel then turns nxt into the new frontier: new = nxt & ~visit.
 *   pull (bottom-up) level: every vertex with slots still missing ORs
 *     cur[u] over its neighbours in adjacency order and stops as soon as
 *     every missing slot is covered; new = acc & missing.
 * Depth of slot b at v = the level at which bit b first appears at v.  The
 * same switching rule as single-source runs picks push or pull per level,
 * on popcount-weighted counts.  Pull levels use the bottom-up round
 * machinery: searching vertices contribute doubling quotas of neighbours,
 * laid end to end over the 64 lanes, with a segmented OR across lanes.
 */
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "dobfs_internal.h"

namespace dobfs {
namespace {

__device__ __forceinline__ void ms_store(const GView& g, const MsView& m, int32_t v, uint64_t bits, int32_t d) {
  while (bits) {
    const int b = __ffsll((unsigned long long)bits) - 1;
    bits &= bits - 1;
    if (m.session) m.slot_out[b][g.new2old ? g.new2old[v] : v] = d - m.slot_start[b];
    else if (m.internal) m.internal[(int64_t)v * m.k + b] = d;
    else m.out[(int64_t)b * g.n + v] = d;
  }
}

__device__ void ms_decide(const GView& g, const MsView& m, const KParams& kp) {
  Ctl* c = m.ctl;
  const int32_t L = c->level;
  const int32_t dir = c->dir;
  const int64_t nfn = ld_agent(&c->nf_next);
  const int64_t mfn = ld_agent(&c->mf_next);
  const int64_t chk = ld_agent(&c->checked);
  const int64_t scn = ld_agent(&c->scanned);
  const int64_t mu = c->m_u;
  if (c->log_len < m.log_cap) {
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
    m.log[c->log_len] = r;
    c->log_len = c->log_len + 1;
  }
  c->reached += nfn;
  c->reached_deg += mfn;
  c->checked_total += chk;
  c->live = ld_agent(&c->live_next);
  c->live_next = 0ull;
  const int64_t mu_next = mu - mfn;
  int next = dir;
  if (nfn == 0) {
    c->done = 1;
    c->levels = L + 1;
  } else if (m.session && kp.policy != DOBFS_POLICY_FORCED_TD && kp.policy != DOBFS_POLICY_FORCED_BU) {
    /* slots join and leave, so edge totals are not tracked: compare the
       frontier with the vertices the active slots can still reach */
    const int64_t room = (int64_t)c->active_slots * g.n_nonisolated;
    if (dir == kDirTD) next = (nfn * (int64_t)kp.alpha > room) ? kDirBU : kDirTD;
    else next = (nfn < c->n_f && nfn * (int64_t)kp.beta < room) ? kDirTD : kDirBU;
  } else if (kp.policy == DOBFS_POLICY_FORCED_TD) {
    next = kDirTD;
  } else if (kp.policy == DOBFS_POLICY_FORCED_BU) {
    next = kDirBU;
  } else if (dir == kDirTD) {
    next = (mfn * (int64_t)kp.alpha > mu_next) ? kDirBU : kDirTD;
  } else {
    next = (nfn < c->n_f && nfn * (int64_t)kp.beta < g.n * (int64_t)m.k) ? kDirTD : kDirBU;
  }
  c->aux = kAuxNone;
  c->n_f = nfn;
  c->m_f = mfn;
  c->m_u = mu_next;
  c->dir = next;
  c->level = L + 1;
  c->nf_next = 0;
  c->mf_next = 0;
  c->checked = 0;
  c->scanned = 0;
}

/* Push level: all neighbours of every frontier vertex, rows laid end to end
   over the lanes in chunks of at most kMsTake entries per row and round. */
__device__ void ms_push(const GView& g, const MsView& m, const uint64_t* cur_in, Acc& a) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t wd = wave; wd < g.words_active; wd += nwaves) {
    const int64_t v = wd * kWave + lane;
    const uint64_t cv = v < g.n ? cur_in[v] : 0ull;
    if (__ballot(cv != 0ull) == 0ull) continue;
    int64_t pos = 0, end = 0;
    if (cv) {
      pos = g.off[v];
      end = g.off[v + 1];
    }
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

/* Pull level: each vertex with slots still missing ORs its neighbours'
   frontier masks until every missing slot is covered. */
__device__ void ms_pull(const GView& g, const MsView& m, const uint64_t* cur_in, uint64_t* cur_out, int32_t L,
                        const KParams& kp, Acc& a) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int max_quota = kp.bu_heavy_cut < kWave ? kWave : kp.bu_heavy_cut;
  /* a slot with an empty frontier cannot reach anything new */
  const uint64_t live = m.full & m.ctl->live;
  for (int64_t wd = wave; wd < g.words_active; wd += nwaves) {
    const int64_t v = wd * kWave + lane;
    const uint64_t vis = v < g.n ? m.visit[v] : ~0ull;
    const uint64_t need = live & ~vis;
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
    uint64_t acc = 0ull;
    if (pos < end) { /* round 0: own first neighbour */
      acc = cur_in[g.idx[pos]];
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
    const uint64_t nw = acc & need;
    if (v < g.n) {
      if (nw) m.visit[v] = vis | nw;
      cur_out[v] = nw;
    }
    if (nw) {
      ms_store(g, m, (int32_t)v, nw, L + 1);
      const int cnt = __popcll(nw);
      a.found += cnt;
      a.found_deg += (int64_t)cnt * deg;
      a.bits |= nw;
    }
  }
}

__global__ void __launch_bounds__(kBlock, 8) k_ms_level(GView g, MsView m, KParams kp) {
  Ctl* c = m.ctl;
  if (c->done || c->aux != kAuxNone) return;
  const int32_t L = c->level;
  const int32_t dir = c->dir;
  const uint64_t* cur_in = (L & 1) ? m.cur1 : m.cur0;
  uint64_t* cur_out = (L & 1) ? m.cur0 : m.cur1;
  Acc a = {0, 0, 0, 0};
  if (dir == kDirTD) ms_push(g, m, cur_in, a);
  else ms_pull(g, m, cur_in, cur_out, L, kp, a);
  if (finish_block(c, a)) {
    if (dir == kDirTD) c->aux = kAuxMsUpdate;
    else ms_decide(g, m, kp);
  }
}

/* After a push level: new = nxt & ~visit for every vertex. */
__global__ void __launch_bounds__(kBlock) k_ms_aux(GView g, MsView m, KParams kp) {
  Ctl* c = m.ctl;
  if (c->done || c->aux != kAuxMsUpdate) return;
  const int32_t L = c->level;
  uint64_t* cur_out = (L & 1) ? m.cur0 : m.cur1;
  Acc a = {0, 0, 0, 0};
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int64_t lim = g.words_active * kWave < g.n ? g.words_active * kWave : g.n;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < lim; v += nth) {
    const uint64_t x = m.nxt[v];
    uint64_t nw = 0ull;
    if (x) {
      m.nxt[v] = 0ull;
      const uint64_t vis = m.visit[v];
      nw = x & ~vis;
      if (nw) {
        m.visit[v] = vis | nw;
        ms_store(g, m, (int32_t)v, nw, L + 1);
        const int cnt = __popcll(nw);
        a.found += cnt;
        a.found_deg += (int64_t)cnt * (g.off[v + 1] - g.off[v]);
        a.bits |= nw;
      }
    }
    cur_out[v] = nw;
  }
  if (finish_block(c, a)) ms_decide(g, m, kp);
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
  if (m.session) return;
  if (m.internal) {
    const int64_t cells = g.n_nonisolated * m.k;
    for (int64_t i = tid; i < cells; i += nth) m.internal[i] = -1;
  } else {
    const int64_t cells = g.n * m.k;
    for (int64_t i = tid; i < cells; i += nth) m.out[i] = -1;
  }
}

__global__ void k_ms_init_roots(GView g, MsView m, MsRoots roots) {
  if (threadIdx.x != 0) return;
  int64_t deg_sum = 0;
  for (int b = 0; b < m.k; ++b) {
    const int32_t rc = roots.r[b];
    const int32_t v = g.old2new ? g.old2new[rc] : rc;
    const uint64_t bit = 1ull << b;
    m.visit[v] |= bit;
    m.cur0[v] |= bit;
    if (!m.internal || (int64_t)v < g.n_nonisolated) ms_store(g, m, v, bit, 0);
    deg_sum += g.off[v + 1] - g.off[v];
  }
  Ctl* c = m.ctl;
  c->level = 0;
  c->dir = kDirTD;
  c->done = 0;
  c->aux = kAuxNone;
  c->bu_run = 0;
  c->bu_phases = 0;
  c->levels = 0;
  c->log_len = 0;
  c->n_f = m.k;
  c->m_f = deg_sum;
  c->m_u = g.m * (int64_t)m.k - deg_sum;
  c->nf_next = 0;
  c->mf_next = 0;
  c->checked = 0;
  c->scanned = 0;
  c->huge_pack = 0ull;
  c->q_fill = 0;
  c->reached = m.k;
  c->reached_deg = deg_sum;
  c->checked_total = 0;
  c->live_next = 0ull;
  c->live = m.full;
  c->active_slots = m.k;
  c->t_begin = wall_clock64();
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
   root in the current frontier. */
__global__ void k_ms_session_seed(GView g, MsView m, MsRoots roots, SlotOuts outs, unsigned long long bits) {
  if (threadIdx.x != 0) return;
  Ctl* c = m.ctl;
  if (c->done) { /* idle: restart the level loop */
    c->done = 0;
    c->dir = kDirTD;
    c->aux = kAuxNone;
    c->n_f = 0;
    c->m_f = 0;
  }
  const int32_t L = c->level;
  uint64_t* cur_in = (L & 1) ? m.cur1 : m.cur0;
  int64_t nb = 0, dsum = 0;
  unsigned long long left = bits;
  while (left) {
    const int b = __ffsll((unsigned long long)left) - 1;
    left &= left - 1;
    const int32_t rc = roots.r[b];
    const int32_t v = g.old2new ? g.old2new[rc] : rc;
    const uint64_t bit = 1ull << b;
    m.visit[v] |= bit;
    cur_in[v] |= bit;
    m.slot_out[b] = outs.p[b];
    m.slot_start[b] = L;
    outs.p[b][rc] = 0;
    ++nb;
    dsum += g.off[v + 1] - g.off[v];
  }
  c->n_f += nb;
  c->m_f += dsum;
  c->live |= bits;
  c->active_slots = __popcll(m.full);
}

__global__ void k_ms_session_ctl(MsView m) {
  if (threadIdx.x != 0) return;
  Ctl* c = m.ctl;
  c->level = 0;
  c->dir = kDirTD;
  c->done = 1;
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
  c->t_begin = wall_clock64();
}

/* Relabelled graphs: out[b][x] = internal[old2new[x]][b]; degree-0
   vertices are unreached except as their own slot's root. */
__global__ void __launch_bounds__(kBlock) k_ms_finalize(GView g, MsView m, MsRoots roots) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < g.n; x += nth) {
    const int32_t v = g.old2new[x];
    if ((int64_t)v < g.n_nonisolated) {
      const int32_t* row = m.internal + (int64_t)v * m.k;
      for (int b = 0; b < m.k; ++b) m.out[(int64_t)b * g.n + x] = row[b];
    } else {
      for (int b = 0; b < m.k; ++b) m.out[(int64_t)b * g.n + x] = (roots.r[b] == (int32_t)x) ? 0 : -1;
    }
  }
}

}  // namespace

hipError_t launch_ms_init(const GView& g, const MsView& m, const MsRoots& r, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_init_fill, dim3(grid), dim3(kBlock), 0, s, g, m);
  hipLaunchKernelGGL(k_ms_init_roots, dim3(1), dim3(kWave), 0, s, g, m, r);
  return hipGetLastError();
}

hipError_t launch_ms_level(const GView& g, const MsView& m, const KParams& kp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_level, dim3(grid), dim3(kBlock), 0, s, g, m, kp);
  hipLaunchKernelGGL(k_ms_aux, dim3(grid), dim3(kBlock), 0, s, g, m, kp);
  return hipGetLastError();
}

hipError_t launch_ms_session_start(const GView& g, const MsView& m, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_init_fill, dim3(grid), dim3(kBlock), 0, s, g, m);
  hipLaunchKernelGGL(k_ms_session_ctl, dim3(1), dim3(kWave), 0, s, m);
  return hipGetLastError();
}

hipError_t launch_ms_session_admit(const GView& g, const MsView& m, unsigned long long clear_bits, const MsRoots& r,
                                   const SlotOuts& outs, unsigned long long new_bits, int grid, hipStream_t s) {
  if (clear_bits) hipLaunchKernelGGL(k_ms_session_clear, dim3(grid), dim3(kBlock), 0, s, g, m, clear_bits);
  hipLaunchKernelGGL(k_ms_session_seed, dim3(1), dim3(kWave), 0, s, g, m, r, outs, new_bits);
  return hipGetLastError();
}

hipError_t launch_ms_finalize(const GView& g, const MsView& m, const MsRoots& r, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_ms_finalize, dim3(grid), dim3(kBlock), 0, s, g, m, r);
  return hipGetLastError();
}

}  // namespace dobfs
