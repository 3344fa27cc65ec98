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
 *   - bottom-up: one wavefront per 64-vertex visited word; lane i owns
 *     vertex 64w+i.  Fully visited words are skipped wave-uniformly, the new
 *     frontier word is the wave's ballot and visited |= ballot is one plain
 *     store: bottom-up needs no atomics.  Vertices above bu_heavy_cut are
 *     scanned 64 neighbours at a time by the whole wave, stopping at the
 *     first hit.
 *   - top-down: degree-binned (the virtual-warp idea of Section 2.1 on
 *     64-wide wavefronts): a lane per vertex up to td_wave_cut, a wavefront
 *     per vertex up to td_huge_cut, and above that the vertex's edges are
 *     cut into kHugeChunk-edge tasks spread over all wavefronts by the aux
 *     kernel.  Queue appends are aggregated per wavefront (one atomic per
 *     ballot).
 *   - frontier representations: top-down levels read a queue and also set
 *     the next frontier's bitmap bits (so a following bottom-up level can
 *     probe it); a bottom-up level followed by top-down converts its bitmap
 *     into a queue in the aux kernel.  Bitmap buffer F[L%2] holds F_L; a
 *     top-down level clears the words of F_L it reads so F[L%2] is zero when
 *     level L+1 starts writing F_{L+2} into it.
 */
#include <hip/hip_runtime.h>

#include "dobfs_internal.h"

namespace dobfs {
namespace {

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

/* Number of set bits of `m` below the calling lane. */
__device__ __forceinline__ int mask_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ __forceinline__ bool test_bit(const uint64_t* bm, int32_t v) {
  return (bm[v >> 6] >> (v & 63)) & 1ull;
}

/* Single-winner claim of v's visited bit. */
__device__ __forceinline__ bool try_claim(uint64_t* vis, int32_t v) {
  const unsigned long long bit = 1ull << (v & 63);
  unsigned long long* p = reinterpret_cast<unsigned long long*>(vis + (v >> 6));
  if (*p & bit) return false;
  return (atomicOr(p, bit) & bit) == 0ull;
}

struct Acc {
  int64_t found, found_deg, checked, scanned;
};

__device__ __forceinline__ int64_t wave_sum(int64_t x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

/* Per-workgroup reduction of the accumulators, one atomic per counter. */
__device__ void flush_acc(Ctl* ctl, Acc a, bool add_found) {
  __shared__ int64_t part[4][kBlock / kWave];
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  a.found = wave_sum(a.found);
  a.found_deg = wave_sum(a.found_deg);
  a.checked = wave_sum(a.checked);
  a.scanned = wave_sum(a.scanned);
  if (lane == 0) {
    part[0][wv] = a.found;
    part[1][wv] = a.found_deg;
    part[2][wv] = a.checked;
    part[3][wv] = a.scanned;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t s[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < kBlock / kWave; ++j) s[k] += part[k][j];
    if (add_found && s[0]) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->nf_next), (unsigned long long)s[0]);
    if (s[1]) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->mf_next), (unsigned long long)s[1]);
    if (s[2]) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->checked), (unsigned long long)s[2]);
    if (s[3]) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->scanned), (unsigned long long)s[3]);
  }
}

/* Returns true in thread 0 of the last workgroup to pass this point. */
__device__ bool last_block(Ctl* ctl) {
  __shared__ int is_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t t = atomicAdd(&ctl->ticket, 1u);
    is_last = (t == gridDim.x - 1);
    if (is_last) __threadfence();
  }
  __syncthreads();
  return threadIdx.x == 0 && is_last;
}

template <class T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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
  c->ticket = 0;
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
      case DOBFS_POLICY_FORCED_TD: next = kDirTD; break;
      case DOBFS_POLICY_FORCED_BU: next = kDirBU; break;
      default: next = random_dir(kp.seed, L + 1); break;
    }
  }
  if (dir == kDirTD && next == kDirBU) c->bu_phases = c->bu_phases + 1;
  c->aux = (!c->done && dir == kDirBU && next == kDirTD) ? kAuxToQueue : kAuxNone;
  if (dir == kDirTD) c->qsel = c->qsel ^ 1;
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

/* Wave-aggregated append of the claimed vertices; writes their labels and
   next-frontier bits and accumulates their degrees. */
__device__ __forceinline__ void emit(const GView& g, const WView& w, int32_t* q_nxt, uint64_t* f_nxt,
                                     bool won, int32_t v, int32_t u, int32_t L, int lane, Acc& a) {
  const uint64_t m = __ballot(won);
  if (m == 0ull) return;
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader)
    base = atomicAdd(reinterpret_cast<unsigned long long*>(&w.ctl->nf_next), (unsigned long long)__popcll(m));
  base = __shfl(base, leader);
  if (won) {
    q_nxt[base + mask_rank(m)] = v;
    w.depth[v] = L + 1;
    w.parent[v] = u;
    atomicOr(reinterpret_cast<unsigned long long*>(f_nxt + (v >> 6)), 1ull << (v & 63));
    a.found_deg += g.off[v + 1] - g.off[v];
  }
}

__device__ void top_down(const GView& g, const WView& w, const KParams& kp, int32_t L, Acc& a) {
  Ctl* c = w.ctl;
  const int64_t nf = c->n_f;
  const int32_t* q_cur = c->qsel ? w.q1 : w.q0;
  int32_t* q_nxt = c->qsel ? w.q0 : w.q1;
  uint64_t* f_cur = (L & 1) ? w.fr1 : w.fr0;
  uint64_t* f_nxt = (L & 1) ? w.fr0 : w.fr1;
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t wave_cut = kp.td_wave_cut, huge_cut = kp.td_huge_cut;

  for (int64_t base = wave * kWave; base < nf; base += nwaves * kWave) {
    const int64_t i = base + lane;
    const bool valid = i < nf;
    int32_t u = 0;
    int64_t beg = 0, deg = 0;
    if (valid) {
      u = q_cur[i];
      f_cur[u >> 6] = 0ull;  /* F_L is consumed by this level */
      beg = g.off[u];
      deg = g.off[u + 1] - beg;
    }
    a.checked += deg;
    const bool huge = deg > huge_cut;
    const bool med = !huge && deg > wave_cut;

    /* lane per vertex */
    const int64_t sdeg = (valid && !huge && !med) ? deg : 0;
    for (int64_t j = 0;; ++j) {
      const bool act = j < sdeg;
      if (__ballot(act) == 0ull) break;
      int32_t v = 0;
      bool won = false;
      if (act) {
        v = g.idx[beg + j];
        won = try_claim(w.vis, v);
      }
      emit(g, w, q_nxt, f_nxt, won, v, u, L, lane, a);
    }

    /* wavefront per vertex */
    uint64_t mm = __ballot(med);
    while (mm) {
      const int src = __ffsll((unsigned long long)mm) - 1;
      mm &= mm - 1;
      const int32_t uu = __shfl(u, src);
      const int64_t bb = __shfl(beg, src);
      const int64_t dd = __shfl(deg, src);
      for (int64_t k0 = 0; k0 < dd; k0 += kWave) {
        const int64_t k = k0 + lane;
        const bool act = k < dd;
        int32_t v = 0;
        bool won = false;
        if (act) {
          v = g.idx[bb + k];
          won = try_claim(w.vis, v);
        }
        emit(g, w, q_nxt, f_nxt, won, v, uu, L, lane, a);
      }
    }

    /* split vertices: defer to the aux kernel */
    if (huge) {
      const unsigned long long nch = (unsigned long long)((deg + kHugeChunk - 1) / kHugeChunk);
      const unsigned long long old =
          atomicAdd(reinterpret_cast<unsigned long long*>(&c->huge_pack), (1ull << 32) | nch);
      const uint32_t slot = (uint32_t)(old >> 32);
      w.huge_u[slot] = u;
      w.huge_base[slot] = (uint32_t)(old & 0xFFFFFFFFull);
    }
  }
}

__device__ void bottom_up(const GView& g, const WView& w, const KParams& kp, int32_t L, Acc& a) {
  const uint64_t* f_cur = (L & 1) ? w.fr1 : w.fr0;
  uint64_t* f_nxt = (L & 1) ? w.fr0 : w.fr1;
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t heavy_cut = kp.bu_heavy_cut;

  for (int64_t wd = wave; wd < g.words_active; wd += nwaves) {
    const uint64_t vis = w.vis[wd];
    if (vis == ~0ull) {
      if (lane == 0) f_nxt[wd] = 0ull;
      continue;
    }
    const int32_t v = (int32_t)(wd * kWave + lane);
    const bool unv = ((vis >> lane) & 1ull) == 0ull;  /* bits >= n are set */
    int64_t beg = 0, end = 0;
    if (unv) {
      beg = g.off[v];
      end = g.off[v + 1];
    }
    const int64_t deg = end - beg;
    const bool heavy = unv && deg > heavy_cut;
    a.scanned += unv ? 1 : 0;
    bool found = false;
    int32_t par = -1;
    if (unv && !heavy) {
      int64_t e = beg;
      for (; e < end; ++e) {
        const int32_t u = g.idx[e];
        if (test_bit(f_cur, u)) {
          found = true;
          par = u;
          break;
        }
      }
      a.checked += found ? (e - beg + 1) : deg;
    }
    uint64_t hm = __ballot(heavy);
    while (hm) {
      const int src = __ffsll((unsigned long long)hm) - 1;
      hm &= hm - 1;
      const int64_t bb = __shfl(beg, src), ee = __shfl(end, src);
      int32_t hp = -1;
      int64_t pos = ee - bb;
      for (int64_t k0 = bb; k0 < ee; k0 += kWave) {
        const int64_t e = k0 + lane;
        int32_t u = 0;
        bool hit = false;
        if (e < ee) {
          u = g.idx[e];
          hit = test_bit(f_cur, u);
        }
        const uint64_t hmask = __ballot(hit);
        if (hmask) {
          const int first = __ffsll((unsigned long long)hmask) - 1;
          hp = __shfl(u, first);
          pos = k0 - bb + first + 1;
          break;
        }
      }
      if (lane == src) {
        found = hp >= 0;
        par = hp;
        a.checked += pos;
      }
    }
    const uint64_t fm = __ballot(found);
    if (found) {
      w.depth[v] = L + 1;
      w.parent[v] = par;
      a.found_deg += deg;
      a.found += 1;
    }
    if (lane == 0) {
      f_nxt[wd] = fm;
      if (fm) w.vis[wd] = vis | fm;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_level(GView g, WView w, KParams kp) {
  Ctl* c = w.ctl;
  if (c->done || c->aux != kAuxNone) return;
  const int32_t L = c->level;
  const int32_t dir = c->dir;
  Acc a = {0, 0, 0, 0};
  if (dir == kDirTD) top_down(g, w, kp, L, a);
  else bottom_up(g, w, kp, L, a);
  flush_acc(c, a, dir == kDirBU);
  if (last_block(c)) {
    if (dir == kDirTD && ld_agent(&c->huge_pack) != 0ull) {
      c->ticket = 0;
      c->aux = kAuxHuge;
    } else {
      decide(g, w, kp);
    }
  }
}

/* Expands the split top-down vertices (kAuxHuge) or turns the bottom-up
   frontier bitmap into a queue (kAuxToQueue). */
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
    int32_t* q_nxt = c->qsel ? w.q0 : w.q1;
    uint64_t* f_nxt = (L & 1) ? w.fr0 : w.fr1;
    for (int64_t ch = wave; ch < nchunks; ch += nwaves) {
      int64_t lo = 0, hi = nent - 1;  /* last entry with base <= ch */
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)w.huge_base[mid] <= ch) lo = mid; else hi = mid - 1;
      }
      const int32_t u = w.huge_u[lo];
      const int64_t rb = g.off[u], re = g.off[u + 1];
      const int64_t beg = rb + (ch - (int64_t)w.huge_base[lo]) * kHugeChunk;
      const int64_t end = min(re, beg + (int64_t)kHugeChunk);
      for (int64_t k0 = beg; k0 < end; k0 += kWave) {
        const int64_t k = k0 + lane;
        const bool act = k < end;
        int32_t v = 0;
        bool won = false;
        if (act) {
          v = g.idx[k];
          won = try_claim(w.vis, v);
        }
        emit(g, w, q_nxt, f_nxt, won, v, u, L, lane, a);
      }
    }
    flush_acc(c, a, false);
    if (last_block(c)) {
      c->aux = kAuxNone;
      decide(g, w, kp);
    }
    return;
  }

  /* kAuxToQueue: level L is top-down after a bottom-up level. */
  const uint64_t* f_cur = (L & 1) ? w.fr1 : w.fr0;
  uint64_t* f_old = (L & 1) ? w.fr0 : w.fr1;
  int32_t* q = c->qsel ? w.q1 : w.q0;
  for (int64_t b = wave * kWave; b < g.words_active; b += nwaves * kWave) {
    const int64_t wd = b + lane;
    uint64_t word = 0ull;
    if (wd < g.words_active) {
      word = f_cur[wd];
      f_old[wd] = 0ull;
    }
    int64_t cnt = __popcll(word);
    /* inclusive wave prefix sum of counts */
    int64_t incl = cnt;
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    const int64_t total = __shfl(incl, kWave - 1);
    if (total == 0) continue;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long*>(&c->q_fill), (unsigned long long)total);
    base = __shfl(base, 0);
    int64_t pos = (int64_t)base + incl - cnt;
    while (word) {
      const int bit = __ffsll((unsigned long long)word) - 1;
      word &= word - 1;
      q[pos++] = (int32_t)(wd * kWave + bit);
    }
  }
  if (last_block(c)) {
    c->ticket = 0;
    c->aux = kAuxNone;
  }
}

__global__ void __launch_bounds__(kBlock) k_init_fill(GView g, WView w) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < g.n; i += nth) {
    w.depth[i] = -1;
    w.parent[i] = -1;
  }
  for (int64_t i = tid; i < g.words; i += nth) {
    w.vis[i] = g.iso[i];
    w.fr0[i] = 0ull;
    w.fr1[i] = 0ull;
  }
}

__global__ void k_init_root(GView g, WView w, int32_t root, int32_t first_dir) {
  if (threadIdx.x != 0) return;
  const uint64_t bit = 1ull << (root & 63);
  w.vis[root >> 6] |= bit;
  w.fr0[root >> 6] |= bit;
  w.depth[root] = 0;
  w.parent[root] = root;
  w.q0[0] = root;
  const int64_t dr = g.off[root + 1] - g.off[root];
  Ctl* c = w.ctl;
  c->level = 0;
  c->dir = first_dir;
  c->done = 0;
  c->qsel = 0;
  c->aux = kAuxNone;
  c->bu_run = 0;
  c->bu_phases = first_dir == kDirBU ? 1 : 0;
  c->levels = 0;
  c->log_len = 0;
  c->n_f = 1;
  c->m_f = dr;
  c->m_u = g.m - dr;
  c->nf_next = 0;
  c->mf_next = 0;
  c->checked = 0;
  c->scanned = 0;
  c->huge_pack = 0ull;
  c->q_fill = 0;
  c->ticket = 0;
  c->reached = 1;
  c->reached_deg = dr;
  c->checked_total = 0;
  c->t_begin = wall_clock64();
}

}  // namespace

hipError_t level_grid(int* grid) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_level), kBlock, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  *grid = cus * per_cu;
  return hipSuccess;
}

hipError_t launch_init(const GView& g, const WView& w, int64_t root, int32_t first_dir, int grid,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_init_fill, dim3(grid), dim3(kBlock), 0, s, g, w);
  hipLaunchKernelGGL(k_init_root, dim3(1), dim3(kWave), 0, s, g, w, (int32_t)root, first_dir);
  return hipGetLastError();
}

hipError_t launch_level(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_level, dim3(grid), dim3(kBlock), 0, s, g, w, kp);
  return hipGetLastError();
}

hipError_t launch_aux(const GView& g, const WView& w, const KParams& kp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_aux, dim3(grid), dim3(kBlock), 0, s, g, w, kp);
  return hipGetLastError();
}

}  // namespace dobfs
