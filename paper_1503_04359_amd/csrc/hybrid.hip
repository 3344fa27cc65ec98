/*
 * Hybrid CPU + GPU direction-optimized BFS for graphs larger than the GPU's
 * memory: the paper's specialized partitioning (Section 3.2), level-
 * synchronous processing with per-level frontier exchange (Section 3.1,
 * Algorithms 2 and 3) and deferred parents (Section 3.1).
 *
 * Partitioning.  Vertices are relabelled by degree class, highest first
 * (as for the resident graphs), so the hubs form a prefix of the internal
 * IDs.  The host partition owns the prefix [0, h) with its rows; the GPU
 * partition owns [h, n) with its rows, where h is the smallest multiple of
 * 64 whose GPU share (the rows of [h, n) plus the per-vertex state) fits
 * the caller's device-memory budget.  The many low-degree vertices thus go
 * to the GPU and the few long hub rows stay on the host, the placement the
 * paper gives each kind of processor.
 *
 * A level L in direction d runs on both partitions at once, each on the
 * vertices it owns:
 *   top-down  (Algorithm 2): each partition expands its own frontier
 *             vertices; a neighbour it owns is claimed at once (depth L+1,
 *             the expanding vertex as parent); a neighbour owned by the
 *             other partition is only marked in an outgoing bitmap.  After
 *             both finish, each partition receives the other's bitmap and
 *             claims the marked vertices it has not reached yet, with the
 *             parent left to be found later (deferred);
 *   bottom-up (Algorithm 3): each partition scans its own unvisited
 *             vertices' rows for a neighbour in the level-L frontier; it
 *             reads the whole frontier bitmap, the other partition's part
 *             of which it received at the end of the previous level.
 * After each level the next frontier's two parts are exchanged, so both
 * sides hold the whole frontier of the next level.  The host sums both
 * partitions' counters and applies the switching rule (Section 3.3).
 * Deferred parents are resolved after the traversal: a vertex claimed
 * through the other partition's bitmap takes any neighbour one level
 * closer to the root, found in its own row against the depths of both
 * partitions.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "dobfs_internal.h"
#include "device_common.h"

namespace dobfs {
namespace {

constexpr int32_t kPending = -2;  /* parent found after the traversal */

/* ---- GPU partition ---------------------------------------------------- */

struct HybGpu {
  const int64_t* off;  /* int64[n+1]: rows of [h, n); rows below h are empty */
  const int32_t* idx;
  int64_t n, h;        /* h is a multiple of 64 */
  int64_t w0, w1;      /* the partition's bitmap words [h/64, ceil(n/64)) */
  uint64_t* vis;       /* visited bits of [h, n) (the rest unused) */
  const uint64_t* cur; /* frontier of level L, all n vertices */
  uint64_t* nxt;       /* frontier of level L+1, bits of [h, n) */
  uint64_t* push;      /* top-down: marks for the host partition, bits of [0, h) */
  const uint64_t* pulled; /* top-down: marks from the host partition, bits of [h, n) */
  int32_t* depth;      /* int32[n]: the partition's own entries */
  int32_t* parent;
  unsigned long long* cnt; /* found, found_deg, checked, scanned */
};

__device__ __forceinline__ void hyb_flush(const HybGpu& p, int64_t found, int64_t found_deg, int64_t checked,
                                          int64_t scanned) {
  found = wave_sum(found);
  found_deg = wave_sum(found_deg);
  checked = wave_sum(checked);
  scanned = wave_sum(scanned);
  if (lane_id() == 0) {
    if (found) atomicAdd(&p.cnt[0], (unsigned long long)found);
    if (found_deg) atomicAdd(&p.cnt[1], (unsigned long long)found_deg);
    if (checked) atomicAdd(&p.cnt[2], (unsigned long long)checked);
    if (scanned) atomicAdd(&p.cnt[3], (unsigned long long)scanned);
  }
}

/* Top-down level on the GPU partition: a wavefront per 64-vertex word of
   the partition; its frontier vertices are expanded one after another with
   all lanes striding the row. */
__global__ void __launch_bounds__(kBlock) k_hyb_td(HybGpu p, int32_t L) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int64_t found = 0, found_deg = 0, checked = 0;
  for (int64_t wd = p.w0 + wave_index(); wd < p.w1; wd += nwaves) {
    const uint64_t fw = p.cur[wd];
    if (!fw) continue;
    const int64_t u = wd * kWave + lane;
    const bool f = ((fw >> lane) & 1ull) && u < p.n;
    int64_t b = 0, e = 0;
    if (f) {
      b = p.off[u];
      e = p.off[u + 1];
    }
    uint64_t mm = __ballot(f && e > b);
    while (mm) {
      const int src = __ffsll((unsigned long long)mm) - 1;
      mm &= mm - 1;
      const int32_t uu = (int32_t)__shfl(u, src);
      const int64_t bb = __shfl(b, src), ee = __shfl(e, src);
      for (int64_t k = bb + lane; k < ee; k += kWave) {
        const int32_t v = p.idx[k];
        ++checked;
        const unsigned long long bit = 1ull << (v & 63);
        if ((int64_t)v < p.h) {
          /* owned by the host partition: mark it for the host */
          unsigned long long* w = reinterpret_cast<unsigned long long*>(p.push + (v >> 6));
          if (!(*w & bit)) atomicOr(w, bit);
        } else if (try_claim(p.vis, v)) {
          p.depth[v] = L + 1;
          p.parent[v] = uu;
          atomicOr(reinterpret_cast<unsigned long long*>(p.nxt + (v >> 6)), bit);
          ++found;
          found_deg += p.off[v + 1] - p.off[v];
        }
      }
    }
  }
  hyb_flush(p, found, found_deg, checked, 0);
}

/* Bottom-up level on the GPU partition: lane i of a wavefront owns vertex
   64w+i of word w; each unvisited vertex scans its row in order and stops
   at the first neighbour in the level-L frontier (all n vertices). */
__global__ void __launch_bounds__(kBlock) k_hyb_bu(HybGpu p, int32_t L) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int64_t found = 0, found_deg = 0, checked = 0, scanned = 0;
  for (int64_t wd = p.w0 + wave_index(); wd < p.w1; wd += nwaves) {
    const uint64_t vw = p.vis[wd];
    if (vw == ~0ull) {
      if (lane == 0) p.nxt[wd] = 0ull;
      continue;
    }
    const int64_t v = wd * kWave + lane;
    bool got = false;
    int32_t par = -1;
    int64_t b = 0, e = 0;
    if (!((vw >> lane) & 1ull) && v < p.n) {
      b = p.off[v];
      e = p.off[v + 1];
      scanned += e > b ? 1 : 0;
      for (int64_t k = b; k < e; ++k) {
        const int32_t u = p.idx[k];
        ++checked;
        if ((p.cur[u >> 6] >> (u & 63)) & 1ull) {
          got = true;
          par = u;
          break;
        }
      }
    }
    const uint64_t fm = __ballot(got);
    if (got) {
      p.depth[v] = L + 1;
      p.parent[v] = par;
      ++found;
      found_deg += e - b;
    }
    if (lane == 0) {
      p.nxt[wd] = fm;
      if (fm) p.vis[wd] = vw | fm;
    }
  }
  hyb_flush(p, found, found_deg, checked, scanned);
}

/* After a top-down level: the vertices the host partition marked for this
   one are claimed where still unreached, their parents deferred. */
__global__ void __launch_bounds__(kBlock) k_hyb_apply(HybGpu p, int32_t L) {
  const int lane = lane_id();
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  int64_t found = 0, found_deg = 0;
  for (int64_t wd = p.w0 + wave_index(); wd < p.w1; wd += nwaves) {
    const uint64_t pw = p.pulled[wd];
    if (!pw) continue;
    const uint64_t vw = p.vis[wd];
    const uint64_t nw = pw & ~vw;
    if (!nw) continue;
    const int64_t v = wd * kWave + lane;
    if ((nw >> lane) & 1ull) {
      p.depth[v] = L + 1;
      p.parent[v] = kPending;
      ++found;
      found_deg += p.off[v + 1] - p.off[v];
    }
    if (lane == 0) {
      p.vis[wd] = vw | nw;
      p.nxt[wd] |= nw;
    }
  }
  hyb_flush(p, found, found_deg, 0, 0);
}

/* Deferred parents of the GPU partition: the first neighbour in the row
   whose depth (either partition's, in `depth_all`) is one less. */
__global__ void __launch_bounds__(kBlock) k_hyb_resolve(HybGpu p, const int32_t* depth_all) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = p.h + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < p.n; v += nth) {
    if (p.parent[v] != kPending) continue;
    const int32_t want = depth_all[v] - 1;
    int32_t par = kPending;
    for (int64_t k = p.off[v]; k < p.off[v + 1]; ++k) {
      const int32_t u = p.idx[k];
      if (depth_all[u] == want) {
        par = u;
        break;
      }
    }
    p.parent[v] = par;
  }
}

__global__ void __launch_bounds__(kBlock) k_hyb_init(HybGpu p, int64_t root) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int64_t W = (p.n + 63) / 64;
  const bool own_root = root >= p.h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.n; i += nth) {
    const bool is_root = own_root && i == root;
    p.depth[i] = is_root ? 0 : -1;
    p.parent[i] = is_root ? (int32_t)root : -1;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < W; i += nth) {
    /* bits past n, and vertices without a row on the GPU side, start visited */
    uint64_t w = 0ull;
    for (int j = 0; j < 64; ++j) {
      const int64_t v = i * 64 + j;
      if (v >= p.n || v < p.h || p.off[v + 1] == p.off[v]) w |= 1ull << j;
    }
    if (root >= i * 64 && root < i * 64 + 64) w |= 1ull << (root - i * 64);
    p.vis[i] = w;
  }
}

/* ---- host partition -------------------------------------------------- */

inline bool get_bit(const uint64_t* bm, int64_t v) { return (bm[v >> 6] >> (v & 63)) & 1ull; }

inline void or_bit(uint64_t* bm, int64_t v) {
  __atomic_fetch_or(bm + (v >> 6), 1ull << (v & 63), __ATOMIC_RELAXED);
}

/* Runs fn(t) on T threads and joins them. */
template <class Fn>
void parallel(int T, Fn fn) {
  std::vector<std::thread> th;
  th.reserve((size_t)T);
  for (int t = 0; t < T; ++t) th.emplace_back(fn, t);
  for (auto& x : th) x.join();
}

struct Counts {
  int64_t found = 0, found_deg = 0, checked = 0, scanned = 0;
};

}  // namespace
}  // namespace dobfs

using namespace dobfs;

struct dobfs_hybrid_s {
  int64_t n = 0, m = 0, h = 0, nn = 0;  /* h: a multiple of 64, possibly past n */
  int threads = 1;
  int device = 0, grid = 0;
  /* relabelling (host) */
  std::vector<int32_t> new2old, old2new;
  /* host partition: rows of [0, min(h, n)), internal IDs */
  std::vector<int64_t> off_h;
  std::vector<int32_t> idx_h;
  std::vector<int64_t> deg;     /* degree of every internal vertex */
  /* GPU partition */
  int64_t* off_g = nullptr;
  int32_t* idx_g = nullptr;
  int64_t gpu_entries = 0;
  uint64_t *vis_g = nullptr, *cur_g = nullptr, *nxt_g = nullptr, *push_g = nullptr, *pulled_g = nullptr;
  int32_t *depth_g = nullptr, *parent_g = nullptr;
  unsigned long long* cnt_g = nullptr;
  /* pinned host buffers of the per-level exchange: the whole frontier, the
     GPU's marks for the host and the host's marks for the GPU (W words
     each), the GPU's counters of a level and of its apply step */
  uint64_t *cur_x = nullptr, *gmarks_x = nullptr, *hmarks_x = nullptr;
  unsigned long long* cnt_x = nullptr;
  std::mutex mu;
};

namespace {

int hfail(int status, const char* what, hipError_t e = hipSuccess) {
  set_last_error(what, e);
  return status;
}

#define HYB_HIP(call, what)                                       \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) return hfail(DOBFS_EDEVICE, what, e_);  \
  } while (0)

uint32_t class_of(int64_t d) {
  if (d <= 0) return 0u;
  uint32_t bl = 0;
  while (bl < 63 && ((int64_t)1 << bl) <= d) ++bl;
  return bl;
}

void free_gpu(dobfs_hybrid_s* H) {
  for (void* p : {(void*)H->off_g, (void*)H->idx_g, (void*)H->vis_g, (void*)H->cur_g, (void*)H->nxt_g,
                  (void*)H->push_g, (void*)H->pulled_g, (void*)H->depth_g, (void*)H->parent_g, (void*)H->cnt_g})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)H->cur_x, (void*)H->gmarks_x, (void*)H->hmarks_x, (void*)H->cnt_x})
    if (p) (void)hipHostFree(p);
}

HybGpu gpu_view(const dobfs_hybrid_s* H) {
  HybGpu p;
  p.off = H->off_g;
  p.idx = H->idx_g;
  p.n = H->n;
  p.h = H->h;
  p.w0 = H->h / 64;
  p.w1 = (H->n + 63) / 64;
  p.vis = H->vis_g;
  p.cur = H->cur_g;
  p.nxt = H->nxt_g;
  p.push = H->push_g;
  p.pulled = H->pulled_g;
  p.depth = H->depth_g;
  p.parent = H->parent_g;
  p.cnt = H->cnt_g;
  return p;
}

/* Host partition, one level.  Top-down: frontier vertices of [0, h) are
   expanded in tasks of at most kTask row entries (hub rows are long), taken
   from a shared counter; bottom-up: threads take kBuTake 64-vertex words at
   a time, each word owned by one thread. */
constexpr int64_t kTask = 1 << 14;
constexpr int64_t kBuTake = 16;

Counts host_level(dobfs_hybrid_s* H, int dir, int32_t L, const uint64_t* cur, uint64_t* vis, uint64_t* nxt,
                  uint64_t* marks, int32_t* depth, int32_t* parent) {
  const int T = H->threads;
  const int64_t h = H->h, hv = std::min(H->h, H->n);
  const int64_t Wh = h / 64;
  std::vector<Counts> part((size_t)T);
  if (dir == kDirTD) {
    struct Task {
      int32_t u;
      int64_t b, e;
    };
    std::vector<Task> tasks;
    for (int64_t w = 0; w < Wh; ++w)
      for (uint64_t x = cur[w]; x; x &= x - 1) {
        const int64_t u = w * 64 + __builtin_ctzll(x);
        if (u >= hv) break;
        for (int64_t b = H->off_h[(size_t)u]; b < H->off_h[(size_t)u + 1]; b += kTask)
          tasks.push_back({(int32_t)u, b, std::min(b + kTask, H->off_h[(size_t)u + 1])});
      }
    std::atomic<size_t> next{0};
    parallel(T, [&](int t) {
      Counts c;
      for (size_t i = next.fetch_add(1); i < tasks.size(); i = next.fetch_add(1)) {
        const Task tk = tasks[i];
        for (int64_t k = tk.b; k < tk.e; ++k) {
          const int32_t v = H->idx_h[(size_t)k];
          ++c.checked;
          if ((int64_t)v >= h) {  /* owned by the GPU partition: mark it */
            if (!get_bit(marks, v)) or_bit(marks, v);
            continue;
          }
          const uint64_t bit = 1ull << (v & 63);
          if (__atomic_load_n(vis + (v >> 6), __ATOMIC_RELAXED) & bit) continue;
          if (__atomic_fetch_or(vis + (v >> 6), bit, __ATOMIC_RELAXED) & bit) continue;
          depth[v] = L + 1;
          parent[v] = tk.u;
          or_bit(nxt, v);
          ++c.found;
          c.found_deg += H->deg[(size_t)v];
        }
      }
      part[(size_t)t] = c;
    });
  } else {
    std::atomic<int64_t> next{0};
    parallel(T, [&](int t) {
      Counts c;
      for (int64_t w0 = next.fetch_add(kBuTake); w0 < Wh; w0 = next.fetch_add(kBuTake)) {
        for (int64_t w = w0; w < std::min(w0 + kBuTake, Wh); ++w) {
          const uint64_t vw = vis[w];
          uint64_t fm = 0ull;
          for (uint64_t x = ~vw; x; x &= x - 1) {
            const int j = __builtin_ctzll(x);
            const int64_t v = w * 64 + j;
            const int64_t b = H->off_h[(size_t)v], e = H->off_h[(size_t)v + 1];
            if (e > b) ++c.scanned;
            for (int64_t k = b; k < e; ++k) {
              const int32_t u = H->idx_h[(size_t)k];
              ++c.checked;
              if (get_bit(cur, u)) {
                depth[v] = L + 1;
                parent[v] = u;
                fm |= 1ull << j;
                ++c.found;
                c.found_deg += e - b;
                break;
              }
            }
          }
          nxt[w] = fm;
          vis[w] = vw | fm;
        }
      }
      part[(size_t)t] = c;
    });
  }
  Counts total;
  for (const Counts& c : part) {
    total.found += c.found;
    total.found_deg += c.found_deg;
    total.checked += c.checked;
    total.scanned += c.scanned;
  }
  return total;
}

}  // namespace

extern "C" {

int dobfs_hybrid_upload(const int64_t* offsets, const int32_t* indices, int64_t n, int64_t m,
                        int64_t gpu_budget_bytes, int32_t threads, void* stream, dobfs_hybrid_t* out) {
  set_last_error("", hipSuccess);
  if (!out) return hfail(DOBFS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!offsets || (!indices && m > 0)) return hfail(DOBFS_EINVAL, "offsets/indices is NULL");
  if (n < 1 || n > 2147483647LL || m < 0) return hfail(DOBFS_EINVAL, "n must be in [1, 2^31-1], m >= 0");
  if (threads < 1 || threads > 1024) return hfail(DOBFS_EINVAL, "threads must be in [1, 1024]");
  if (offsets[0] != 0 || offsets[n] != m) return hfail(DOBFS_EINVAL, "offsets[0] must be 0 and offsets[n] = m");
  for (int64_t v = 0; v < n; ++v)
    if (offsets[v + 1] < offsets[v]) return hfail(DOBFS_EINVAL, "offsets not monotone");
  for (int64_t k = 0; k < m; ++k)
    if (indices[k] < 0 || indices[k] >= n) return hfail(DOBFS_EINVAL, "neighbour ID out of range");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dobfs_hybrid_s* H = new (std::nothrow) dobfs_hybrid_s();
  if (!H) return hfail(DOBFS_ENOMEM, "hybrid graph");
  H->n = n;
  H->m = m;
  H->threads = threads;
  auto undo = [&](int st) {
    free_gpu(H);
    delete H;
    return st;
  };
  hipError_t e;
  if ((e = hipGetDevice(&H->device)) != hipSuccess) return undo(hfail(DOBFS_EDEVICE, "hipGetDevice", e));
  if ((e = level_grid(&H->grid)) != hipSuccess) return undo(hfail(DOBFS_EDEVICE, "occupancy query", e));

  /* relabel by degree class, highest first, ties by caller ID (a stable
     counting sort over the classes) */
  std::vector<uint32_t> cls((size_t)n);
  uint32_t max_cls = 0;
  for (int64_t v = 0; v < n; ++v) {
    cls[(size_t)v] = class_of(offsets[v + 1] - offsets[v]);
    max_cls = std::max(max_cls, cls[(size_t)v]);
  }
  std::vector<int64_t> start((size_t)max_cls + 2, 0);
  for (int64_t v = 0; v < n; ++v) ++start[(size_t)(max_cls - cls[(size_t)v]) + 1];
  for (size_t c = 1; c < start.size(); ++c) start[c] += start[c - 1];
  H->new2old.resize((size_t)n);
  H->old2new.resize((size_t)n);
  for (int64_t v = 0; v < n; ++v) {
    const int64_t pos = start[(size_t)(max_cls - cls[(size_t)v])]++;
    H->new2old[(size_t)pos] = (int32_t)v;
    H->old2new[(size_t)v] = (int32_t)pos;
  }
  std::vector<int64_t> off_i((size_t)n + 1, 0);
  H->deg.resize((size_t)n);
  for (int64_t v = 0; v < n; ++v) {
    const int32_t o = H->new2old[(size_t)v];
    H->deg[(size_t)v] = offsets[o + 1] - offsets[o];
    off_i[(size_t)v + 1] = off_i[(size_t)v] + H->deg[(size_t)v];
  }
  H->nn = 0;
  while (H->nn < n && H->deg[(size_t)H->nn] > 0) ++H->nn;

  /* split: the smallest multiple of 64 whose GPU share fits the budget */
  const int64_t W = (n + 63) / 64;
  const int64_t fixed = 8 * (n + 1) + 5 * 8 * W + 8 * n + 64;
  if (gpu_budget_bytes < fixed) return undo(hfail(DOBFS_EINVAL, "device-memory budget below the per-vertex state"));
  const int64_t room = (gpu_budget_bytes - fixed) / 4;  /* row entries the GPU can hold */
  int64_t h = 0;
  {
    int64_t lo = 0, hi = n;  /* first v with m - off_i[v] <= room */
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (m - off_i[(size_t)mid] <= room) hi = mid; else lo = mid + 1;
    }
    h = (lo + 63) / 64 * 64;  /* may pass n by less than 64: then the host holds every row */
  }
  H->h = h;
  const int64_t hv = std::min(h, n);

  /* internal rows, sorted by internal ID (highest degree first) */
  std::vector<int32_t> idx_i((size_t)m);
  parallel(threads, [&](int t) {
    const int64_t lo = n * t / threads, hi = n * (t + 1) / threads;
    for (int64_t v = lo; v < hi; ++v) {
      const int32_t o = H->new2old[(size_t)v];
      int32_t* row = idx_i.data() + off_i[(size_t)v];
      const int64_t d = offsets[o + 1] - offsets[o];
      for (int64_t k = 0; k < d; ++k) row[k] = H->old2new[(size_t)indices[offsets[o] + k]];
      std::sort(row, row + d);
    }
  });
  H->off_h.assign(off_i.begin(), off_i.begin() + (hv + 1));
  H->idx_h.assign(idx_i.begin(), idx_i.begin() + off_i[(size_t)hv]);

  /* GPU partition: every vertex's row slot, the rows of [h, n) filled */
  H->gpu_entries = m - off_i[(size_t)hv];
  std::vector<int64_t> off_gh((size_t)n + 1, 0);
  for (int64_t v = hv; v <= n; ++v) off_gh[(size_t)v] = off_i[(size_t)v] - off_i[(size_t)hv];
  if ((e = hipMalloc(&H->off_g, sizeof(int64_t) * (size_t)(n + 1))) != hipSuccess ||
      (e = hipMalloc(&H->idx_g, sizeof(int32_t) * (size_t)std::max<int64_t>(H->gpu_entries, 1))) != hipSuccess ||
      (e = hipMalloc(&H->vis_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->cur_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->nxt_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->push_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->pulled_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->depth_g, sizeof(int32_t) * (size_t)n)) != hipSuccess ||
      (e = hipMalloc(&H->parent_g, sizeof(int32_t) * (size_t)n)) != hipSuccess ||
      (e = hipMalloc(&H->cnt_g, sizeof(unsigned long long) * 4)) != hipSuccess)
    return undo(hfail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "GPU partition allocation", e));
  if ((e = hipHostMalloc(&H->cur_x, sizeof(uint64_t) * (size_t)W, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc(&H->gmarks_x, sizeof(uint64_t) * (size_t)W, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc(&H->hmarks_x, sizeof(uint64_t) * (size_t)W, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc(&H->cnt_x, sizeof(unsigned long long) * 8, hipHostMallocDefault)) != hipSuccess)
    return undo(hfail(DOBFS_ENOMEM, "pinned exchange buffers", e));
  if ((e = hipMemcpyAsync(H->off_g, off_gh.data(), sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (H->gpu_entries > 0 &&
       (e = hipMemcpyAsync(H->idx_g, idx_i.data() + off_i[(size_t)hv], sizeof(int32_t) * (size_t)H->gpu_entries,
                           hipMemcpyHostToDevice, s)) != hipSuccess) ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return undo(hfail(DOBFS_EDEVICE, "GPU partition upload", e));
  *out = H;
  return DOBFS_OK;
}

int dobfs_hybrid_info(dobfs_hybrid_t H, int64_t* split, int64_t* host_entries, int64_t* gpu_entries,
                      int64_t* gpu_bytes) {
  if (!H) return hfail(DOBFS_EINVAL, "graph is NULL");
  const int64_t W = (H->n + 63) / 64;
  if (split) *split = std::min(H->h, H->n);
  if (host_entries) *host_entries = (int64_t)H->idx_h.size();
  if (gpu_entries) *gpu_entries = H->gpu_entries;
  if (gpu_bytes) *gpu_bytes = 8 * (H->n + 1) + 4 * H->gpu_entries + 5 * 8 * W + 8 * H->n + 32;
  return DOBFS_OK;
}

int dobfs_hybrid_run(dobfs_hybrid_t H, int64_t root, int32_t* depth, int32_t* parent, const dobfs_params* p,
                     dobfs_stats* stats, void* stream) {
  set_last_error("", hipSuccess);
  if (!H || !depth) return hfail(DOBFS_EINVAL, "graph or depth is NULL");
  if (root < 0 || root >= H->n) return hfail(DOBFS_ERANGE, "root outside [0, n)");
  dobfs_params prm;
  if (p) prm = *p; else dobfs_default_params(&prm);
  if (prm.policy < DOBFS_POLICY_EDGE || prm.policy > DOBFS_POLICY_COST)
    return hfail(DOBFS_EINVAL, "unknown policy");
  if (prm.policy == DOBFS_POLICY_RANDOM)
    return hfail(DOBFS_ENOTSUP, "the hybrid run takes the EDGE, PAPER, COST and forced policies");
  if (prm.alpha < 1 || prm.beta < 1 || prm.paper_pct < 1 || prm.paper_div < 1 || prm.paper_bu_steps < 1 ||
      prm.kappa_x1000 < 1)
    return hfail(DOBFS_EINVAL, "switching constants must be >= 1");
  if (stats && stats->log_cap > 0 && !stats->log) return hfail(DOBFS_EINVAL, "stats->log is NULL with log_cap > 0");
  std::lock_guard<std::mutex> lk(H->mu);  /* one run of a hybrid graph at a time */
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t n = H->n, h = H->h, hv = std::min(h, n), W = (n + 63) / 64, Wh = h / 64, Wg = W - Wh;
  const int32_t r = H->old2new[(size_t)root];
  uint64_t* cur = H->cur_x;
  uint64_t* gmarks = H->gmarks_x;
  uint64_t* hmarks = H->hmarks_x;
  unsigned long long* cg = H->cnt_x;      /* [0, 4): the level kernel's counters */
  unsigned long long* ca = H->cnt_x + 4;  /* [4, 8): the apply kernel's */
  /* host state, internal IDs; bits of the GPU's vertices, of degree-0
     vertices and past n start visited, so the host never claims them */
  std::vector<uint64_t> vis((size_t)std::max<int64_t>(Wh, 1), 0ull), nxt((size_t)std::max<int64_t>(Wh, 1), 0ull);
  std::vector<int32_t> dep((size_t)n, -1), par((size_t)n, -1);
  for (int64_t v = 0; v < Wh * 64; ++v)
    if (v >= n || H->deg[(size_t)v] == 0) vis[(size_t)(v >> 6)] |= 1ull << (v & 63);
  std::memset(cur, 0, sizeof(uint64_t) * (size_t)W);
  cur[r >> 6] |= 1ull << (r & 63);
  if (r < hv) {
    vis[(size_t)(r >> 6)] |= 1ull << (r & 63);
    dep[(size_t)r] = 0;
    par[(size_t)r] = r;
  }
  HybGpu g = gpu_view(H);
  const int grid = H->grid;
  hipLaunchKernelGGL(k_hyb_init, dim3(grid), dim3(kBlock), 0, s, g, (int64_t)r);
  HYB_HIP(hipGetLastError(), "init launch");
  HYB_HIP(hipMemcpyAsync(H->cur_g, cur, sizeof(uint64_t) * (size_t)W, hipMemcpyHostToDevice, s), "frontier copy");

  int32_t dir = prm.policy == DOBFS_POLICY_FORCED_BU ? kDirBU : kDirTD;
  int64_t n_f = 1, m_f = H->deg[(size_t)r], m_u = H->m - m_f;
  int32_t bu_run = 0, bu_phases = dir == kDirBU ? 1 : 0;
  int64_t reached = 1, reached_deg = m_f, checked_total = 0;
  int32_t levels = 0, log_len = 0;
  for (int32_t L = 0;; ++L) {
    /* both partitions run level L at once: the GPU's kernel is enqueued,
       then the host threads take the host's share */
    HYB_HIP(hipMemsetAsync(H->nxt_g, 0, sizeof(uint64_t) * (size_t)W, s), "level reset");
    HYB_HIP(hipMemsetAsync(H->push_g, 0, sizeof(uint64_t) * (size_t)W, s), "level reset");
    HYB_HIP(hipMemsetAsync(H->cnt_g, 0, sizeof(unsigned long long) * 4, s), "level reset");
    if (dir == kDirTD) hipLaunchKernelGGL(k_hyb_td, dim3(grid), dim3(kBlock), 0, s, g, L);
    else hipLaunchKernelGGL(k_hyb_bu, dim3(grid), dim3(kBlock), 0, s, g, L);
    HYB_HIP(hipGetLastError(), "level launch");
    HYB_HIP(hipMemcpyAsync(cg, H->cnt_g, sizeof(unsigned long long) * 4, hipMemcpyDeviceToHost, s), "counter copy");
    if (dir == kDirTD && Wh > 0)
      HYB_HIP(hipMemcpyAsync(gmarks, H->push_g, sizeof(uint64_t) * (size_t)Wh, hipMemcpyDeviceToHost, s),
              "marks copy");
    std::fill(nxt.begin(), nxt.end(), 0ull);
    if (dir == kDirTD) std::memset(hmarks, 0, sizeof(uint64_t) * (size_t)W);
    Counts ch = host_level(H, dir, L, cur, vis.data(), nxt.data(), hmarks, dep.data(), par.data());
    HYB_HIP(hipStreamSynchronize(s), "level");
    ca[0] = ca[1] = ca[2] = ca[3] = 0ull;
    if (dir == kDirTD) {
      /* the marks each side made for the other (Algorithm 2): the GPU's
         claim host vertices still unreached, the host's go to the GPU */
      if (Wg > 0) {
        HYB_HIP(hipMemcpyAsync(H->pulled_g + Wh, hmarks + Wh, sizeof(uint64_t) * (size_t)Wg, hipMemcpyHostToDevice, s),
                "marks copy");
        HYB_HIP(hipMemsetAsync(H->cnt_g, 0, sizeof(unsigned long long) * 4, s), "apply reset");
        hipLaunchKernelGGL(k_hyb_apply, dim3(grid), dim3(kBlock), 0, s, g, L);
        HYB_HIP(hipGetLastError(), "apply launch");
        HYB_HIP(hipMemcpyAsync(ca, H->cnt_g, sizeof(unsigned long long) * 4, hipMemcpyDeviceToHost, s),
                "counter copy");
      }
      for (int64_t w = 0; w < Wh; ++w) {
        const uint64_t nw = gmarks[w] & ~vis[(size_t)w];
        if (!nw) continue;
        vis[(size_t)w] |= nw;
        nxt[(size_t)w] |= nw;
        for (uint64_t x = nw; x; x &= x - 1) {
          const int64_t v = w * 64 + __builtin_ctzll(x);
          dep[(size_t)v] = L + 1;
          par[(size_t)v] = kPending;
          ++ch.found;
          ch.found_deg += H->deg[(size_t)v];
        }
      }
    }
    /* the next frontier's two parts, so that both sides hold all of it */
    if (Wg > 0)
      HYB_HIP(hipMemcpyAsync(cur + Wh, H->nxt_g + Wh, sizeof(uint64_t) * (size_t)Wg, hipMemcpyDeviceToHost, s),
              "frontier copy");
    HYB_HIP(hipStreamSynchronize(s), "frontier copy");
    std::copy(nxt.begin(), nxt.begin() + Wh, cur);
    HYB_HIP(hipMemcpyAsync(H->cur_g, cur, sizeof(uint64_t) * (size_t)W, hipMemcpyHostToDevice, s), "frontier copy");
    const int64_t nfn = ch.found + (int64_t)(cg[0] + ca[0]);
    const int64_t mfn = ch.found_deg + (int64_t)(cg[1] + ca[1]);
    const int64_t chk = ch.checked + (int64_t)cg[2];
    const int64_t scn = ch.scanned + (int64_t)cg[3];
    if (stats && log_len < stats->log_cap) {
      dobfs_level_rec& rec = stats->log[log_len];
      std::memset(&rec, 0, sizeof(rec));
      rec.level = L;
      rec.dir = dir;
      rec.n_f = n_f;
      rec.m_f = m_f;
      rec.m_u = m_u;
      rec.scanned = scn;
      rec.checked = chk;
      rec.found = nfn;
      rec.found_deg = mfn;
    }
    ++log_len;
    reached += nfn;
    reached_deg += mfn;
    checked_total += chk;
    const int64_t mu_next = m_u - mfn;
    const int32_t run = dir == kDirBU ? bu_run + 1 : 0;
    if (nfn == 0) {
      levels = L + 1;
      break;
    }
    int32_t next = dir;  /* the switching rule (Section 3.3) on both partitions' counts */
    switch (prm.policy) {
      case DOBFS_POLICY_EDGE:
        if (dir == kDirTD) next = (mfn * (int64_t)prm.alpha > mu_next) ? kDirBU : kDirTD;
        else next = (nfn < n_f && nfn * (int64_t)prm.beta < n) ? kDirTD : kDirBU;
        break;
      case DOBFS_POLICY_PAPER:
        if (dir == kDirTD)
          next = (bu_phases == 0 && mfn * (int64_t)prm.paper_pct > (n / prm.paper_div) * 100) ? kDirBU : kDirTD;
        else
          next = (run >= prm.paper_bu_steps) ? kDirTD : kDirBU;
        break;
      case DOBFS_POLICY_COST: {
        const int64_t unvisited = H->nn - reached;
        if (dir == kDirTD) next = (mfn * 1000 > (int64_t)prm.kappa_x1000 * unvisited) ? kDirBU : kDirTD;
        else next = (nfn < n_f && nfn * (int64_t)prm.beta < n) ? kDirTD : kDirBU;
        break;
      }
      case DOBFS_POLICY_FORCED_TD: next = kDirTD; break;
      default: next = kDirBU; break;
    }
    if (dir == kDirTD && next == kDirBU) ++bu_phases;
    bu_run = run;
    n_f = nfn;
    m_f = mfn;
    m_u = mu_next;
    dir = next;
  }
  /* deferred parents: each partition finds them in its own rows against
     both partitions' depths */
  std::vector<int32_t> dg((size_t)n), pg((size_t)n);
  HYB_HIP(hipMemcpyAsync(dg.data(), H->depth_g, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s), "depth copy");
  HYB_HIP(hipStreamSynchronize(s), "depth copy");
  for (int64_t v = hv; v < n; ++v) dep[(size_t)v] = dg[(size_t)v];
  if (hv > 0)
    HYB_HIP(hipMemcpyAsync(H->depth_g, dep.data(), sizeof(int32_t) * (size_t)hv, hipMemcpyHostToDevice, s),
            "depth copy");
  hipLaunchKernelGGL(k_hyb_resolve, dim3(grid), dim3(kBlock), 0, s, g, (const int32_t*)H->depth_g);
  HYB_HIP(hipGetLastError(), "resolve launch");
  HYB_HIP(hipMemcpyAsync(pg.data(), H->parent_g, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s),
          "parent copy");
  parallel(H->threads, [&](int t) {
    const int64_t lo = hv * t / H->threads, hi = hv * (t + 1) / H->threads;
    for (int64_t v = lo; v < hi; ++v) {
      if (par[(size_t)v] != kPending) continue;
      const int32_t want = dep[(size_t)v] - 1;
      for (int64_t k = H->off_h[(size_t)v]; k < H->off_h[(size_t)v + 1]; ++k)
        if (dep[(size_t)H->idx_h[(size_t)k]] == want) {
          par[(size_t)v] = H->idx_h[(size_t)k];
          break;
        }
    }
  });
  HYB_HIP(hipStreamSynchronize(s), "parent copy");
  for (int64_t v = hv; v < n; ++v) par[(size_t)v] = pg[(size_t)v];
  /* caller IDs */
  for (int64_t v = 0; v < n; ++v) {
    const int32_t x = H->new2old[(size_t)v];
    depth[x] = dep[(size_t)v];
    if (parent) parent[x] = par[(size_t)v] >= 0 ? H->new2old[(size_t)par[(size_t)v]] : -1;
  }
  if (stats) {
    stats->levels = levels;
    stats->log_len = std::min(log_len, std::max(stats->log_cap, 0));
    stats->reached = reached;
    stats->m_c = reached_deg / 2;
    stats->checked = checked_total;
    stats->t_begin = 0;
    stats->level_launches = levels;
    stats->level_kernel_ms = stats->td_kernel_ms = stats->bu_kernel_ms = stats->aux_kernel_ms = 0.0;
  }
  return DOBFS_OK;
}

int dobfs_hybrid_free(dobfs_hybrid_t H) {
  if (!H) return DOBFS_OK;
  {
    std::lock_guard<std::mutex> lk(H->mu);
  }
  free_gpu(H);
  delete H;
  return DOBFS_OK;
}

}  // extern "C"
