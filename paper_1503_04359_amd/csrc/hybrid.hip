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
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <memory>
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
  uint64_t* push;      /* top-down: marks for the host partition, bits of [0, h),
                          kept over the levels of a run */
  const uint64_t* pulled; /* top-down: marks from the host partition, bits of [h, n) */
  int32_t* depth;      /* int32[n]: the partition's own entries */
  int32_t* parent;     /* int32[n]: the partition's own entries; entry v < h
                          holds the GPU vertex whose mark first reached v */
  unsigned long long* cnt; /* found, found_deg, checked, scanned; [4]: entries of lng */
  int32_t* lng;        /* top-down: frontier vertices whose rows are longer than
                          kHybLongRow, expanded by the whole grid */
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
   the partition.  A frontier vertex with at most kHybLaneRow neighbours is
   expanded by its own lane; longer rows are taken one after another by the
   whole wavefront, lanes striding the row; rows longer than kHybLongRow
   (hubs, when the device holds them) are listed for k_hyb_td_long. */
constexpr int64_t kHybLaneRow = 16;
constexpr int64_t kHybLongRow = 2048;

__device__ __forceinline__ void hyb_visit(const HybGpu& p, int32_t L, int32_t u, int32_t v, int64_t& found,
                                          int64_t& found_deg) {
  const unsigned long long bit = 1ull << (v & 63);
  if ((int64_t)v < p.h) {
    /* owned by the host partition: mark it for the host.  The first mark of
       v in a run records u, a vertex of depth L, as v's parent should the
       host first reach v through this mark (at level L) */
    unsigned long long* w = reinterpret_cast<unsigned long long*>(p.push + (v >> 6));
    if (!(*w & bit) && !(atomicOr(w, bit) & bit)) p.parent[v] = u;
  } else if (try_claim(p.vis, v)) {
    p.depth[v] = L + 1;
    p.parent[v] = u;
    atomicOr(reinterpret_cast<unsigned long long*>(p.nxt + (v >> 6)), bit);
    ++found;
    found_deg += p.off[v + 1] - p.off[v];
  }
}

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
    if (e - b <= kHybLaneRow) {
      for (int64_t k = b; k < e; ++k) hyb_visit(p, L, (int32_t)u, p.idx[k], found, found_deg);
      checked += e - b;
    } else if (e - b > kHybLongRow) {
      p.lng[atomicAdd(&p.cnt[4], 1ull)] = (int32_t)u;
    }
    uint64_t mm = __ballot(e - b > kHybLaneRow && e - b <= kHybLongRow);
    while (mm) {
      const int src = __ffsll((unsigned long long)mm) - 1;
      mm &= mm - 1;
      const int32_t uu = (int32_t)__shfl(u, src);
      const int64_t bb = __shfl(b, src), ee = __shfl(e, src);
      for (int64_t k = bb + lane; k < ee; k += kWave) {
        hyb_visit(p, L, uu, p.idx[k], found, found_deg);
        ++checked;
      }
    }
  }
  hyb_flush(p, found, found_deg, checked, 0);
}

/* The long rows a top-down level listed, one after another, each striped
   over every thread of the grid. */
__global__ void __launch_bounds__(kBlock) k_hyb_td_long(HybGpu p, int32_t L) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cnt = (int64_t)p.cnt[4];
  int64_t found = 0, found_deg = 0, checked = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    const int32_t u = p.lng[i];
    const int64_t b = p.off[u], e = p.off[u + 1];
    for (int64_t k = b + t; k < e; k += nth) {
      hyb_visit(p, L, u, p.idx[k], found, found_deg);
      ++checked;
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
  /* a wavefront per visited word: bits past n, vertices without a row on
     the GPU side and the root start visited */
  const int lane = lane_id();
  const int64_t nwaves = nth / kWave;
  for (int64_t wd = wave_index(); wd < W; wd += nwaves) {
    const int64_t v = wd * kWave + lane;
    const bool set = v >= p.n || v < p.h || v == root || p.off[v + 1] == p.off[v];
    const uint64_t w = __ballot(set);
    if (lane == 0) {
      p.vis[wd] = w;
      if (wd < p.w0) p.push[wd] = 0ull;
    }
  }
}

/* Parents of the host partition, read in place from its pinned host array:
   a hub first reached through a GPU mark (kPending there) keeps the marking
   GPU vertex that the device recorded in its own parent entry; every other
   hub takes the host's parent. */
__global__ void __launch_bounds__(kBlock) k_hyb_merge(int32_t* parent, const int32_t* par_host, int64_t hv) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < hv; v += nth) {
    const int32_t ph = par_host[v];
    if (ph != kPending) parent[v] = ph;
  }
}

/* Results in caller IDs: entry x takes its internal vertex's depth and the
   caller ID of its parent. */
__global__ void __launch_bounds__(kBlock) k_hyb_out(const int32_t* depth_i, const int32_t* parent_i,
                                                    const int32_t* old2new, const int32_t* new2old, int64_t n,
                                                    int32_t* depth, int32_t* parent) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += nth) {
    const int32_t v = old2new[x];
    depth[x] = depth_i[v];
    if (parent) {
      const int32_t pv = parent_i[v];
      parent[x] = pv >= 0 ? new2old[pv] : -1;
    }
  }
}

/* ---- host partition -------------------------------------------------- */

inline bool get_bit(const uint64_t* bm, int64_t v) { return (bm[v >> 6] >> (v & 63)) & 1ull; }

/* A fixed set of host threads kept for a hybrid graph's lifetime: run(fn)
   calls fn(t) once for every t in [0, size()), the calling thread taking
   t = 0, and returns when all calls have returned.  A level hands the pool
   two or three short jobs, so workers spin on the job counter for up to
   kSpinUs before blocking on a condition variable, and the caller spins on
   the count of unfinished workers.  An exception thrown by fn in any thread
   is caught there and reported to the caller of run() as std::bad_alloc,
   the one kind the jobs can throw, once every call has returned. */
class Pool {
 public:
  static constexpr int64_t kSpinUs = 200;

  explicit Pool(int n) : n_(n) {
    for (int t = 1; t < n; ++t) th_.emplace_back([this, t] { loop(t); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stop_.store(true, std::memory_order_release);
    }
    cv_.notify_all();
    for (auto& x : th_) x.join();
  }
  int size() const { return n_; }
  void run(const std::function<void(int)>& fn) {
    job_ = &fn;
    failed_.store(false, std::memory_order_relaxed);
    left_.store(n_ - 1, std::memory_order_relaxed);
    {
      std::lock_guard<std::mutex> g(mu_);  /* a worker about to block sees the new job */
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    try {
      fn(0);
    } catch (...) {
      failed_.store(true, std::memory_order_relaxed);
    }
    while (left_.load(std::memory_order_acquire) != 0) std::this_thread::yield();
    if (failed_.load(std::memory_order_relaxed)) throw std::bad_alloc();
  }

 private:
  void loop(int t) {
    uint64_t seen = 0;
    for (;;) {
      uint64_t g = gen_.load(std::memory_order_acquire);
      const auto t0 = std::chrono::steady_clock::now();
      for (int i = 0; g == seen && !stop_.load(std::memory_order_acquire); ++i) {
        if ((i & 255) == 255 &&
            std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(kSpinUs)) {
          std::unique_lock<std::mutex> lk(mu_);
          cv_.wait(lk, [&] {
            return stop_.load(std::memory_order_acquire) || gen_.load(std::memory_order_acquire) != seen;
          });
        }
        g = gen_.load(std::memory_order_acquire);
      }
      if (stop_.load(std::memory_order_acquire)) return;
      seen = g;
      try {
        (*job_)(t);
      } catch (...) {
        failed_.store(true, std::memory_order_relaxed);
      }
      left_.fetch_sub(1, std::memory_order_acq_rel);
    }
  }
  int n_;
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_;
  const std::function<void(int)>* job_ = nullptr;
  std::atomic<int> left_{0};
  std::atomic<uint64_t> gen_{0};
  std::atomic<bool> stop_{false};
  std::atomic<bool> failed_{false};
};

struct Counts {
  int64_t found = 0, found_deg = 0, checked = 0, scanned = 0;
  int64_t marks = 0;  /* host top-down: entries pointing at GPU vertices */
};

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace dobfs

using namespace dobfs;

struct dobfs_hybrid_s {
  int64_t n = 0, m = 0, h = 0, hv = 0, nn = 0;  /* h: a multiple of 64, possibly past n; hv = min(h, n) */
  int device = 0, grid = 0;
  std::unique_ptr<Pool> pool;
  /* relabelling (host) */
  std::vector<int32_t> new2old, old2new;
  /* host partition: rows of [0, hv), internal IDs, and its per-run state */
  std::vector<int64_t> off_h;
  std::vector<int32_t> idx_h;
  std::vector<int64_t> deg;      /* degree of every internal vertex */
  std::vector<int32_t> first_h;  /* first neighbour of each vertex of the host's
                                    words (0: none), read densely by bottom-up
                                    levels, where most scans end there */
  std::vector<uint64_t> vis0_h;  /* visited words [0, h/64) at the start of a run */
  std::vector<uint64_t> vis_h, nxt_h;
  /* top-down marks of GPU vertices, bucketed by host thread (first index)
     and by range of 2^bshift bitmap words past h/64 (second index), so that
     each range is merged into the bitmap by one thread without atomics */
  std::vector<std::vector<int32_t>> bk;
  int nb = 1, bshift = 0;
  /* top-down claims of host vertices as (v << 32 | parent) pairs, bucketed
     the same way over the words below h/64; the owner of a range claims
     its vertices, so the claims need no atomics either */
  std::vector<std::vector<uint64_t>> lk;
  int nbl = 1, lshift = 0;
  /* GPU partition */
  int64_t* off_g = nullptr;
  int32_t* idx_g = nullptr;
  int64_t gpu_entries = 0;
  uint64_t *vis_g = nullptr, *cur_g = nullptr, *nxt_g = nullptr, *push_g = nullptr, *pulled_g = nullptr;
  int32_t *depth_g = nullptr, *parent_g = nullptr;
  int32_t *old2new_g = nullptr, *new2old_g = nullptr;
  unsigned long long* cnt_g = nullptr;  /* 5 counters, see HybGpu::cnt */
  int32_t* lng_g = nullptr;             /* capacity: the device's rows longer than kHybLongRow */
  int64_t n_long = 0;
  /* pinned host buffers: the whole frontier, the GPU's marks for the host
     and the host's marks for the GPU (W words each), the GPU's counters of
     a level and of its apply step; the host partition's depths and parents
     (max(hv, 1) each; the parents are also read in place by the device) */
  uint64_t *cur_x = nullptr, *gmarks_x = nullptr, *hmarks_x = nullptr;
  unsigned long long* cnt_x = nullptr;
  int32_t *dep_h = nullptr, *par_h = nullptr;
  const int32_t* par_h_dev = nullptr;  /* par_h as the device addresses it */
  hipEvent_t ev[2] = {nullptr, nullptr};
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

void release(dobfs_hybrid_s* H) {
  for (void* p : {(void*)H->off_g, (void*)H->idx_g, (void*)H->vis_g, (void*)H->cur_g, (void*)H->nxt_g,
                  (void*)H->push_g, (void*)H->pulled_g, (void*)H->depth_g, (void*)H->parent_g, (void*)H->cnt_g,
                  (void*)H->old2new_g, (void*)H->new2old_g, (void*)H->lng_g})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)H->cur_x, (void*)H->gmarks_x, (void*)H->hmarks_x, (void*)H->cnt_x, (void*)H->dep_h,
                  (void*)H->par_h})
    if (p) (void)hipHostFree(p);
  for (hipEvent_t e : H->ev)
    if (e) (void)hipEventDestroy(e);
  delete H;
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
  p.lng = H->lng_g;
  return p;
}

/* Host partition, one level.  Top-down: frontier vertices of [0, hv) are
   expanded in tasks of at most kTask row entries (hub rows are long), taken
   from a shared counter; a neighbour not yet visited goes to the bucket of
   its word range, and then the owner of each range claims the host
   vertices and marks the GPU vertices of its range.  Bottom-up: threads
   take kBuTake 64-vertex words at a time, each word owned by one thread. */
constexpr int64_t kTask = 1 << 14;
constexpr int64_t kBuTake = 16;
constexpr int64_t kRangesPerThread = 8;

Counts host_level(dobfs_hybrid_s* H, int dir, int32_t L, const uint64_t* cur, uint64_t* marks) {
  Pool& pool = *H->pool;
  const int T = pool.size();
  const int64_t h = H->h, hv = H->hv, Wh = h / 64;
  uint64_t* vis = H->vis_h.data();
  uint64_t* nxt = H->nxt_h.data();
  int32_t* depth = H->dep_h;
  int32_t* parent = H->par_h;
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
    const int nb = H->nb, bshift = H->bshift, nbl = H->nbl, lshift = H->lshift;
    pool.run([&](int t) {
      Counts c;
      std::vector<int32_t>* bk = H->bk.data() + (size_t)t * nb;
      std::vector<uint64_t>* lk = H->lk.data() + (size_t)t * nbl;
      for (size_t i = next.fetch_add(1); i < tasks.size(); i = next.fetch_add(1)) {
        const Task tk = tasks[i];
        c.checked += tk.e - tk.b;
        for (int64_t k = tk.b; k < tk.e; ++k) {
          const int32_t v = H->idx_h[(size_t)k];
          if ((int64_t)v >= h) {  /* owned by the GPU partition: to be marked */
            bk[((v >> 6) - Wh) >> bshift].push_back(v);
            ++c.marks;
          } else if (!get_bit(vis, v)) {  /* vis does not change in this phase */
            lk[(v >> 6) >> lshift].push_back(((uint64_t)(uint32_t)v << 32) | (uint32_t)tk.u);
          }
        }
      }
      part[(size_t)t] = c;
    });
    /* owners of the word ranges: each range of either kind is taken by one
       thread, ranges handed out from a shared counter */
    const int64_t W = (H->n + 63) / 64;
    std::vector<Counts> claimed((size_t)T);
    std::atomic<int> next_range{0};
    int64_t n_marks = 0;
    for (const Counts& c : part) n_marks += c.marks;
    pool.run([&](int t) {
      Counts c;
      for (int r = next_range.fetch_add(1); r < nb + nbl; r = next_range.fetch_add(1)) {
        if (r < nb) {
          if (n_marks == 0) continue;  /* the marks bitmap is not sent then */
          const int64_t w_lo = Wh + ((int64_t)r << bshift), w_hi = std::min(W, Wh + ((int64_t)(r + 1) << bshift));
          if (w_lo < w_hi) std::memset(marks + w_lo, 0, sizeof(uint64_t) * (size_t)(w_hi - w_lo));
          for (int src = 0; src < T; ++src) {
            std::vector<int32_t>& b = H->bk[(size_t)src * nb + r];
            for (const int32_t v : b) marks[v >> 6] |= 1ull << (v & 63);
            b.clear();
          }
          continue;
        }
        for (int src = 0; src < T; ++src) {
          std::vector<uint64_t>& b = H->lk[(size_t)src * nbl + (r - nb)];
          for (const uint64_t x : b) {
            const int32_t v = (int32_t)(x >> 32);
            const uint64_t bit = 1ull << (v & 63);
            if (vis[v >> 6] & bit) continue;
            vis[v >> 6] |= bit;
            nxt[v >> 6] |= bit;
            depth[v] = L + 1;
            parent[v] = (int32_t)(uint32_t)x;
            ++c.found;
            c.found_deg += H->deg[(size_t)v];
          }
          b.clear();
        }
      }
      claimed[(size_t)t] = c;
    });
    for (int t = 0; t < T; ++t) {
      part[(size_t)t].found += claimed[(size_t)t].found;
      part[(size_t)t].found_deg += claimed[(size_t)t].found_deg;
    }
  } else {
    const int32_t* first = H->first_h.data();
    std::atomic<int64_t> next{0};
    pool.run([&](int t) {
      Counts c;
      for (int64_t w0 = next.fetch_add(kBuTake); w0 < Wh; w0 = next.fetch_add(kBuTake)) {
        for (int64_t w = w0; w < std::min(w0 + kBuTake, Wh); ++w) {
          const uint64_t vw = vis[w];
          const uint64_t unv = ~vw;
          if (!unv) {
            nxt[w] = 0ull;
            continue;
          }
          /* every vertex of the word tests its first neighbour, without
             branches; the rest of a row is read only on a miss */
          const int32_t* fr = first + w * 64;
          uint64_t hit = 0ull;
          for (int j = 0; j < 64; ++j) {
            const uint32_t u = (uint32_t)fr[j];
            hit |= ((cur[u >> 6] >> (u & 63)) & 1ull) << j;
          }
          hit &= unv;
          const int n_unv = __builtin_popcountll(unv);
          c.scanned += n_unv;
          c.checked += n_unv;
          for (uint64_t x = hit; x; x &= x - 1) {
            const int j = __builtin_ctzll(x);
            const int64_t v = w * 64 + j;
            depth[v] = L + 1;
            parent[v] = fr[j];
            ++c.found;
            c.found_deg += H->off_h[(size_t)v + 1] - H->off_h[(size_t)v];
          }
          uint64_t fm = hit;
          /* the rows still to read start at scattered places: their first
             lines are requested together before any is scanned */
          for (uint64_t x = unv & ~hit; x; x &= x - 1) {
            const int64_t v = w * 64 + __builtin_ctzll(x);
            __builtin_prefetch(H->idx_h.data() + H->off_h[(size_t)v] + 1);
          }
          for (uint64_t x = unv & ~hit; x; x &= x - 1) {
            const int j = __builtin_ctzll(x);
            const int64_t v = w * 64 + j;
            const int64_t b = H->off_h[(size_t)v], e = H->off_h[(size_t)v + 1];
            for (int64_t k = b + 1; k < e; ++k) {
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
    total.marks += c.marks;
  }
  return total;
}

/* [lo, hi) share of thread t of T over [0, n) */
inline void share(int64_t n, int t, int T, int64_t* lo, int64_t* hi) {
  *lo = n * t / T;
  *hi = n * (t + 1) / T;
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
  const int64_t W = (n + 63) / 64;
  const int64_t fixed = 8 * (n + 1) + 5 * 8 * W + 16 * n + 64;
  if (gpu_budget_bytes < fixed) return hfail(DOBFS_EINVAL, "device-memory budget below the per-vertex state");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  dobfs_hybrid_s* H = new (std::nothrow) dobfs_hybrid_s();
  if (!H) return hfail(DOBFS_ENOMEM, "hybrid graph");
  H->n = n;
  H->m = m;
  auto undo = [&](int st) {
    release(H);
    return st;
  };
  try {
    H->pool.reset(new Pool(threads));
  } catch (...) {
    return undo(hfail(DOBFS_ENOMEM, "host threads"));
  }
  Pool& pool = *H->pool;
  {
    std::atomic<bool> bad{false};
    pool.run([&](int t) {
      int64_t lo, hi;
      share(m, t, pool.size(), &lo, &hi);
      for (int64_t k = lo; k < hi; ++k)
        if (indices[k] < 0 || indices[k] >= n) {
          bad = true;
          break;
        }
    });
    if (bad) return undo(hfail(DOBFS_EINVAL, "neighbour ID out of range"));
  }
  hipError_t e;
  if ((e = hipGetDevice(&H->device)) != hipSuccess) return undo(hfail(DOBFS_EDEVICE, "hipGetDevice", e));
  if ((e = level_grid(&H->grid)) != hipSuccess) return undo(hfail(DOBFS_EDEVICE, "occupancy query", e));

  /* relabel by degree class, highest first, ties by caller ID (a stable
     counting sort over the classes) */
  std::vector<int64_t> off_i;
  std::vector<int32_t> idx_i;
  try {
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
    off_i.assign((size_t)n + 1, 0);
    H->deg.resize((size_t)n);
    for (int64_t v = 0; v < n; ++v) {
      const int32_t o = H->new2old[(size_t)v];
      H->deg[(size_t)v] = offsets[o + 1] - offsets[o];
      off_i[(size_t)v + 1] = off_i[(size_t)v] + H->deg[(size_t)v];
    }
    H->nn = 0;
    while (H->nn < n && H->deg[(size_t)H->nn] > 0) ++H->nn;

    /* split: the smallest multiple of 64 whose GPU share fits the budget */
    const int64_t room = (gpu_budget_bytes - fixed) / 4;  /* row entries the GPU can hold */
    int64_t lo = 0, hi = n;  /* first v with m - off_i[v] <= room */
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      if (m - off_i[(size_t)mid] <= room) hi = mid; else lo = mid + 1;
    }
    H->h = (lo + 63) / 64 * 64;  /* may pass n by less than 64: then the host holds every row */
    H->hv = std::min(H->h, n);

    /* internal rows, sorted by internal ID (highest degree first) */
    idx_i.resize((size_t)m);
    std::atomic<int64_t> next{0};
    pool.run([&](int) {
      for (int64_t v0 = next.fetch_add(4096); v0 < n; v0 = next.fetch_add(4096))
        for (int64_t v = v0; v < std::min(v0 + 4096, n); ++v) {
          const int32_t o = H->new2old[(size_t)v];
          int32_t* row = idx_i.data() + off_i[(size_t)v];
          const int64_t d = offsets[o + 1] - offsets[o];
          for (int64_t k = 0; k < d; ++k) row[k] = H->old2new[(size_t)indices[offsets[o] + k]];
          std::sort(row, row + d);
        }
    });
    const int64_t h = H->h, hv = H->hv, Wh = h / 64;
    H->off_h.assign(off_i.begin(), off_i.begin() + (hv + 1));
    H->idx_h.assign(idx_i.begin(), idx_i.begin() + off_i[(size_t)hv]);
    /* every vertex of the host's words has an entry; one without a row
       (never unvisited there) reads vertex 0 */
    H->first_h.assign((size_t)std::max<int64_t>(Wh * 64, 1), 0);
    for (int64_t v = 0; v < hv; ++v)
      if (off_i[(size_t)v + 1] > off_i[(size_t)v]) H->first_h[(size_t)v] = idx_i[(size_t)off_i[(size_t)v]];
    H->vis0_h.assign((size_t)std::max<int64_t>(Wh, 1), 0ull);
    for (int64_t v = 0; v < Wh * 64; ++v)  /* degree-0 vertices and bits past n never take a claim */
      if (v >= n || H->deg[(size_t)v] == 0) H->vis0_h[(size_t)(v >> 6)] |= 1ull << (v & 63);
    H->vis_h.assign(H->vis0_h.size(), 0ull);
    H->nxt_h.assign(H->vis0_h.size(), 0ull);
    const int64_t Wg = W - Wh;
    /* at most kRangesPerThread ranges of each kind per thread */
    const int64_t max_ranges = (int64_t)threads * kRangesPerThread;
    while (H->bshift < 62 && ((Wg + ((int64_t)1 << H->bshift) - 1) >> H->bshift) > max_ranges) ++H->bshift;
    H->nb = (int)std::max<int64_t>(1, (Wg + ((int64_t)1 << H->bshift) - 1) >> H->bshift);
    H->bk.resize((size_t)threads * (size_t)H->nb);
    while (H->lshift < 62 && ((Wh + ((int64_t)1 << H->lshift) - 1) >> H->lshift) > max_ranges) ++H->lshift;
    H->nbl = (int)std::max<int64_t>(1, (Wh + ((int64_t)1 << H->lshift) - 1) >> H->lshift);
    H->lk.resize((size_t)threads * (size_t)H->nbl);
  } catch (const std::bad_alloc&) {
    return undo(hfail(DOBFS_ENOMEM, "host partition"));
  }
  const int64_t hv = H->hv;

  /* GPU partition: every vertex's row slot, the rows of [h, n) filled */
  H->gpu_entries = m - off_i[(size_t)hv];
  int64_t& n_long = H->n_long;
  for (int64_t v = hv; v < n; ++v)
    if (H->deg[(size_t)v] > kHybLongRow) ++n_long;
  for (int64_t v = 0; v <= n; ++v) off_i[(size_t)v] = v < hv ? 0 : off_i[(size_t)v] - H->off_h[(size_t)hv];
  if ((e = hipMalloc(&H->off_g, sizeof(int64_t) * (size_t)(n + 1))) != hipSuccess ||
      (e = hipMalloc(&H->idx_g, sizeof(int32_t) * (size_t)std::max<int64_t>(H->gpu_entries, 1))) != hipSuccess ||
      (e = hipMalloc(&H->vis_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->cur_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->nxt_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->push_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->pulled_g, sizeof(uint64_t) * (size_t)W)) != hipSuccess ||
      (e = hipMalloc(&H->depth_g, sizeof(int32_t) * (size_t)n)) != hipSuccess ||
      (e = hipMalloc(&H->parent_g, sizeof(int32_t) * (size_t)n)) != hipSuccess ||
      (e = hipMalloc(&H->cnt_g, sizeof(unsigned long long) * 5)) != hipSuccess ||
      (e = hipMalloc(&H->lng_g, sizeof(int32_t) * (size_t)std::max<int64_t>(n_long, 1))) != hipSuccess ||
      (e = hipMalloc(&H->old2new_g, sizeof(int32_t) * (size_t)n)) != hipSuccess ||
      (e = hipMalloc(&H->new2old_g, sizeof(int32_t) * (size_t)n)) != hipSuccess)
    return undo(hfail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "GPU partition allocation", e));
  if ((e = hipHostMalloc(&H->cur_x, sizeof(uint64_t) * (size_t)W, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc(&H->gmarks_x, sizeof(uint64_t) * (size_t)W, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc(&H->hmarks_x, sizeof(uint64_t) * (size_t)W, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc(&H->cnt_x, sizeof(unsigned long long) * 8, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc(&H->dep_h, sizeof(int32_t) * (size_t)std::max<int64_t>(hv, 1), hipHostMallocDefault)) !=
          hipSuccess ||
      (e = hipHostMalloc(&H->par_h, sizeof(int32_t) * (size_t)std::max<int64_t>(hv, 1), hipHostMallocMapped)) !=
          hipSuccess)
    return undo(hfail(DOBFS_ENOMEM, "pinned exchange buffers", e));
  {
    void* dp = nullptr;
    if ((e = hipHostGetDevicePointer(&dp, H->par_h, 0)) != hipSuccess)
      return undo(hfail(DOBFS_EDEVICE, "device address of the host parents", e));
    H->par_h_dev = static_cast<const int32_t*>(dp);
  }
  if ((e = hipEventCreate(&H->ev[0])) != hipSuccess || (e = hipEventCreate(&H->ev[1])) != hipSuccess)
    return undo(hfail(DOBFS_EDEVICE, "event creation", e));
  if ((e = hipMemcpyAsync(H->off_g, off_i.data(), sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (H->gpu_entries > 0 &&
       (e = hipMemcpyAsync(H->idx_g, idx_i.data() + H->off_h[(size_t)hv], sizeof(int32_t) * (size_t)H->gpu_entries,
                           hipMemcpyHostToDevice, s)) != hipSuccess) ||
      (e = hipMemcpyAsync(H->old2new_g, H->old2new.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(H->new2old_g, H->new2old.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return undo(hfail(DOBFS_EDEVICE, "GPU partition upload", e));
  *out = H;
  return DOBFS_OK;
}

int dobfs_hybrid_info(dobfs_hybrid_t H, int64_t* split, int64_t* host_entries, int64_t* gpu_entries,
                      int64_t* gpu_bytes) {
  if (!H) return hfail(DOBFS_EINVAL, "graph is NULL");
  const int64_t W = (H->n + 63) / 64;
  if (split) *split = H->hv;
  if (host_entries) *host_entries = (int64_t)H->idx_h.size();
  if (gpu_entries) *gpu_entries = H->gpu_entries;
  if (gpu_bytes)
    *gpu_bytes = 8 * (H->n + 1) + 4 * H->gpu_entries + 5 * 8 * W + 16 * H->n + 40 + 4 * std::max<int64_t>(H->n_long, 1);
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
  const bool hub_decides = (prm.flags & DOBFS_RUN_HUB_DECIDES) != 0u;
  if (hub_decides && prm.policy != DOBFS_POLICY_PAPER)
    return hfail(DOBFS_EINVAL, "DOBFS_RUN_HUB_DECIDES needs the PAPER policy");
  const bool timed = (prm.flags & DOBFS_RUN_TIME_KERNELS) != 0u;
  if (stats && stats->log_cap > 0 && !stats->log) return hfail(DOBFS_EINVAL, "stats->log is NULL with log_cap > 0");
  std::lock_guard<std::mutex> lk(H->mu);  /* one run of a hybrid graph at a time */
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Pool& pool = *H->pool;
  const int T = pool.size();
  const int64_t n = H->n, h = H->h, hv = H->hv, W = (n + 63) / 64, Wh = h / 64, Wg = W - Wh;
  const int32_t r = H->old2new[(size_t)root];
  uint64_t* cur = H->cur_x;
  uint64_t* gmarks = H->gmarks_x;
  uint64_t* hmarks = H->hmarks_x;
  unsigned long long* cg = H->cnt_x;      /* [0, 4): the level kernel's counters */
  unsigned long long* ca = H->cnt_x + 4;  /* [4, 8): the apply kernel's */
  double td_ms = 0.0, bu_ms = 0.0, aux_ms = 0.0;
  auto kernel_ms = [&](double* acc) -> hipError_t {  /* after a synchronize */
    float ms = 0.f;
    const hipError_t e = hipEventElapsedTime(&ms, H->ev[0], H->ev[1]);
    *acc += ms;
    return e;
  };
  /* the device's state is set up while the host threads reset the host's
     (internal IDs); buckets left filled by a failed run are emptied */
  HybGpu g = gpu_view(H);
  const int grid = H->grid;
  hipLaunchKernelGGL(k_hyb_init, dim3(grid), dim3(kBlock), 0, s, g, (int64_t)r);
  HYB_HIP(hipGetLastError(), "init launch");
  for (auto& b : H->bk) b.clear();
  for (auto& b : H->lk) b.clear();
  pool.run([&](int t) {
    int64_t lo, hi;
    share((int64_t)H->vis0_h.size(), t, T, &lo, &hi);
    std::copy(H->vis0_h.begin() + lo, H->vis0_h.begin() + hi, H->vis_h.begin() + lo);
    share(std::max<int64_t>(hv, 1), t, T, &lo, &hi);
    std::fill(H->dep_h + lo, H->dep_h + hi, -1);
    std::fill(H->par_h + lo, H->par_h + hi, -1);
    share(W, t, T, &lo, &hi);
    std::memset(cur + lo, 0, sizeof(uint64_t) * (size_t)(hi - lo));
  });
  cur[r >> 6] |= 1ull << (r & 63);
  if (r < hv) {
    H->vis_h[(size_t)(r >> 6)] |= 1ull << (r & 63);
    H->dep_h[(size_t)r] = 0;
    H->par_h[(size_t)r] = r;
  }
  HYB_HIP(hipMemcpyAsync(H->cur_g, cur, sizeof(uint64_t) * (size_t)W, hipMemcpyHostToDevice, s), "frontier copy");

  int32_t dir = prm.policy == DOBFS_POLICY_FORCED_BU ? kDirBU : kDirTD;
  int64_t n_f = 1, m_f = H->deg[(size_t)r], m_u = H->m - m_f;
  int32_t bu_run = 0, bu_phases = dir == kDirBU ? 1 : 0;
  int64_t reached = 1, reached_deg = m_f, checked_total = 0;
  int32_t levels = 0, log_len = 0;
  for (int32_t L = 0;; ++L) {
    /* both partitions run level L at once: the GPU's kernel is enqueued,
       then the host threads take the host's share */
    HYB_HIP(hipMemsetAsync(H->nxt_g + Wh, 0, sizeof(uint64_t) * (size_t)Wg, s), "level reset");
    HYB_HIP(hipMemsetAsync(H->cnt_g, 0, sizeof(unsigned long long) * 5, s), "level reset");
    if (timed) HYB_HIP(hipEventRecord(H->ev[0], s), "event");
    if (dir == kDirTD) {
      hipLaunchKernelGGL(k_hyb_td, dim3(grid), dim3(kBlock), 0, s, g, L);
      hipLaunchKernelGGL(k_hyb_td_long, dim3(grid), dim3(kBlock), 0, s, g, L);
    } else {
      hipLaunchKernelGGL(k_hyb_bu, dim3(grid), dim3(kBlock), 0, s, g, L);
    }
    HYB_HIP(hipGetLastError(), "level launch");
    if (timed) HYB_HIP(hipEventRecord(H->ev[1], s), "event");
    HYB_HIP(hipMemcpyAsync(cg, H->cnt_g, sizeof(unsigned long long) * 4, hipMemcpyDeviceToHost, s), "counter copy");
    if (dir == kDirTD && Wh > 0)
      HYB_HIP(hipMemcpyAsync(gmarks, H->push_g, sizeof(uint64_t) * (size_t)Wh, hipMemcpyDeviceToHost, s),
              "marks copy");
    const auto t_host = std::chrono::steady_clock::now();
    std::fill(H->nxt_h.begin(), H->nxt_h.end(), 0ull);
    Counts ch;
    try {
      ch = host_level(H, dir, L, cur, hmarks);
    } catch (const std::bad_alloc&) {
      (void)hipStreamSynchronize(s);
      return hfail(DOBFS_ENOMEM, "host level");
    }
    const double host_ms = ms_since(t_host);
    HYB_HIP(hipStreamSynchronize(s), "level");
    if (timed) HYB_HIP(kernel_ms(dir == kDirTD ? &td_ms : &bu_ms), "event time");
    ca[0] = ca[1] = ca[2] = ca[3] = 0ull;
    if (dir == kDirTD) {
      /* the marks each side made for the other (Algorithm 2): the host's go
         to the GPU (when there are any), the GPU's claim host vertices
         still unreached */
      const bool apply = Wg > 0 && ch.marks > 0;
      if (apply) {
        HYB_HIP(hipMemcpyAsync(H->pulled_g + Wh, hmarks + Wh, sizeof(uint64_t) * (size_t)Wg, hipMemcpyHostToDevice, s),
                "marks copy");
        HYB_HIP(hipMemsetAsync(H->cnt_g, 0, sizeof(unsigned long long) * 4, s), "apply reset");
        if (timed) HYB_HIP(hipEventRecord(H->ev[0], s), "event");
        hipLaunchKernelGGL(k_hyb_apply, dim3(grid), dim3(kBlock), 0, s, g, L);
        HYB_HIP(hipGetLastError(), "apply launch");
        if (timed) HYB_HIP(hipEventRecord(H->ev[1], s), "event");
        HYB_HIP(hipMemcpyAsync(ca, H->cnt_g, sizeof(unsigned long long) * 4, hipMemcpyDeviceToHost, s),
                "counter copy");
      }
      for (int64_t w = 0; w < Wh; ++w) {
        const uint64_t nw = gmarks[w] & ~H->vis_h[(size_t)w];
        if (!nw) continue;
        H->vis_h[(size_t)w] |= nw;
        H->nxt_h[(size_t)w] |= nw;
        for (uint64_t x = nw; x; x &= x - 1) {
          const int64_t v = w * 64 + __builtin_ctzll(x);
          H->dep_h[(size_t)v] = L + 1;
          H->par_h[(size_t)v] = kPending;
          ++ch.found;
          ch.found_deg += H->deg[(size_t)v];
        }
      }
      if (apply) {
        HYB_HIP(hipStreamSynchronize(s), "apply");
        if (timed) HYB_HIP(kernel_ms(&aux_ms), "event time");
      }
    }
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
      rec.t_end = (uint64_t)(ms_since(t_start) * 1e6);
      rec.kernel_ms = (float)host_ms;
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
    int32_t next = dir;  /* the switching rule (Section 3.3) */
    switch (prm.policy) {
      case DOBFS_POLICY_EDGE:
        if (dir == kDirTD) next = (mfn * (int64_t)prm.alpha > mu_next) ? kDirBU : kDirTD;
        else next = (nfn < n_f && nfn * (int64_t)prm.beta < n) ? kDirTD : kDirBU;
        break;
      case DOBFS_POLICY_PAPER: {
        /* with the hub partition deciding, its own next frontier (its
           claims and those the GPU's marks gave it) stands for the whole */
        const int64_t m_dec = hub_decides ? ch.found_deg : mfn;
        if (dir == kDirTD)
          next = (bu_phases == 0 && m_dec * (int64_t)prm.paper_pct > (n / prm.paper_div) * 100) ? kDirBU : kDirTD;
        else
          next = (run >= prm.paper_bu_steps) ? kDirTD : kDirBU;
        break;
      }
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
    /* the next frontier: the host's part goes to the device, whose own part
       is already in place (the two device bitmaps swap roles); the device's
       part comes to the host only for a bottom-up level, the one kind of
       host level that reads it */
    std::copy(H->nxt_h.begin(), H->nxt_h.begin() + Wh, cur);
    if (Wh > 0)
      HYB_HIP(hipMemcpyAsync(H->nxt_g, cur, sizeof(uint64_t) * (size_t)Wh, hipMemcpyHostToDevice, s),
              "frontier copy");
    if (dir == kDirBU && Wg > 0)
      HYB_HIP(hipMemcpyAsync(cur + Wh, H->nxt_g + Wh, sizeof(uint64_t) * (size_t)Wg, hipMemcpyDeviceToHost, s),
              "frontier copy");
    HYB_HIP(hipStreamSynchronize(s), "frontier copy");
    std::swap(H->cur_g, H->nxt_g);
    g = gpu_view(H);
    if (stats && log_len - 1 < stats->log_cap) stats->log[log_len - 1].t_end = (uint64_t)(ms_since(t_start) * 1e6);
  }
  /* deferred parents (Section 3.1), collected after the traversal: the
     GPU partition finds its own in its rows against both partitions'
     depths; a host vertex first reached through a GPU mark takes the GPU
     vertex whose mark first reached it, which the device recorded */
  if (hv > 0)
    HYB_HIP(hipMemcpyAsync(H->depth_g, H->dep_h, sizeof(int32_t) * (size_t)hv, hipMemcpyHostToDevice, s),
            "depth copy");
  if (timed) HYB_HIP(hipEventRecord(H->ev[0], s), "event");
  hipLaunchKernelGGL(k_hyb_resolve, dim3(grid), dim3(kBlock), 0, s, g, (const int32_t*)H->depth_g);
  HYB_HIP(hipGetLastError(), "resolve launch");
  if (hv > 0) {
    hipLaunchKernelGGL(k_hyb_merge, dim3(grid), dim3(kBlock), 0, s, H->parent_g, H->par_h_dev, hv);
    HYB_HIP(hipGetLastError(), "merge launch");
  }
  if (timed) HYB_HIP(hipEventRecord(H->ev[1], s), "event");
  /* caller IDs */
  hipLaunchKernelGGL(k_hyb_out, dim3(grid), dim3(kBlock), 0, s, (const int32_t*)H->depth_g,
                     (const int32_t*)H->parent_g, (const int32_t*)H->old2new_g, (const int32_t*)H->new2old_g, n,
                     depth, parent);
  HYB_HIP(hipGetLastError(), "output launch");
  HYB_HIP(hipStreamSynchronize(s), "output");
  if (timed) HYB_HIP(kernel_ms(&aux_ms), "event time");
  if (stats) {
    stats->levels = levels;
    stats->log_len = std::min(log_len, std::max(stats->log_cap, 0));
    stats->reached = reached;
    stats->m_c = reached_deg / 2;
    stats->checked = checked_total;
    stats->t_begin = 0;
    stats->level_launches = levels;
    stats->level_kernel_ms = td_ms + bu_ms;
    stats->td_kernel_ms = td_ms;
    stats->bu_kernel_ms = bu_ms;
    stats->aux_kernel_ms = aux_ms;
  }
  return DOBFS_OK;
}

int dobfs_hybrid_free(dobfs_hybrid_t H) {
  if (!H) return DOBFS_OK;
  {
    std::lock_guard<std::mutex> lk(H->mu);
  }
  release(H);
  return DOBFS_OK;
}

}  // extern "C"
