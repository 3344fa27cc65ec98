/*
 * C ABI of the direction-optimized BFS library: graph residency, workspaces
 * and the host side of the level loop.
 */
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dobfs_internal.h"

namespace dobfs {
namespace {

thread_local std::string g_last_error;

int fail(int status, const char* what, hipError_t e = hipSuccess) {
  g_last_error = what;
  if (e != hipSuccess) {
    g_last_error += ": ";
    g_last_error += hipGetErrorString(e);
  }
  return status;
}

#define DOBFS_HIP(call, what)                                             \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) return fail(DOBFS_EDEVICE, what, e_);           \
  } while (0)

template <class T>
hipError_t dalloc(T** p, int64_t count) {
  if (count < 1) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)count);
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

struct Workspace {
  uint64_t* vis = nullptr;
  uint64_t* fr0 = nullptr;
  uint64_t* fr1 = nullptr;
  int32_t* q0 = nullptr;
  int32_t* huge_u = nullptr;
  uint32_t* huge_base = nullptr;
  int32_t* parent_scratch = nullptr;
  int64_t* packed = nullptr;     /* relabelled graphs: internal (parent, depth) */
  Ctl* ctl = nullptr;
  dobfs_level_rec* log = nullptr;
  int32_t log_cap = 0;
  int32_t* done_host = nullptr;  /* pinned, 2 slots */
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipEvent_t idle = nullptr;     /* recorded after the last kernel of a run */
  std::vector<hipEvent_t> tev;   /* level-kernel timing events, 2 per launch */
  bool busy = false;

  void release() {
    dfree(vis); dfree(fr0); dfree(fr1); dfree(q0);
    dfree(huge_u); dfree(huge_base); dfree(parent_scratch); dfree(packed); dfree(ctl); dfree(log);
    if (done_host) (void)hipHostFree(done_host);
    for (auto& e : ev) if (e) (void)hipEventDestroy(e);
    if (idle) (void)hipEventDestroy(idle);
    for (auto& e : tev) (void)hipEventDestroy(e);
    *this = Workspace();
  }
};

constexpr int32_t kLogCap = 4096;

}  // namespace
}  // namespace dobfs

using namespace dobfs;

struct dobfs_graph_s {
  int64_t n = 0, m = 0;
  int64_t words = 0, words_active = 0;
  int64_t n_nonisolated = 0, max_degree = 0, n_huge = 0;
  uint32_t flags = 0;
  bool owns_csr = true;
  int64_t* off = nullptr;
  int32_t* idx = nullptr;
  uint64_t* iso = nullptr;
  int32_t* new2old = nullptr;  /* relabelled graphs only */
  int32_t* old2new = nullptr;
  int64_t* seg_lo = nullptr;
  int32_t nseg = 0;
  int device = 0;
  int grid = 0;
  std::mutex mu;
  std::vector<Workspace*> pool;

  GView view() const {
    GView g;
    g.off = off;
    g.idx = idx;
    g.iso = iso;
    g.old2new = old2new;
    g.new2old = new2old;
    g.seg_lo = seg_lo;
    g.nseg = nseg;
    g.pad_seg = 0;
    g.n = n;
    g.m = m;
    g.n_nonisolated = n_nonisolated;
    g.words = words;
    g.words_active = words_active;
    return g;
  }
};

namespace {

int alloc_workspace(dobfs_graph_s* g, Workspace* w) {
  const int64_t W = g->words;
  hipError_t e;
  if ((e = dalloc(&w->vis, W)) != hipSuccess || (e = dalloc(&w->fr0, W)) != hipSuccess ||
      (e = dalloc(&w->fr1, W)) != hipSuccess || (e = dalloc(&w->q0, g->n)) != hipSuccess || (e = dalloc(&w->huge_u, g->n_huge)) != hipSuccess ||
      (e = dalloc(&w->huge_base, g->n_huge)) != hipSuccess || (e = dalloc(&w->ctl, 1)) != hipSuccess ||
      (e = dalloc(&w->log, kLogCap)) != hipSuccess ||
      (g->new2old && (e = dalloc(&w->packed, g->n)) != hipSuccess)) {
    w->release();
    return fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "workspace allocation", e);
  }
  w->log_cap = kLogCap;
  if ((e = hipMemset(w->ctl, 0, sizeof(Ctl))) != hipSuccess) {  /* completion groups start at zero */
    w->release();
    return fail(DOBFS_EDEVICE, "workspace init", e);
  }
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&w->done_host), 2 * sizeof(int32_t))) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->ev[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->ev[1], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->idle, hipEventDisableTiming)) != hipSuccess) {
    w->release();
    return fail(DOBFS_EDEVICE, "workspace events", e);
  }
  return DOBFS_OK;
}

/* A workspace whose previous run has drained, or a new one. */
int acquire_workspace(dobfs_graph_s* g, Workspace** out) {
  std::lock_guard<std::mutex> lk(g->mu);
  for (Workspace* w : g->pool) {
    if (w->busy) continue;
    if (hipEventQuery(w->idle) != hipSuccess) continue;
    w->busy = true;
    *out = w;
    return DOBFS_OK;
  }
  Workspace* w = new (std::nothrow) Workspace();
  if (!w) return fail(DOBFS_ENOMEM, "workspace");
  const int st = alloc_workspace(g, w);
  if (st != DOBFS_OK) {
    delete w;
    return st;
  }
  w->busy = true;
  g->pool.push_back(w);
  *out = w;
  return DOBFS_OK;
}

void release_workspace(dobfs_graph_s* g, Workspace* w) {
  std::lock_guard<std::mutex> lk(g->mu);
  w->busy = false;
}

KParams to_kparams(const dobfs_params& p) {
  KParams k;
  k.policy = p.policy;
  k.alpha = p.alpha;
  k.beta = p.beta;
  k.paper_pct = p.paper_pct;
  k.paper_div = p.paper_div;
  k.paper_bu_steps = p.paper_bu_steps;
  k.td_wave_cut = p.td_wave_cut;
  k.td_huge_cut = p.td_huge_cut < kMinHugeCut ? kMinHugeCut : p.td_huge_cut;
  k.bu_heavy_cut = p.bu_heavy_cut;
  k.kappa_x1000 = p.kappa_x1000;
  k.seed = p.seed;
  return k;
}

int check_params(const dobfs_params& p) {
  if (p.policy < DOBFS_POLICY_EDGE || p.policy > DOBFS_POLICY_COST) return fail(DOBFS_EINVAL, "unknown policy");
  if (p.alpha < 1 || p.beta < 1 || p.paper_pct < 1 || p.paper_div < 1 || p.paper_bu_steps < 1 || p.kappa_x1000 < 1)
    return fail(DOBFS_EINVAL, "switching constants must be >= 1");
  if (p.td_wave_cut < 0 || p.td_wave_cut > 4096 || p.td_huge_cut < 1 || p.bu_heavy_cut < 1)
    return fail(DOBFS_EINVAL, "degree cut-offs out of range");
  if (p.chunk_levels < 1 || p.chunk_levels > 1024) return fail(DOBFS_EINVAL, "chunk_levels out of range");
  if (p.flags & ~DOBFS_RUN_TIME_KERNELS) return fail(DOBFS_EINVAL, "unknown run flag");
  return DOBFS_OK;
}

int first_direction(const dobfs_params& p) {
  if (p.policy == DOBFS_POLICY_FORCED_BU) return kDirBU;
  if (p.policy == DOBFS_POLICY_RANDOM) {
    uint64_t z = p.seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (int)(z & 1ull);
  }
  return kDirTD;
}

}  // namespace

extern "C" {

void dobfs_default_params(dobfs_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->policy = DOBFS_POLICY_EDGE;
  p->alpha = 14;
  p->beta = 24;
  p->paper_pct = 10;
  p->paper_div = 64;
  p->paper_bu_steps = 3;
  p->td_wave_cut = 16;
  p->td_huge_cut = 256;
  p->bu_heavy_cut = 256;
  p->chunk_levels = 8;
  p->flags = 0;
  p->kappa_x1000 = 500;
  p->seed = 0;
}

const char* dobfs_strerror(int status) {
  switch (status) {
    case DOBFS_OK: return "ok";
    case DOBFS_EINVAL: return "invalid argument";
    case DOBFS_ERANGE: return "vertex out of range";
    case DOBFS_ENOMEM: return "out of device memory";
    case DOBFS_EDEVICE: return "device error";
    case DOBFS_EBUSY: return "graph busy";
    case DOBFS_ENOTSUP: return "not supported";
    default: return "unknown status";
  }
}

const char* dobfs_last_error(void) { return g_last_error.c_str(); }

int dobfs_graph_upload(const int64_t* offsets, const int32_t* indices, int64_t n, int64_t m, uint32_t flags,
                       void* stream, dobfs_graph_t* out) {
  g_last_error.clear();
  if (!out) return fail(DOBFS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!offsets || (!indices && m > 0)) return fail(DOBFS_EINVAL, "offsets/indices is NULL");
  if (n < 1 || n > 2147483647LL || m < 0) return fail(DOBFS_EINVAL, "n must be in [1, 2^31-1], m >= 0");
  const uint32_t known =
      DOBFS_SRC_DEVICE | DOBFS_VALIDATE | DOBFS_VALIDATE_SYMMETRY | DOBFS_REINDEX_DEGREE | DOBFS_BORROW;
  if (flags & ~known) return fail(DOBFS_EINVAL, "unknown flag");
  if ((flags & DOBFS_BORROW) && !(flags & DOBFS_SRC_DEVICE)) return fail(DOBFS_EINVAL, "DOBFS_BORROW needs DOBFS_SRC_DEVICE");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  dobfs_graph_s* g = new (std::nothrow) dobfs_graph_s();
  if (!g) return fail(DOBFS_ENOMEM, "graph");
  g->n = n;
  g->m = m;
  g->words = (n + 63) / 64;
  g->flags = flags & DOBFS_REINDEX_DEGREE;
  int st = DOBFS_OK;
  int64_t* counters = nullptr;
  int32_t* bad = nullptr;
  hipError_t e;
  auto cleanup = [&](int status) {
    dfree(counters);
    dfree(bad);
    if (status != DOBFS_OK) {
      if (g->owns_csr) {
        dfree(g->off);
        dfree(g->idx);
      }
      dfree(g->iso);
      dfree(g->new2old);
      dfree(g->old2new);
      dfree(g->seg_lo);
      delete g;
    }
    return status;
  };
  if ((e = hipGetDevice(&g->device)) != hipSuccess) return cleanup(fail(DOBFS_EDEVICE, "hipGetDevice", e));
  if ((e = level_grid(&g->grid)) != hipSuccess) return cleanup(fail(DOBFS_EDEVICE, "occupancy query", e));
  const bool reindex = (flags & DOBFS_REINDEX_DEGREE) != 0;
  /* src_off/src_idx: the CSR as given, on the device */
  const int64_t* src_off = offsets;
  const int32_t* src_idx = indices;
  int64_t* tmp_off = nullptr;
  int32_t* tmp_idx = nullptr;
  auto drop_tmp = [&]() {
    dfree(tmp_off);
    dfree(tmp_idx);
    tmp_off = nullptr;
    tmp_idx = nullptr;
  };
  if ((flags & DOBFS_BORROW) && !reindex) {
    g->owns_csr = false;
    g->off = const_cast<int64_t*>(offsets);
    g->idx = const_cast<int32_t*>(indices);
    src_off = g->off;
    src_idx = g->idx;
  } else if (!(flags & DOBFS_SRC_DEVICE) || !reindex) {
    /* copy to the device: the graph itself, or the relabelling's source */
    int64_t** po = reindex ? &tmp_off : &g->off;
    int32_t** pi = reindex ? &tmp_idx : &g->idx;
    if ((e = dalloc(po, n + 1)) != hipSuccess || (e = dalloc(pi, m)) != hipSuccess) {
      drop_tmp();
      return cleanup(fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "graph allocation", e));
    }
    const hipMemcpyKind kind = (flags & DOBFS_SRC_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if ((e = hipMemcpyAsync(*po, offsets, sizeof(int64_t) * (size_t)(n + 1), kind, s)) != hipSuccess ||
        (m > 0 && (e = hipMemcpyAsync(*pi, indices, sizeof(int32_t) * (size_t)m, kind, s)) != hipSuccess)) {
      drop_tmp();
      return cleanup(fail(DOBFS_EDEVICE, "graph copy", e));
    }
    src_off = *po;
    src_idx = *pi;
  }
  if ((e = dalloc(&g->iso, g->words)) != hipSuccess || (e = dalloc(&counters, 4)) != hipSuccess ||
      (e = dalloc(&bad, 1)) != hipSuccess) {
    drop_tmp();
    return cleanup(fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "graph allocation", e));
  }
  /* Structure is always checked: a bad offset or index would make every
     later kernel read out of bounds. */
  if ((e = hipMemsetAsync(bad, 0, sizeof(int32_t), s)) != hipSuccess ||
      (e = launch_validate(src_off, src_idx, n, m, (flags & DOBFS_VALIDATE_SYMMETRY) ? 1 : 0, bad, g->grid, s)) !=
          hipSuccess) {
    drop_tmp();
    return cleanup(fail(DOBFS_EDEVICE, "validation launch", e));
  }
  int32_t bad_h = 0;
  if ((e = hipMemcpyAsync(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    drop_tmp();
    return cleanup(fail(DOBFS_EDEVICE, "validation", e));
  }
  if (bad_h) {
    static const char* what[] = {"", "offsets not monotone or not ending at m", "neighbour ID out of range",
                                 "self-loop", "missing reverse edge (CSR not symmetric or rows unsorted)"};
    drop_tmp();
    return cleanup(fail(DOBFS_EINVAL, what[bad_h < 5 ? bad_h : 0]));
  }
  if (reindex) {
    std::string err;
    st = build_reindexed(src_off, src_idx, n, m, g->grid, s, &g->off, &g->idx, &g->new2old, &g->old2new,
                         &g->seg_lo, &g->nseg, &err);
    drop_tmp();
    if (st != DOBFS_OK) return cleanup(fail(st, err.c_str()));
  }
  if ((e = hipMemsetAsync(counters, 0, 4 * sizeof(int64_t), s)) != hipSuccess ||
      (e = launch_graph_scan(g->off, n, g->iso, counters, g->grid, s)) != hipSuccess)
    return cleanup(fail(DOBFS_EDEVICE, "degree scan", e));
  int64_t ch[4] = {0, 0, 0, 0};
  if ((e = hipMemcpyAsync(ch, counters, sizeof(ch), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return cleanup(fail(DOBFS_EDEVICE, "degree scan", e));
  g->n_nonisolated = ch[0];
  g->max_degree = ch[1];
  g->n_huge = ch[2];
  /* relabelled graphs keep every degree-0 vertex in a suffix */
  g->words_active = reindex ? (g->n_nonisolated + 63) / 64 : g->words;
  (void)st;
  *out = g;
  return cleanup(DOBFS_OK);
}

int dobfs_graph_free(dobfs_graph_t g) {
  if (!g) return DOBFS_OK;
  for (Workspace* w : g->pool) {
    if (w->idle) (void)hipEventSynchronize(w->idle);
    w->release();
    delete w;
  }
  g->pool.clear();
  if (g->owns_csr) {
    dfree(g->off);
    dfree(g->idx);
  }
  dfree(g->iso);
  dfree(g->new2old);
  dfree(g->old2new);
  dfree(g->seg_lo);
  delete g;
  return DOBFS_OK;
}

int dobfs_graph_info(dobfs_graph_t g, dobfs_graph_info_t* info) {
  if (!g || !info) return fail(DOBFS_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n = g->n;
  info->m = g->m;
  info->n_nonisolated = g->n_nonisolated;
  info->max_degree = g->max_degree;
  info->device_bytes = (g->owns_csr ? (int64_t)sizeof(int64_t) * (g->n + 1) + (int64_t)sizeof(int32_t) * g->m : 0) +
                       (int64_t)sizeof(uint64_t) * g->words + (g->new2old ? 8 * g->n : 0);
  info->flags = g->flags;
  return DOBFS_OK;
}

int dobfs_run(dobfs_graph_t g, int64_t root, int32_t* depth, int32_t* parent, const dobfs_params* p,
              dobfs_stats* stats, void* stream) {
  g_last_error.clear();
  if (!g || !depth) return fail(DOBFS_EINVAL, "graph or depth is NULL");
  if (root < 0 || root >= g->n) return fail(DOBFS_ERANGE, "root outside [0, n)");
  dobfs_params prm;
  if (p) prm = *p; else dobfs_default_params(&prm);
  int st = check_params(prm);
  if (st != DOBFS_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Workspace* w = nullptr;
  if ((st = acquire_workspace(g, &w)) != DOBFS_OK) return st;
  struct Guard {
    dobfs_graph_s* g;
    Workspace* w;
    ~Guard() { release_workspace(g, w); }
  } guard{g, w};

  if (!parent && !g->new2old) {
    if (!w->parent_scratch) {
      hipError_t e = dalloc(&w->parent_scratch, g->n);
      if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "parent scratch", e);
    }
    parent = w->parent_scratch;
  }
  const GView gv = g->view();
  WView wv;
  wv.vis = w->vis;
  wv.fr0 = w->fr0;
  wv.fr1 = w->fr1;
  wv.q0 = w->q0;
  wv.huge_u = w->huge_u;
  wv.huge_base = w->huge_base;
  wv.depth = depth;
  wv.parent = parent;
  wv.packed = g->new2old ? w->packed : nullptr;
  wv.ctl = w->ctl;
  wv.log = w->log;
  wv.log_cap = w->log_cap;
  wv.pad = 0;
  const KParams kp = to_kparams(prm);

  DOBFS_HIP(launch_init(gv, wv, root, first_direction(prm), g->grid, s), "init launch");
  const int K = prm.chunk_levels;
  const bool timed = (prm.flags & DOBFS_RUN_TIME_KERNELS) != 0;
  int64_t launches = 0;
  auto enqueue_chunk = [&](int slot) -> int {
    for (int i = 0; i < K; ++i) {
      if (timed) {
        while ((int64_t)w->tev.size() < 2 * (launches + 1)) {
          hipEvent_t ev;
          DOBFS_HIP(hipEventCreate(&ev), "timing event");
          w->tev.push_back(ev);
        }
        DOBFS_HIP(hipEventRecord(w->tev[2 * launches], s), "timing event");
      }
      DOBFS_HIP(launch_level(gv, wv, kp, g->grid, s), "level launch");
      if (timed) DOBFS_HIP(hipEventRecord(w->tev[2 * launches + 1], s), "timing event");
      ++launches;
      DOBFS_HIP(launch_aux(gv, wv, kp, g->grid, s), "aux launch");
    }
    DOBFS_HIP(hipMemcpyAsync(&w->done_host[slot], &w->ctl->done, sizeof(int32_t), hipMemcpyDeviceToHost, s),
              "done flag copy");
    DOBFS_HIP(hipEventRecord(w->ev[slot], s), "event record");
    return DOBFS_OK;
  };
  /* One chunk is always queued ahead of the one being waited for, so the
     device never idles on the host's check. */
  if ((st = enqueue_chunk(0)) != DOBFS_OK) return st;
  const int64_t max_chunks = (g->n + 1) / K + 3;
  for (int64_t c = 0;; ++c) {
    if (c + 1 >= max_chunks) return fail(DOBFS_EDEVICE, "level loop did not terminate");
    if ((st = enqueue_chunk((int)((c + 1) & 1))) != DOBFS_OK) return st;
    DOBFS_HIP(hipEventSynchronize(w->ev[c & 1]), "level chunk");
    if (w->done_host[c & 1]) break;
  }
  if (g->new2old) DOBFS_HIP(launch_finalize(gv, wv, root, g->grid, s), "finalize launch");
  DOBFS_HIP(hipEventRecord(w->idle, s), "idle event");
  if (stats || timed) {
    Ctl ctl;
    DOBFS_HIP(hipMemcpyAsync(&ctl, w->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s), "stats copy");
    DOBFS_HIP(hipStreamSynchronize(s), "stats sync");
    if (!stats) return DOBFS_OK;
    stats->level_launches = (int32_t)launches;
    stats->level_kernel_ms = 0.0;
    std::vector<float> kms;
    if (timed) {
      kms.resize((size_t)launches);
      for (int64_t i = 0; i < launches; ++i) {
        float ms = 0.f;
        DOBFS_HIP(hipEventElapsedTime(&ms, w->tev[2 * i], w->tev[2 * i + 1]), "timing");
        kms[(size_t)i] = ms;
        stats->level_kernel_ms += ms;
      }
    }
    stats->levels = ctl.levels;
    stats->log_len = ctl.log_len < w->log_cap ? ctl.log_len : w->log_cap;
    stats->reached = ctl.reached;
    stats->m_c = ctl.reached_deg / 2;
    stats->checked = ctl.checked_total;
    stats->t_begin = ctl.t_begin;
    if (stats->log && stats->log_cap > 0) {
      const int32_t k = stats->log_len < stats->log_cap ? stats->log_len : stats->log_cap;
      if (k > 0)
        DOBFS_HIP(hipMemcpy(stats->log, w->log, sizeof(dobfs_level_rec) * (size_t)k, hipMemcpyDeviceToHost),
                  "log copy");
      for (int32_t i = 0; i < k; ++i) stats->log[i].kernel_ms = i < (int32_t)kms.size() ? kms[(size_t)i] : 0.f;
    }
  }
  return DOBFS_OK;
}

}  // extern "C"
