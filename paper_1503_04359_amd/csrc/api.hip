/*
 * C ABI of the direction-optimized BFS library: graph residency, workspaces
 * and the host side of the level loop.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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
  int32_t* qd0 = nullptr;
  int32_t* qd1 = nullptr;
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
  /* batched traversals, allocated on first use */
  uint64_t* ms_visit = nullptr;
  uint64_t* ms_cur0 = nullptr;
  uint64_t* ms_cur1 = nullptr;
  uint64_t* ms_nxt = nullptr;
  int32_t* ms_internal = nullptr;
  int64_t ms_internal_cap = 0;
  int32_t* roots_dev = nullptr;   /* multi-root runs */
  int64_t roots_cap = 0;
  bool busy = false;
  /* captured runs: a traversal's launches recorded once as a HIP graph and
     replayed while the arguments repeat (kind 0 single- and multi-source,
     kind 1 batched) */
  struct Captured {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
  };
  Captured cap[2];
  hipStream_t cap_stream = nullptr;  /* capture only: nothing runs on it */

  void release() {
    for (auto& c : cap)
      if (c.exec) (void)hipGraphExecDestroy(c.exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    dfree(ms_visit); dfree(ms_cur0); dfree(ms_cur1); dfree(ms_nxt); dfree(ms_internal); dfree(roots_dev);
    dfree(vis); dfree(fr0); dfree(fr1); dfree(q0); dfree(qd0); dfree(qd1);
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

void set_last_error(const char* what, hipError_t e) { (void)fail(DOBFS_OK, what, e); }

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
  int32_t* first = nullptr;    /* first neighbour of each vertex, -1 if none */
  /* Relabelled graphs: the caller ID of first[v], built by the first run
     (the caller may free its source CSR after upload, which makes room),
     skipped if memory is short.  Published only once filled: a run reads
     the pointer with acquire order, and the build sets first_caller_tried
     with release order after the column is complete (or given up), both
     under `mu`. */
  std::atomic<int32_t*> first_caller{nullptr};
  std::atomic<bool> first_caller_tried{false};
  int32_t* new2old = nullptr;  /* relabelled graphs only */
  int32_t* old2new = nullptr;
  int64_t* seg_lo = nullptr;
  int32_t nseg = 0;
  std::vector<int64_t> pack_base;  /* packs: first union ID of each graph, then n */
  int open_sessions = 0;
  int device = 0;
  int grid = 0;
  std::mutex mu;
  std::vector<Workspace*> pool;

  GView view() const {
    GView g;
    g.off = off;
    g.idx = idx;
    g.iso = iso;
    g.first = first;
    g.first_caller = first_caller.load(std::memory_order_acquire);
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

struct dobfs_session_s {
  dobfs_graph_s* g = nullptr;
  Workspace* w = nullptr;
  hipStream_t stream = nullptr;
  dobfs_params prm;
  KParams kp;
  int32_t** slot_out = nullptr;  /* device tables read by the kernels */
  int32_t* slot_start = nullptr;
  dobfs::Ctl* host_ctl = nullptr;  /* pinned copy of the control block */
  hipEvent_t ev = nullptr;
  uint64_t active = 0;   /* slots whose query runs */
  uint64_t dirty = 0;    /* slots whose bits still mark an ended query */
  int64_t tag[64] = {};
  int32_t root[64] = {};       /* caller ID of each slot's root */
  int32_t* out[64] = {};       /* caller's depth array of each slot */
  struct Pending {
    int32_t root;
    int32_t* depth;
    int64_t tag;
  };
  std::vector<Pending> pending;
  std::vector<int64_t> done;  /* ended, not yet reported */
  int64_t levels = 0;
  std::vector<dobfs_level_rec> last_log;  /* levels of the last chunk */
};

namespace {

int alloc_workspace(dobfs_graph_s* g, Workspace* w, hipStream_t s) {
  const int64_t W = g->words;
  hipError_t e;
  if ((e = dalloc(&w->vis, W)) != hipSuccess || (e = dalloc(&w->fr0, W)) != hipSuccess ||
      (e = dalloc(&w->fr1, W)) != hipSuccess || (e = dalloc(&w->q0, std::max(g->n, 4 * W))) != hipSuccess ||
      (e = dalloc(&w->qd0, kDirectCap)) != hipSuccess || (e = dalloc(&w->qd1, kDirectCap)) != hipSuccess ||
      (e = dalloc(&w->huge_u, g->n_huge)) != hipSuccess ||
      (e = dalloc(&w->huge_base, g->n_huge)) != hipSuccess || (e = dalloc(&w->ctl, 1)) != hipSuccess ||
      (e = dalloc(&w->log, kLogCap)) != hipSuccess ||
      (g->new2old && (e = dalloc(&w->packed, g->n)) != hipSuccess)) {
    w->release();
    return fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "workspace allocation", e);
  }
  w->log_cap = kLogCap;
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&w->done_host), 2 * sizeof(int32_t))) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->ev[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->ev[1], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&w->idle, hipEventDisableTiming)) != hipSuccess) {
    w->release();
    return fail(DOBFS_EDEVICE, "workspace events", e);
  }
  /* Completion groups start at zero.  The fill goes on the stream of the
     run that asked for the workspace, followed by the idle event: the null
     stream is not ordered with the caller's (non-blocking) streams, so a
     fill there could land after that run's first kernels had set up the
     control block; and a run that fails before launching anything still
     leaves the workspace marked busy until the fill is done. */
  if ((e = hipMemsetAsync(w->ctl, 0, sizeof(Ctl), s)) != hipSuccess ||
      (e = hipEventRecord(w->idle, s)) != hipSuccess) {
    (void)hipStreamSynchronize(s);
    w->release();
    return fail(DOBFS_EDEVICE, "workspace init", e);
  }
  return DOBFS_OK;
}

/* A workspace whose previous run has drained, or a new one (initialised on
   stream s, the stream its first run will use). */
int acquire_workspace(dobfs_graph_s* g, Workspace** out, hipStream_t s) {
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
  const int st = alloc_workspace(g, w, s);
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

/* Returns a run's workspace to the pool on every exit path.  Once anything
   has been enqueued (`launched`), an early return still marks the end of
   the stream's work with the idle event, so the workspace is not handed to
   another run while kernels of this one may still use it; if even that
   record fails, the stream is drained first. */
struct RunGuard {
  dobfs_graph_s* g;
  Workspace* w;
  hipStream_t s;
  bool launched = false;
  ~RunGuard() {
    if (launched && hipEventRecord(w->idle, s) != hipSuccess) (void)hipStreamSynchronize(s);
    release_workspace(g, w);
  }
};

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
  if (p.flags & ~(DOBFS_RUN_TIME_KERNELS | DOBFS_RUN_GRAPH | DOBFS_RUN_EAGER))
    return fail(DOBFS_EINVAL, "unknown run flag");
  if ((p.flags & DOBFS_RUN_GRAPH) && (p.flags & (DOBFS_RUN_EAGER | DOBFS_RUN_TIME_KERNELS)))
    return fail(DOBFS_EINVAL, "DOBFS_RUN_GRAPH excludes DOBFS_RUN_EAGER and DOBFS_RUN_TIME_KERNELS");
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

/* Host side of the level loop: chunks of K levels, each enqueued by
   `level(i)`, with one chunk always queued ahead of the one whose done flag
   the host waits for.  Returns the number of level slots enqueued. */
template <class LevelFn>
int level_loop(Workspace* w, const Ctl* ctl_dev, int K, int64_t max_levels, hipStream_t s, LevelFn level,
               int64_t* enqueued) {
  int64_t launches = 0;
  auto chunk = [&](int slot) -> int {
    for (int i = 0; i < K; ++i) {
      const int st = level(launches);
      if (st != DOBFS_OK) return st;
      ++launches;
    }
    DOBFS_HIP(hipMemcpyAsync(&w->done_host[slot], &ctl_dev->done, sizeof(int32_t), hipMemcpyDeviceToHost, s),
              "done flag copy");
    DOBFS_HIP(hipEventRecord(w->ev[slot], s), "event record");
    return DOBFS_OK;
  };
  int st = chunk(0);
  if (st != DOBFS_OK) return st;
  const int64_t max_chunks = max_levels / K + 3;
  for (int64_t c = 0;; ++c) {
    if (c + 1 >= max_chunks) return fail(DOBFS_EDEVICE, "level loop did not terminate");
    if ((st = chunk((int)((c + 1) & 1))) != DOBFS_OK) return st;
    DOBFS_HIP(hipEventSynchronize(w->ev[c & 1]), "level chunk");
    if (w->done_host[c & 1]) break;
  }
  *enqueued = launches;
  return DOBFS_OK;
}

/* Raw bytes of the arguments a captured run bakes in (the structs have no
   implicit padding). */
struct KeyBytes {
  std::vector<unsigned char> b;
  template <class T>
  KeyBytes& add(const T& x) {
    const unsigned char* p = reinterpret_cast<const unsigned char*>(&x);
    b.insert(b.end(), p, p + sizeof(T));
    return *this;
  }
};

/* The workspace's captured run of `kind` for these argument bytes: the
   cached graph when the bytes repeat, otherwise `enqueue(stream)` recorded
   on the workspace's capture stream and instantiated (nothing runs during
   capture).  The workspace is exclusive to one run at a time and its
   previous run has drained, so an old graph can be replaced. */
template <class Enqueue>
int captured_run(Workspace* w, int kind, const std::vector<unsigned char>& key, Enqueue enqueue,
                 hipGraphExec_t* out) {
  Workspace::Captured& c = w->cap[kind];
  if (c.exec && c.key == key) {
    *out = c.exec;
    return DOBFS_OK;
  }
  if (!w->cap_stream)
    DOBFS_HIP(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking), "capture stream");
  DOBFS_HIP(hipStreamBeginCapture(w->cap_stream, hipStreamCaptureModeThreadLocal), "graph capture");
  const int st = enqueue(w->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(w->cap_stream, &graph);
  if (st != DOBFS_OK || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return st != DOBFS_OK ? st : fail(DOBFS_EDEVICE, "graph capture", e);
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(DOBFS_EDEVICE, "graph instantiate", e2);
  if (c.exec) (void)hipGraphExecDestroy(c.exec);
  c.exec = exec;
  c.key = key;
  *out = exec;
  return DOBFS_OK;
}

/* Launches a captured run on s and reports, after waiting for it, whether
   the traversal ended within the run's level slots. */
int launch_captured(Workspace* w, hipGraphExec_t exec, const Ctl* ctl_dev, hipStream_t s, bool* done) {
  DOBFS_HIP(hipGraphLaunch(exec, s), "graph launch");
  DOBFS_HIP(hipMemcpyAsync(&w->done_host[0], &ctl_dev->done, sizeof(int32_t), hipMemcpyDeviceToHost, s),
            "done flag copy");
  DOBFS_HIP(hipEventRecord(w->ev[0], s), "event record");
  DOBFS_HIP(hipEventSynchronize(w->ev[0]), "captured run");
  *done = w->done_host[0] != 0;
  return DOBFS_OK;
}

int ensure_ms_buffers(dobfs_graph_s* g, Workspace* w, int32_t k) {
  hipError_t e = hipSuccess;
  if (!w->ms_visit) {
    if ((e = dalloc(&w->ms_visit, g->n)) != hipSuccess || (e = dalloc(&w->ms_cur0, g->n)) != hipSuccess ||
        (e = dalloc(&w->ms_cur1, g->n)) != hipSuccess || (e = dalloc(&w->ms_nxt, g->n)) != hipSuccess) {
      dfree(w->ms_visit); dfree(w->ms_cur0); dfree(w->ms_cur1); dfree(w->ms_nxt);
      w->ms_visit = w->ms_cur0 = w->ms_cur1 = w->ms_nxt = nullptr;
      return fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "batch workspace", e);
    }
  }
  if (g->new2old) {
    const int64_t need = g->n_nonisolated * (int64_t)k;
    if (need > w->ms_internal_cap) {
      dfree(w->ms_internal);
      w->ms_internal = nullptr;
      w->ms_internal_cap = 0;
      if ((e = dalloc(&w->ms_internal, need)) != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "batch labels", e);
      w->ms_internal_cap = need;
    }
  }
  return DOBFS_OK;
}

/* Stats of a finished traversal from its control block and level log. */
int fill_stats(const Ctl* ctl_dev, const dobfs_level_rec* log_dev, int32_t log_cap, hipStream_t s,
               dobfs_stats* stats, int64_t launches, const std::vector<float>& kms) {
  Ctl ctl;
  DOBFS_HIP(hipMemcpyAsync(&ctl, ctl_dev, sizeof(Ctl), hipMemcpyDeviceToHost, s), "stats copy");
  DOBFS_HIP(hipStreamSynchronize(s), "stats sync");
  stats->level_launches = (int32_t)launches;
  stats->level_kernel_ms = stats->td_kernel_ms = stats->bu_kernel_ms = stats->aux_kernel_ms = 0.0;
  for (size_t i = 0; i + 2 < kms.size(); i += 3) {
    stats->td_kernel_ms += kms[i];
    stats->bu_kernel_ms += kms[i + 1];
    stats->aux_kernel_ms += kms[i + 2];
  }
  stats->level_kernel_ms = stats->td_kernel_ms + stats->bu_kernel_ms + stats->aux_kernel_ms;
  stats->levels = ctl.levels;
  stats->log_len = ctl.log_len < log_cap ? ctl.log_len : log_cap;
  stats->reached = ctl.reached;
  stats->m_c = ctl.reached_deg / 2;
  stats->checked = ctl.checked_total;
  stats->t_begin = ctl.t_begin;
  if (stats->log && stats->log_cap > 0) {
    const int32_t k = stats->log_len < stats->log_cap ? stats->log_len : stats->log_cap;
    if (k > 0)
      DOBFS_HIP(hipMemcpyAsync(stats->log, log_dev, sizeof(dobfs_level_rec) * (size_t)k, hipMemcpyDeviceToHost, s),
                "log copy");
    DOBFS_HIP(hipStreamSynchronize(s), "log copy");
    for (int32_t i = 0; i < k; ++i) stats->log[i].kernel_ms = 0.f;
  }
  return DOBFS_OK;
}

/* ---- scratch of the allocation-free entry point -------------------------

   One fixed array per device holds the whole workspace of a traversal:
   bitmaps, queues, split list, control block, level log, and the packed
   labels (relabelled graphs) or the parent array (unrelabelled graphs run
   without a parent output).  Its device address is looked up once per
   device and kept; the array's name is only a host-side handle. */
constexpr uint64_t kScratchBytes = 64ull << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

/* Device address of `scratch` on device dev (current), looked up on the
   first call for that device. */
int scratch_base(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DOBFS_ENOTSUP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(DOBFS_EDEVICE, "scratch address", e);
    g_scratch[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch[dev];
  return DOBFS_OK;
}

struct NoallocLayout {
  uint64_t vis, fr0, fr1, q0, qd0, qd1, huge_u, huge_base, ctl, log, packed, parent, total;
};

/* Byte offsets of the workspace arrays in the scratch array (each on a
   256-byte boundary); the same sizes as a pooled workspace. */
NoallocLayout noalloc_layout(const dobfs_graph_s* g, bool own_parent) {
  NoallocLayout l;
  uint64_t at = 0;
  auto put = [&](uint64_t bytes) {
    const uint64_t here = at;
    at += (bytes + 255) & ~255ull;
    return here;
  };
  const uint64_t W = (uint64_t)g->words;
  const uint64_t n = (uint64_t)g->n;
  const uint64_t nh = (uint64_t)std::max<int64_t>(g->n_huge, 1);
  l.vis = put(8 * W);
  l.fr0 = put(8 * W);
  l.fr1 = put(8 * W);
  l.q0 = put(4 * std::max<uint64_t>(n, 4 * W));
  l.qd0 = put(4 * (uint64_t)kDirectCap);
  l.qd1 = put(4 * (uint64_t)kDirectCap);
  l.huge_u = put(4 * nh);
  l.huge_base = put(4 * nh);
  l.ctl = put(sizeof(Ctl));
  l.log = put(sizeof(dobfs_level_rec) * (uint64_t)kLogCap);
  l.packed = g->new2old ? put(8 * n) : 0;
  l.parent = own_parent ? put(4 * n) : 0;
  l.total = at;
  return l;
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
      dfree(g->first);
      dfree(g->first_caller.load());
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
  if ((e = dalloc(&g->first, n)) != hipSuccess)
    return cleanup(fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "first-neighbour column", e));
  if ((e = hipMemsetAsync(counters, 0, 4 * sizeof(int64_t), s)) != hipSuccess ||
      (e = launch_graph_scan(g->off, n, g->iso, counters, g->grid, s)) != hipSuccess ||
      (e = launch_first_column(g->off, g->idx, n, g->first, g->grid, s)) != hipSuccess)
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
  if (g->open_sessions > 0) return fail(DOBFS_EBUSY, "a session of this graph is still open");
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
  dfree(g->first);
  dfree(g->first_caller.load());
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
                       (int64_t)sizeof(uint64_t) * g->words + 4 * g->n + (g->new2old ? 8 * g->n : 0) +
                       (g->first_caller.load() ? 4 * g->n : 0);
  info->flags = g->flags;
  return DOBFS_OK;
}

/* One traversal seeded from nroots roots (host caller IDs in roots), or
   from root when roots is NULL. */
static int run_multi(dobfs_graph_t g, const int64_t* roots, int32_t nroots, int64_t root, int32_t* depth,
                     int32_t* parent, const dobfs_params* p, dobfs_stats* stats, void* stream,
                     bool graph_default = false) {
  g_last_error.clear();
  if (!g || !depth) return fail(DOBFS_EINVAL, "graph or depth is NULL");
  if (roots) {
    if (nroots < 1) return fail(DOBFS_EINVAL, "no roots");
    for (int32_t i = 0; i < nroots; ++i)
      if (roots[i] < 0 || roots[i] >= g->n) return fail(DOBFS_ERANGE, "root outside [0, n)");
  } else if (root < 0 || root >= g->n) {
    return fail(DOBFS_ERANGE, "root outside [0, n)");
  }
  dobfs_params prm;
  if (p) prm = *p; else dobfs_default_params(&prm);
  int st = check_params(prm);
  if (st != DOBFS_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Workspace* w = nullptr;
  if (g->new2old && !g->first_caller_tried.load(std::memory_order_acquire)) {
    std::lock_guard<std::mutex> lk(g->mu);
    if (!g->first_caller_tried.load(std::memory_order_relaxed)) {
      int32_t* col = nullptr;
      hipError_t e2 = dalloc(&col, g->n);
      if (e2 == hipSuccess) {
        e2 = launch_first_caller(g->first, g->new2old, g->n, col, g->grid, s);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
        if (e2 != hipSuccess) {
          dfree(col); /* not published; a later run tries again */
          return fail(DOBFS_EDEVICE, "first-neighbour caller column", e2);
        }
        g->first_caller.store(col, std::memory_order_release);
      } else {
        (void)hipGetLastError(); /* optional: parents are then all mapped by the finalize kernel */
      }
      g->first_caller_tried.store(true, std::memory_order_release);
    }
  }
  if ((st = acquire_workspace(g, &w, s)) != DOBFS_OK) return st;
  RunGuard guard{g, w, s};
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
  wv.qd0 = w->qd0;
  wv.qd1 = w->qd1;
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

  const int32_t* roots_dev = nullptr;
  if (roots) {
    if (w->roots_cap < nroots) {
      dfree(w->roots_dev);
      w->roots_dev = nullptr;
      w->roots_cap = 0;
      hipError_t e = dalloc(&w->roots_dev, nroots);
      if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "roots", e);
      w->roots_cap = nroots;
    }
    std::vector<int32_t> r32(roots, roots + nroots);
    DOBFS_HIP(hipMemcpyAsync(w->roots_dev, r32.data(), sizeof(int32_t) * (size_t)nroots, hipMemcpyHostToDevice, s),
              "roots copy");
    DOBFS_HIP(hipStreamSynchronize(s), "roots copy");
    roots_dev = w->roots_dev;
  }
  const bool timed = (prm.flags & DOBFS_RUN_TIME_KERNELS) != 0;
  const bool graph = !timed && !(prm.flags & DOBFS_RUN_EAGER) && (graph_default || (prm.flags & DOBFS_RUN_GRAPH));
  /* timed runs bracket each of the slot's three kernels with events:
     tev[4i] k_level_td tev[4i+1] k_level_bu tev[4i+2] k_aux tev[4i+3] */
  auto level = [&](int64_t i) -> int {
    if (!timed) {
      DOBFS_HIP(launch_level(gv, wv, kp, g->grid, s), "level launch");
      DOBFS_HIP(launch_aux(gv, wv, kp, g->grid, s), "aux launch");
      return DOBFS_OK;
    }
    while ((int64_t)w->tev.size() < 4 * (i + 1)) {
      hipEvent_t ev;
      DOBFS_HIP(hipEventCreate(&ev), "timing event");
      w->tev.push_back(ev);
    }
    hipEvent_t* ev = &w->tev[4 * i];
    DOBFS_HIP(hipEventRecord(ev[0], s), "timing event");
    DOBFS_HIP(launch_level_td(gv, wv, kp, g->grid, s), "level launch");
    DOBFS_HIP(hipEventRecord(ev[1], s), "timing event");
    DOBFS_HIP(launch_level_bu(gv, wv, kp, g->grid, s), "level launch");
    DOBFS_HIP(hipEventRecord(ev[2], s), "timing event");
    DOBFS_HIP(launch_aux(gv, wv, kp, g->grid, s), "aux launch");
    DOBFS_HIP(hipEventRecord(ev[3], s), "timing event");
    return DOBFS_OK;
  };
  auto finalize = [&](hipStream_t cs) -> int {
    if (g->new2old) {
      DOBFS_HIP(launch_finalize(gv, wv, roots ? -1 : root, g->grid, cs), "finalize launch");
      if (roots) DOBFS_HIP(launch_fix_roots(wv, roots_dev, nroots, cs), "root labels launch");
    }
    return DOBFS_OK;
  };
  int64_t launches = 0;
  if (graph) {
    /* one captured run: init, 2 * chunk_levels level slots and the
       finalize; a traversal with more levels continues with ordinary
       launches and maps its results again at the end */
    const int K0 = 2 * prm.chunk_levels;
    const int32_t first_dir = first_direction(prm);
    auto enqueue = [&](hipStream_t cs) -> int {
      DOBFS_HIP(launch_init(gv, wv, roots_dev, roots ? nroots : 1, root, first_dir, g->grid, cs), "init launch");
      for (int i = 0; i < K0; ++i) {
        DOBFS_HIP(launch_level(gv, wv, kp, g->grid, cs), "level launch");
        DOBFS_HIP(launch_aux(gv, wv, kp, g->grid, cs), "aux launch");
      }
      return finalize(cs);
    };
    KeyBytes key;
    key.add(gv).add(wv).add(kp).add(K0).add(root).add(nroots).add(roots_dev).add(first_dir);
    hipGraphExec_t exec = nullptr;
    if ((st = captured_run(w, 0, key.b, enqueue, &exec)) != DOBFS_OK) return st;
    guard.launched = true;
    bool done = false;
    if ((st = launch_captured(w, exec, w->ctl, s, &done)) != DOBFS_OK) return st;
    launches = K0;
    if (!done) {
      int64_t more = 0;
      if ((st = level_loop(w, w->ctl, prm.chunk_levels, g->n + 1, s, level, &more)) != DOBFS_OK) return st;
      launches += more;
      if ((st = finalize(s)) != DOBFS_OK) return st;
    }
  } else {
    guard.launched = true;
    DOBFS_HIP(launch_init(gv, wv, roots_dev, roots ? nroots : 1, root, first_direction(prm), g->grid, s),
              "init launch");
    if ((st = level_loop(w, w->ctl, prm.chunk_levels, g->n + 1, s, level, &launches)) != DOBFS_OK) return st;
    if ((st = finalize(s)) != DOBFS_OK) return st;
  }
  DOBFS_HIP(hipEventRecord(w->idle, s), "idle event");
  guard.launched = false;
  if (!stats) return DOBFS_OK;
  std::vector<float> kms;  /* per slot: k_level_td, k_level_bu, k_aux */
  if (timed) {
    /* the lookahead chunk may still be running: wait before reading its events */
    DOBFS_HIP(hipEventSynchronize(w->idle), "timing wait");
    kms.resize((size_t)(3 * launches));
    for (int64_t i = 0; i < launches; ++i)
      for (int k = 0; k < 3; ++k)
        DOBFS_HIP(hipEventElapsedTime(&kms[(size_t)(3 * i + k)], w->tev[4 * i + k], w->tev[4 * i + k + 1]),
                  "timing");
  }
  return fill_stats(w->ctl, w->log, w->log_cap, s, stats, launches, kms);
}

int dobfs_run(dobfs_graph_t g, int64_t root, int32_t* depth, int32_t* parent, const dobfs_params* p,
              dobfs_stats* stats, void* stream) {
  return run_multi(g, nullptr, 0, root, depth, parent, p, stats, stream);
}

/* Single-source run whose workspace is the device's fixed scratch array
   (see noalloc_layout): no device or pinned allocation, no events.  The
   host checks the done flag after each chunk of levels with a plain copy
   and a stream synchronisation, and the call returns once the outputs are
   complete.  Overlapping calls on one device share the array and race. */
int dobfs_run_noalloc(dobfs_graph_t g, int64_t root, int32_t* depth, int32_t* parent, const dobfs_params* p,
                      dobfs_stats* stats, void* stream) {
  g_last_error.clear();
  if (!g || !depth) return fail(DOBFS_EINVAL, "graph or depth is NULL");
  if (root < 0 || root >= g->n) return fail(DOBFS_ERANGE, "root outside [0, n)");
  dobfs_params prm;
  if (p) prm = *p; else dobfs_default_params(&prm);
  int st = check_params(prm);
  if (st != DOBFS_OK) return st;
  if (prm.flags & (DOBFS_RUN_TIME_KERNELS | DOBFS_RUN_GRAPH))
    return fail(DOBFS_EINVAL, "DOBFS_RUN_TIME_KERNELS and DOBFS_RUN_GRAPH need events or graphs, which the "
                              "allocation-free run does not create");
  int dev = 0;
  DOBFS_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev != g->device) return fail(DOBFS_EINVAL, "the graph is resident on another device");
  unsigned char* base = nullptr;
  if ((st = scratch_base(dev, &base)) != DOBFS_OK) return st;
  const bool own_parent = !parent && !g->new2old;  /* parents kept in scratch, not returned */
  const NoallocLayout lay = noalloc_layout(g, own_parent);
  if (lay.total > kScratchBytes) {
    char msg[192];
    std::snprintf(msg, sizeof(msg),
                  "graph needs %llu bytes of traversal scratch; the allocation-free run has %llu (n <= ~2.5M vertices)",
                  (unsigned long long)lay.total, (unsigned long long)kScratchBytes);
    return fail(DOBFS_ENOTSUP, msg);
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const GView gv = g->view();
  WView wv;
  wv.vis = reinterpret_cast<uint64_t*>(base + lay.vis);
  wv.fr0 = reinterpret_cast<uint64_t*>(base + lay.fr0);
  wv.fr1 = reinterpret_cast<uint64_t*>(base + lay.fr1);
  wv.q0 = reinterpret_cast<int32_t*>(base + lay.q0);
  wv.qd0 = reinterpret_cast<int32_t*>(base + lay.qd0);
  wv.qd1 = reinterpret_cast<int32_t*>(base + lay.qd1);
  wv.huge_u = reinterpret_cast<int32_t*>(base + lay.huge_u);
  wv.huge_base = reinterpret_cast<uint32_t*>(base + lay.huge_base);
  wv.depth = depth;
  wv.parent = own_parent ? reinterpret_cast<int32_t*>(base + lay.parent) : parent;
  wv.packed = g->new2old ? reinterpret_cast<int64_t*>(base + lay.packed) : nullptr;
  wv.ctl = reinterpret_cast<Ctl*>(base + lay.ctl);
  wv.log = reinterpret_cast<dobfs_level_rec*>(base + lay.log);
  wv.log_cap = kLogCap;
  wv.pad = 0;
  const KParams kp = to_kparams(prm);
  /* the init kernels clear everything a traversal reads before writing it,
     the completion groups included, so the array's previous contents do
     not matter */
  DOBFS_HIP(launch_init(gv, wv, nullptr, 1, root, first_direction(prm), g->grid, s), "init launch");
  const int K = prm.chunk_levels;
  const int64_t max_chunks = (g->n + 1) / K + 3;
  int64_t launches = 0;
  for (int64_t c = 0;; ++c) {
    if (c >= max_chunks) return fail(DOBFS_EDEVICE, "level loop did not terminate");
    for (int i = 0; i < K; ++i, ++launches) {
      DOBFS_HIP(launch_level(gv, wv, kp, g->grid, s), "level launch");
      DOBFS_HIP(launch_aux(gv, wv, kp, g->grid, s), "aux launch");
    }
    int32_t done = 0;
    DOBFS_HIP(hipMemcpyAsync(&done, &wv.ctl->done, sizeof(int32_t), hipMemcpyDeviceToHost, s), "done flag copy");
    DOBFS_HIP(hipStreamSynchronize(s), "level chunk");
    if (done) break;
  }
  if (g->new2old) DOBFS_HIP(launch_finalize(gv, wv, root, g->grid, s), "finalize launch");
  if (stats) {
    const std::vector<float> none;
    if ((st = fill_stats(wv.ctl, wv.log, wv.log_cap, s, stats, launches, none)) != DOBFS_OK) return st;
  }
  DOBFS_HIP(hipStreamSynchronize(s), "finalize");
  return DOBFS_OK;
}

int dobfs_run_multi(dobfs_graph_t g, const int64_t* roots, int32_t nroots, int32_t* depth, int32_t* parent,
                    const dobfs_params* p, dobfs_stats* stats, void* stream) {
  if (!roots) return fail(DOBFS_EINVAL, "roots is NULL");
  return run_multi(g, roots, nroots, -1, depth, parent, p, stats, stream);
}

int dobfs_batch_submit(dobfs_graph_t g, const int64_t* roots, int32_t k, int32_t* depth, const dobfs_params* p,
                       dobfs_stats* stats, void* stream) {
  g_last_error.clear();
  if (!g || !roots || !depth) return fail(DOBFS_EINVAL, "graph, roots or depth is NULL");
  if (k < 1 || k > 64) return fail(DOBFS_EINVAL, "k must be in [1, 64]");
  MsRoots r;
  std::memset(&r, 0, sizeof(r));
  for (int32_t b = 0; b < k; ++b) {
    if (roots[b] < 0 || roots[b] >= g->n) return fail(DOBFS_ERANGE, "root outside [0, n)");
    r.r[b] = (int32_t)roots[b];
  }
  dobfs_params prm;
  if (p) prm = *p; else dobfs_default_params(&prm);
  int st = check_params(prm);
  if (st != DOBFS_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Workspace* w = nullptr;
  if ((st = acquire_workspace(g, &w, s)) != DOBFS_OK) return st;
  RunGuard guard{g, w, s};
  if ((st = ensure_ms_buffers(g, w, k)) != DOBFS_OK) return st;
  const GView gv = g->view();
  MsView m;
  m.visit = w->ms_visit;
  m.cur0 = w->ms_cur0;
  m.cur1 = w->ms_cur1;
  m.nxt = w->ms_nxt;
  m.out = depth;
  m.internal = g->new2old ? w->ms_internal : nullptr;
  m.k = k;
  m.pad = 0;
  m.full = k == 64 ? ~0ull : ((1ull << k) - 1ull);
  m.ctl = w->ctl;
  m.log = w->log;
  m.log_cap = w->log_cap;
  m.session = 0;
  m.slot_out = nullptr;
  m.slot_start = nullptr;
  m.split_u = w->huge_u;
  m.split_base = w->huge_base;
  const KParams kp = to_kparams(prm);
  const int32_t first_pull = first_direction(prm) == kDirBU ? 1 : 0;
  auto level = [&](int64_t) -> int {
    DOBFS_HIP(launch_ms_level(gv, m, kp, g->grid, s), "batch level launch");
    return DOBFS_OK;
  };
  auto finalize = [&](hipStream_t cs) -> int {
    if (g->new2old) DOBFS_HIP(launch_ms_finalize(gv, m, r, g->grid, cs), "batch finalize launch");
    return DOBFS_OK;
  };
  int64_t launches = 0;
  if (!(prm.flags & (DOBFS_RUN_EAGER | DOBFS_RUN_TIME_KERNELS))) {
    /* the whole batch as one captured run: init, 2 * chunk_levels level
       slots (three kernels each) and the finalize; more levels continue
       with ordinary launches, then the finalize runs again */
    const int K0 = 2 * prm.chunk_levels;
    auto enqueue = [&](hipStream_t cs) -> int {
      DOBFS_HIP(launch_ms_init(gv, m, r, first_pull, g->grid, cs), "batch init launch");
      for (int i = 0; i < K0; ++i) DOBFS_HIP(launch_ms_level(gv, m, kp, g->grid, cs), "batch level launch");
      return finalize(cs);
    };
    KeyBytes key;
    key.add(gv).add(m).add(kp).add(r).add(K0).add(first_pull);
    hipGraphExec_t exec = nullptr;
    if ((st = captured_run(w, 1, key.b, enqueue, &exec)) != DOBFS_OK) return st;
    guard.launched = true;
    bool done = false;
    if ((st = launch_captured(w, exec, w->ctl, s, &done)) != DOBFS_OK) return st;
    launches = K0;
    if (!done) {
      int64_t more = 0;
      if ((st = level_loop(w, w->ctl, prm.chunk_levels, g->n + 1, s, level, &more)) != DOBFS_OK) return st;
      launches += more;
      if ((st = finalize(s)) != DOBFS_OK) return st;
    }
  } else {
    guard.launched = true;
    DOBFS_HIP(launch_ms_init(gv, m, r, first_pull, g->grid, s), "batch init launch");
    if ((st = level_loop(w, w->ctl, prm.chunk_levels, g->n + 1, s, level, &launches)) != DOBFS_OK) return st;
    if ((st = finalize(s)) != DOBFS_OK) return st;
  }
  DOBFS_HIP(hipEventRecord(w->idle, s), "idle event");
  guard.launched = false;
  if (!stats) return DOBFS_OK;
  return fill_stats(w->ctl, w->log, w->log_cap, s, stats, launches, std::vector<float>());
}

int dobfs_pack_upload(int32_t count, const int64_t* const* offsets, const int32_t* const* indices, const int64_t* n,
                      const int64_t* m, uint32_t flags, void* stream, dobfs_graph_t* out) {
  g_last_error.clear();
  if (!out) return fail(DOBFS_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || !offsets || !indices || !n || !m) return fail(DOBFS_EINVAL, "empty pack or NULL arrays");
  if (flags & ~(DOBFS_SRC_DEVICE | DOBFS_VALIDATE | DOBFS_VALIDATE_SYMMETRY | DOBFS_REINDEX_DEGREE))
    return fail(DOBFS_EINVAL, "unknown flag");
  std::vector<int64_t> nb((size_t)count + 1, 0), mb((size_t)count + 1, 0);
  for (int32_t i = 0; i < count; ++i) {
    if (!offsets[i] || (!indices[i] && m[i] > 0) || n[i] < 1 || m[i] < 0) return fail(DOBFS_EINVAL, "bad graph in pack");
    nb[(size_t)i + 1] = nb[(size_t)i] + n[i];
    mb[(size_t)i + 1] = mb[(size_t)i] + m[i];
  }
  const int64_t N = nb[(size_t)count], M = mb[(size_t)count];
  if (N > 2147483647LL) return fail(DOBFS_EINVAL, "pack has more than 2^31-1 vertices");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int64_t* uoff = nullptr;
  int32_t* uidx = nullptr;
  hipError_t e;
  if ((e = dalloc(&uoff, N + 1)) != hipSuccess || (e = dalloc(&uidx, M)) != hipSuccess) {
    dfree(uoff);
    dfree(uidx);
    return fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "pack allocation", e);
  }
  const bool dev = (flags & DOBFS_SRC_DEVICE) != 0;
  int st = DOBFS_OK;
  for (int32_t i = 0; i < count && st == DOBFS_OK; ++i) {
    e = launch_pack_copy(offsets[i], indices[i], n[i], m[i], nb[(size_t)i], mb[(size_t)i], dev, uoff, uidx, s);
    if (e != hipSuccess) st = fail(DOBFS_EDEVICE, "pack copy", e);
  }
  if (st == DOBFS_OK && (e = hipStreamSynchronize(s)) != hipSuccess) st = fail(DOBFS_EDEVICE, "pack copy", e);
  if (st != DOBFS_OK) {
    dfree(uoff);
    dfree(uidx);
    return st;
  }
  const bool reindex = (flags & DOBFS_REINDEX_DEGREE) != 0;
  dobfs_graph_t g = nullptr;
  st = dobfs_graph_upload(uoff, uidx, N, M, (flags & ~DOBFS_SRC_DEVICE) | DOBFS_SRC_DEVICE | (reindex ? 0u : DOBFS_BORROW),
                          stream, &g);
  if (st != DOBFS_OK || reindex) {
    dfree(uoff);
    dfree(uidx);
  }
  if (st != DOBFS_OK) return st;
  if (!reindex) g->owns_csr = true;  /* the union arrays now belong to the graph */
  g->pack_base = nb;
  *out = g;
  return DOBFS_OK;
}

int dobfs_pack_bases(dobfs_graph_t pack, int64_t* bases) {
  if (!pack || !bases) return fail(DOBFS_EINVAL, "NULL argument");
  if (pack->pack_base.empty()) return fail(DOBFS_EINVAL, "not a pack");
  for (size_t i = 0; i < pack->pack_base.size(); ++i) bases[i] = pack->pack_base[i];
  return DOBFS_OK;
}

int dobfs_pack_run(dobfs_graph_t pack, const int64_t* roots, int32_t* depth, int32_t* parent, const dobfs_params* p,
                   dobfs_stats* stats, void* stream) {
  g_last_error.clear();
  if (!pack || !roots || !depth) return fail(DOBFS_EINVAL, "pack, roots or depth is NULL");
  if (pack->pack_base.empty()) return fail(DOBFS_EINVAL, "not a pack");
  const int32_t count = (int32_t)pack->pack_base.size() - 1;
  std::vector<int64_t> global((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    const int64_t lo = pack->pack_base[(size_t)i], hi = pack->pack_base[(size_t)i + 1];
    if (roots[i] < 0 || lo + roots[i] >= hi) return fail(DOBFS_ERANGE, "root outside its graph");
    global[(size_t)i] = lo + roots[i];
  }
  return run_multi(pack, global.data(), count, -1, depth, parent, p, stats, stream, /*graph_default=*/true);
}

static int session_view(dobfs_session_s* ss, MsView* m) {
  Workspace* w = ss->w;
  m->visit = w->ms_visit;
  m->cur0 = w->ms_cur0;
  m->cur1 = w->ms_cur1;
  m->nxt = w->ms_nxt;
  m->out = nullptr;
  m->internal = ss->g->new2old ? w->ms_internal : nullptr;
  m->k = 64;
  m->pad = 0;
  m->full = ss->active;
  m->ctl = w->ctl;
  m->log = w->log;
  m->log_cap = ss->prm.chunk_levels < w->log_cap ? ss->prm.chunk_levels : w->log_cap;
  m->session = 1;
  m->slot_out = ss->slot_out;
  m->slot_start = ss->slot_start;
  m->split_u = w->huge_u;
  m->split_base = w->huge_base;
  return DOBFS_OK;
}

int dobfs_session_open(dobfs_graph_t g, const dobfs_params* p, void* stream, dobfs_session_t* out) {
  g_last_error.clear();
  if (!g || !out) return fail(DOBFS_EINVAL, "graph or out is NULL");
  *out = nullptr;
  dobfs_params prm;
  if (p) prm = *p; else dobfs_default_params(&prm);
  int st = check_params(prm);
  if (st != DOBFS_OK) return st;
  dobfs_session_s* ss = new (std::nothrow) dobfs_session_s();
  if (!ss) return fail(DOBFS_ENOMEM, "session");
  ss->g = g;
  ss->stream = reinterpret_cast<hipStream_t>(stream);
  ss->prm = prm;
  ss->kp = to_kparams(prm);
  auto undo = [&](int status) {
    dfree(ss->slot_out);
    dfree(ss->slot_start);
    if (ss->host_ctl) (void)hipHostFree(ss->host_ctl);
    if (ss->ev) (void)hipEventDestroy(ss->ev);
    if (ss->w) release_workspace(g, ss->w);
    delete ss;
    return status;
  };
  if ((st = acquire_workspace(g, &ss->w, ss->stream)) != DOBFS_OK) {
    ss->w = nullptr;
    return undo(st);
  }
  /* relabelled graphs: depths go to internal order first (one slot-major
     row per slot), mapped to caller order when the query ends */
  if ((st = ensure_ms_buffers(g, ss->w, 64)) != DOBFS_OK) return undo(st);
  hipError_t e;
  if ((e = dalloc(&ss->slot_out, 64)) != hipSuccess || (e = dalloc(&ss->slot_start, 64)) != hipSuccess)
    return undo(fail(e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE, "session tables", e));
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&ss->host_ctl), sizeof(Ctl))) != hipSuccess ||
      (e = hipEventCreateWithFlags(&ss->ev, hipEventDisableTiming)) != hipSuccess)
    return undo(fail(DOBFS_EDEVICE, "session host state", e));
  MsView m;
  session_view(ss, &m);
  if ((e = launch_ms_session_start(g->view(), m, g->grid, ss->stream)) != hipSuccess)
    return undo(fail(DOBFS_EDEVICE, "session start launch", e));
  {
    std::lock_guard<std::mutex> lk(g->mu);
    ++g->open_sessions;
  }
  *out = ss;
  return DOBFS_OK;
}

int dobfs_session_admit(dobfs_session_t ss, int64_t root, int32_t* depth, int64_t tag) {
  g_last_error.clear();
  if (!ss || !depth) return fail(DOBFS_EINVAL, "session or depth is NULL");
  if (root < 0 || root >= ss->g->n) return fail(DOBFS_ERANGE, "root outside [0, n)");
  if (__builtin_popcountll(ss->active) + (int)ss->pending.size() >= 64) return fail(DOBFS_EBUSY, "64 queries in flight");
  ss->pending.push_back({(int32_t)root, depth, tag});
  return DOBFS_OK;
}

int dobfs_session_step(dobfs_session_t ss, int64_t* done_tags, int32_t cap, int32_t* n_done) {
  g_last_error.clear();
  if (!ss || !n_done || (cap > 0 && !done_tags) || cap < 0) return fail(DOBFS_EINVAL, "NULL argument or cap < 0");
  *n_done = 0;
  dobfs_graph_s* g = ss->g;
  const hipStream_t s = ss->stream;
  const GView gv = g->view();
  if (!ss->pending.empty()) {
    /* free slots: never used first, then those of ended queries (cleared
       all at once, so that a clearing pass serves many admissions) */
    const uint64_t free_clean = ~(ss->active | ss->dirty);
    const int need = (int)ss->pending.size();
    uint64_t clear = 0;
    if (__builtin_popcountll(free_clean) < need) {
      clear = ss->dirty;
      ss->dirty = 0;
    }
    uint64_t avail = ~ss->active & ~ss->dirty;
    MsRoots r;
    SlotOuts outs;
    std::memset(&r, 0, sizeof(r));
    std::memset(&outs, 0, sizeof(outs));
    uint64_t bits = 0;
    for (const auto& q : ss->pending) {
      const int b = __builtin_ctzll(avail);
      avail &= avail - 1;
      bits |= 1ull << b;
      r.r[b] = q.root;
      outs.p[b] = q.depth;
      ss->tag[b] = q.tag;
      ss->root[b] = q.root;
      ss->out[b] = q.depth;
      /* unrelabelled graphs write depths straight into the caller's array */
      if (!g->new2old)
        DOBFS_HIP(hipMemsetAsync(q.depth, 0xff, sizeof(int32_t) * (size_t)g->n, s), "query output init");
    }
    ss->pending.clear();
    ss->active |= bits;
    MsView m;
    session_view(ss, &m);
    DOBFS_HIP(launch_ms_session_admit(gv, m, clear, r, outs, bits,
                                      ss->prm.policy == DOBFS_POLICY_FORCED_BU ? 1 : 0, g->grid, s),
              "admission launch");
  }
  ss->last_log.clear();
  if (ss->active) {
    MsView m;
    session_view(ss, &m);
    /* the log holds the levels of this chunk only */
    DOBFS_HIP(hipMemsetAsync(&ss->w->ctl->log_len, 0, sizeof(int32_t), s), "log reset");
    for (int i = 0; i < ss->prm.chunk_levels; ++i)
      DOBFS_HIP(launch_ms_level(gv, m, ss->kp, g->grid, s), "session level launch");
    DOBFS_HIP(hipMemcpyAsync(ss->host_ctl, ss->w->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s), "state copy");
    DOBFS_HIP(hipEventRecord(ss->ev, s), "event record");
    DOBFS_HIP(hipEventSynchronize(ss->ev), "session chunk");
    ss->levels = ss->host_ctl->level;
    const int32_t nlog = std::min(ss->host_ctl->log_len, m.log_cap);
    if (nlog > 0) {
      ss->last_log.resize((size_t)nlog);
      DOBFS_HIP(hipMemcpyAsync(ss->last_log.data(), ss->w->log, sizeof(dobfs_level_rec) * (size_t)nlog,
                               hipMemcpyDeviceToHost, s), "log copy");
      DOBFS_HIP(hipStreamSynchronize(s), "log copy");
    }
    const uint64_t ended = ss->active & ~ss->host_ctl->live;
    if (ended && g->new2old) {
      MsRoots r;
      SlotOuts outs;
      std::memset(&r, 0, sizeof(r));
      std::memset(&outs, 0, sizeof(outs));
      for (uint64_t x = ended; x; x &= x - 1) {
        const int b = __builtin_ctzll(x);
        r.r[b] = ss->root[b];
        outs.p[b] = ss->out[b];
      }
      DOBFS_HIP(launch_ms_session_finalize(gv, m, r, outs, ended, g->grid, s), "query finalize launch");
      DOBFS_HIP(hipEventRecord(ss->ev, s), "event record");
      DOBFS_HIP(hipEventSynchronize(ss->ev), "query finalize");
    }
    for (uint64_t x = ended; x; x &= x - 1) ss->done.push_back(ss->tag[__builtin_ctzll(x)]);
    ss->active &= ~ended;
    ss->dirty |= ended;
  }
  const int32_t k = (int32_t)std::min<size_t>((size_t)cap, ss->done.size());
  for (int32_t i = 0; i < k; ++i) done_tags[i] = ss->done[(size_t)i];
  ss->done.erase(ss->done.begin(), ss->done.begin() + k);
  *n_done = k;
  return DOBFS_OK;
}

int dobfs_session_counts(dobfs_session_t ss, int32_t* active, int32_t* pending, int64_t* levels) {
  if (!ss) return fail(DOBFS_EINVAL, "session is NULL");
  if (active) *active = __builtin_popcountll(ss->active);
  if (pending) *pending = (int32_t)ss->pending.size();
  if (levels) *levels = ss->levels;
  return DOBFS_OK;
}

int dobfs_session_levels(dobfs_session_t ss, dobfs_level_rec* recs, int32_t cap, int32_t* n) {
  if (!ss || !n || (cap > 0 && !recs)) return fail(DOBFS_EINVAL, "NULL argument");
  const int32_t k = (int32_t)std::min<size_t>((size_t)std::max(cap, 0), ss->last_log.size());
  for (int32_t i = 0; i < k; ++i) recs[i] = ss->last_log[(size_t)i];
  *n = k;
  return DOBFS_OK;
}

int dobfs_session_close(dobfs_session_t ss) {
  if (!ss) return DOBFS_OK;
  hipError_t e = hipStreamSynchronize(ss->stream);
  ss->w->busy = true;
  (void)hipEventRecord(ss->w->idle, ss->stream);
  release_workspace(ss->g, ss->w);
  {
    std::lock_guard<std::mutex> lk(ss->g->mu);
    --ss->g->open_sessions;
  }
  dfree(ss->slot_out);
  dfree(ss->slot_start);
  (void)hipHostFree(ss->host_ctl);
  (void)hipEventDestroy(ss->ev);
  delete ss;
  if (e != hipSuccess) return fail(DOBFS_EDEVICE, "session close", e);
  return DOBFS_OK;
}

}  // extern "C"
