/*
 * Device builder of the seeded Kronecker and Chung-Lu graphs, for sizes the
 * host builder cannot hold or builds slowly (Kronecker up to scale 30: ~34
 * billion directed entries; Chung-Lu with 100M core vertices).
 *
 * Produces exactly the CSR of the host builder (gg_cpu.cpp) for the same
 * parameters: the same counter-based edge stream (gg_rng.h), self-loops
 * dropped, both directions stored, each row sorted ascending and
 * de-duplicated.  Steps, all on one device:
 *   1. count    every generated edge adds 1 to the duplicate-including
 *               degree of both endpoints (atomics);
 *   2. scan     -> row starts of the duplicate-including CSR;
 *   3. fill     every edge is written into both rows at an atomic cursor;
 *   4. sort     rows are sorted in batches of whole rows (rocPRIM segmented
 *               radix sort over the ID bits only, into a bounded buffer),
 *               then de-duplicated back into their own row range;
 *   5. compact  unique counts are scanned into the final offsets and the
 *               rows are moved down in place, one bounded batch at a time
 *               through the same buffer (a batch's destination never
 *               reaches the next batch's source, since final offsets never
 *               exceed duplicate-including ones).
 * Peak device memory ~ 4*m_dup + 20*n bytes plus one batch buffer.
 *
 * Nothing here performs a breadth-first search.
 */
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>

#include <rocprim/rocprim.hpp>
#include <string>
#include <vector>

#include "gg_chunglu.h"
#include "gg_rng.h"

namespace {

thread_local std::string g_err;

constexpr int kBlock = 256;
constexpr int64_t kBatchEntries = 1ll << 30;  /* sort/compact batch bound */

int fail(const char* what, hipError_t e) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? -3 : -4;
}

#define GG_HIP(call, what)                        \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return fail(what, e_);  \
  } while (0)

struct KronParams {
  uint64_t key, pkey;
  gg_rmat_t t;
  int scale;
  int permute;
};

__device__ __forceinline__ void kron_edge(const KronParams& p, uint64_t k, uint32_t& u, uint32_t& v) {
  gg_rmat_edge(p.key, p.scale, p.t, k, &u, &v);
  if (p.permute) {
    u = gg_permute(p.pkey, p.scale, u);
    v = gg_permute(p.pkey, p.scale, v);
  }
}

/* Edge generators: edge k of the stream, both endpoints. */
struct KronGen {
  KronParams p;
  __device__ __forceinline__ void edge(uint64_t k, uint32_t& u, uint32_t& v) const { kron_edge(p, k, u, v); }
};

struct ClGen {
  gg_cl_core_t t;       /* alias table in device memory */
  int64_t m_core;
  const uint32_t* anchor;
  int64_t tail_len;
  __device__ __forceinline__ void edge(uint64_t k, uint32_t& u, uint32_t& v) const {
    gg_cl_edge(t, m_core, anchor, tail_len, (int64_t)k, &u, &v);
  }
};

template <class Gen>
__global__ void __launch_bounds__(kBlock) k_count(Gen gen, int64_t count, uint32_t* cnt) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += nth) {
    uint32_t u, v;
    gen.edge((uint64_t)k, u, v);
    if (u == v) continue;
    atomicAdd(&cnt[u], 1u);
    atomicAdd(&cnt[v], 1u);
  }
}

template <class Gen>
__global__ void __launch_bounds__(kBlock) k_fill(Gen gen, int64_t count, uint32_t* cur, const int64_t* off,
                                               int32_t* idx) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += nth) {
    uint32_t u, v;
    gen.edge((uint64_t)k, u, v);
    if (u == v) continue;
    const uint32_t pu = atomicAdd(&cur[u], 1u);
    const uint32_t pv = atomicAdd(&cur[v], 1u);
    idx[off[u] + pu] = (int32_t)v;
    idx[off[v] + pv] = (int32_t)u;
  }
}

/* Chung-Lu: marks the core vertices with a non-loop generated edge. */
__global__ void __launch_bounds__(kBlock) k_cl_marks(gg_cl_core_t t, int64_t m_core, uint8_t* has_edge) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m_core; k += nth) {
    uint32_t u, v;
    gg_cl_core_edge(t, k, &u, &v);
    if (u == v) continue;
    has_edge[u] = 1;
    has_edge[v] = 1;
  }
}

/* First row r in [0, n] with off[r] >= target, for each target j*B. */
__global__ void k_bounds(const int64_t* off, int64_t n, int64_t step, int64_t nb, int64_t* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb) return;
  const int64_t target = j * step;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] < target) lo = mid + 1; else hi = mid;
  }
  out[j] = lo;
}

__global__ void k_rel_offsets(const int64_t* off, int64_t r0, int64_t rows, uint32_t* rel) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= rows) rel[i] = (uint32_t)(off[r0 + i] - off[r0]);
}

/* One wavefront per row: copy the sorted row from tmp back to the row's own
   range without repeats; ucnt[r] = number kept. */
__global__ void __launch_bounds__(kBlock) k_unique(const int64_t* off, int64_t r0, int64_t r1, const int32_t* tmp,
                                                 int32_t* idx, uint32_t* ucnt) {
  const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / 64;
  const int64_t base = off[r0];
  for (int64_t r = r0 + wave; r < r1; r += nwaves) {
    const int64_t b = off[r], e = off[r + 1];
    int64_t kept = 0;
    for (int64_t k0 = b; k0 < e; k0 += 64) {
      const int64_t k = k0 + lane;
      bool keep = false;
      int32_t x = 0;
      if (k < e) {
        x = tmp[k - base];
        keep = (k == b) || (tmp[k - 1 - base] != x);
      }
      const uint64_t m = __ballot(keep);
      const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
      if (keep) idx[b + kept + rank] = x;
      kept += __popcll(m);
    }
    if (lane == 0) ucnt[r] = (uint32_t)kept;
  }
}

/* Rows [r0, r1): unique entries from their duplicate-including start into
   tmp at their final position relative to off_new[r0]. */
__global__ void __launch_bounds__(kBlock) k_gather_rows(const int64_t* off_dup, const int64_t* off_new, int64_t r0,
                                                      int64_t r1, const int32_t* idx, int32_t* tmp) {
  const int lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / 64;
  const int64_t base = off_new[r0];
  for (int64_t r = r0 + wave; r < r1; r += nwaves) {
    const int64_t src = off_dup[r], dst = off_new[r] - base, len = off_new[r + 1] - off_new[r];
    for (int64_t k = lane; k < len; k += 64) tmp[dst + k] = idx[src + k];
  }
}

__global__ void k_set_last(int64_t* off, int64_t n, const uint32_t* cnt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) off[n] = off[n - 1] + (int64_t)cnt[n - 1];
}

int grid_for(int64_t work) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int64_t g = (work + kBlock - 1) / kBlock;
  const int64_t cap = (int64_t)cus * 16;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

/* offsets[0..n] = exclusive scan of cnt[0..n-1] (uint32 -> int64). */
int scan_counts(const uint32_t* cnt, int64_t n, int64_t* off, hipStream_t s) {
  size_t bytes = 0;
  GG_HIP(rocprim::exclusive_scan(nullptr, bytes, cnt, off, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), s),
         "scan size");
  void* tmp = nullptr;
  GG_HIP(hipMalloc(&tmp, bytes ? bytes : 1), "scan temp");
  hipError_t e = rocprim::exclusive_scan(tmp, bytes, cnt, off, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_set_last, dim3(1), dim3(64), 0, s, off, n, cnt);
    e = hipStreamSynchronize(s);
  }
  (void)hipFree(tmp);
  if (e != hipSuccess) return fail("scan", e);
  return 0;
}

/* Row batch starts: rows whose entries begin at or after j*step. */
int batch_bounds(const int64_t* off, int64_t n, int64_t total, int64_t step, std::vector<int64_t>& bounds,
                 hipStream_t s) {
  const int64_t nb = total / step + 1;
  int64_t* d = nullptr;
  GG_HIP(hipMalloc(&d, sizeof(int64_t) * (size_t)nb), "bounds alloc");
  hipLaunchKernelGGL(k_bounds, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, off, n, step, nb, d);
  bounds.assign((size_t)nb, 0);
  hipError_t e = hipMemcpyAsync(bounds.data(), d, sizeof(int64_t) * (size_t)nb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  if (e != hipSuccess) return fail("bounds", e);
  bounds[0] = 0;
  bounds.push_back(n);
  std::vector<int64_t> uniq;
  for (int64_t b : bounds)
    if (uniq.empty() || b > uniq.back()) uniq.push_back(b);
  if (uniq.back() != n) uniq.push_back(n);
  bounds.swap(uniq);
  return 0;
}

/* The CSR of `count` generated edges over n vertices (IDs below 2^bits). */
template <class Gen>
int build_csr_dev(const Gen& gen, int64_t n, int64_t count, int bits, int64_t** out_off, int32_t** out_idx,
                  int64_t* out_m, hipStream_t s) {
  uint32_t* cnt = nullptr;
  int64_t* off_dup = nullptr;
  int64_t* off = nullptr;
  int32_t* idx = nullptr;
  int32_t* tmp = nullptr;
  uint32_t* rel = nullptr;
  void* sort_tmp = nullptr;
  int rc = 0;
  auto cleanup = [&](int status) {
    (void)hipFree(cnt);
    (void)hipFree(off_dup);
    (void)hipFree(tmp);
    (void)hipFree(rel);
    (void)hipFree(sort_tmp);
    if (status) {
      (void)hipFree(off);
      (void)hipFree(idx);
    }
    return status;
  };
#define GG_TRY(call, what)                                     \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return cleanup(fail(what, e_));      \
  } while (0)

  GG_TRY(hipMalloc(&cnt, sizeof(uint32_t) * (size_t)(n + 1)), "counts");
  GG_TRY(hipMalloc(&off_dup, sizeof(int64_t) * (size_t)(n + 1)), "offsets");
  GG_TRY(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (size_t)(n + 1), s), "memset");
  hipLaunchKernelGGL(k_count<Gen>, dim3(grid_for(count)), dim3(kBlock), 0, s, gen, count, cnt);
  GG_TRY(hipGetLastError(), "count");
  if ((rc = scan_counts(cnt, n, off_dup, s))) return cleanup(rc);
  int64_t m_dup = 0;
  GG_TRY(hipMemcpy(&m_dup, off_dup + n, sizeof(int64_t), hipMemcpyDeviceToHost), "m_dup");
  GG_TRY(hipMalloc(&idx, sizeof(int32_t) * (size_t)(m_dup > 0 ? m_dup : 1)), "indices");
  GG_TRY(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (size_t)(n + 1), s), "memset");
  hipLaunchKernelGGL(k_fill<Gen>, dim3(grid_for(count)), dim3(kBlock), 0, s, gen, count, cnt, off_dup, idx);
  GG_TRY(hipGetLastError(), "fill");

  /* 4. sort + de-duplicate in batches of whole rows. */
  std::vector<int64_t> bounds;
  if ((rc = batch_bounds(off_dup, n, m_dup, kBatchEntries, bounds, s))) return cleanup(rc);
  int64_t max_batch = 0, max_rows = 0;
  {
    std::vector<int64_t> ob(bounds.size());
    for (size_t i = 0; i < bounds.size(); ++i)
      GG_TRY(hipMemcpy(&ob[i], off_dup + bounds[i], sizeof(int64_t), hipMemcpyDeviceToHost), "bounds");
    for (size_t i = 0; i + 1 < bounds.size(); ++i) {
      max_batch = std::max(max_batch, ob[i + 1] - ob[i]);
      max_rows = std::max(max_rows, bounds[i + 1] - bounds[i]);
    }
    if (max_batch >= (int64_t)UINT32_MAX) return cleanup(fail("row batch too large", hipErrorInvalidValue));
  }
  GG_TRY(hipMalloc(&tmp, sizeof(int32_t) * (size_t)(max_batch > 0 ? max_batch : 1)), "batch buffer");
  GG_TRY(hipMalloc(&rel, sizeof(uint32_t) * (size_t)(max_rows + 1)), "relative offsets");
  size_t sort_bytes = 0;
  {
    GG_TRY(rocprim::segmented_radix_sort_keys(nullptr, sort_bytes, reinterpret_cast<uint32_t*>(idx),
                                              reinterpret_cast<uint32_t*>(tmp), (unsigned int)max_batch,
                                              (unsigned int)max_rows, rel, rel + 1, 0, bits, s),
           "sort size");
    GG_TRY(hipMalloc(&sort_tmp, sort_bytes ? sort_bytes : 1), "sort temp");
    for (size_t i = 0; i + 1 < bounds.size(); ++i) {
      const int64_t r0 = bounds[i], r1 = bounds[i + 1], rows = r1 - r0;
      int64_t b0 = 0, b1 = 0;
      GG_TRY(hipMemcpyAsync(&b0, off_dup + r0, sizeof(int64_t), hipMemcpyDeviceToHost, s), "batch");
      GG_TRY(hipMemcpyAsync(&b1, off_dup + r1, sizeof(int64_t), hipMemcpyDeviceToHost, s), "batch");
      GG_TRY(hipStreamSynchronize(s), "batch");
      if (rows == 0) continue;
      hipLaunchKernelGGL(k_rel_offsets, dim3((unsigned)((rows + 1 + 255) / 256)), dim3(256), 0, s, off_dup, r0,
                         rows, rel);
      if (b1 > b0) {
        size_t bytes = sort_bytes;
        GG_TRY(rocprim::segmented_radix_sort_keys(sort_tmp, bytes, reinterpret_cast<uint32_t*>(idx + b0),
                                                  reinterpret_cast<uint32_t*>(tmp), (unsigned int)(b1 - b0),
                                                  (unsigned int)rows, rel, rel + 1, 0, bits, s),
               "segmented sort");
      }
      hipLaunchKernelGGL(k_unique, dim3(grid_for(rows * 64)), dim3(kBlock), 0, s, off_dup, r0, r1, tmp, idx, cnt);
      GG_TRY(hipGetLastError(), "unique");
    }
  }
  (void)hipFree(sort_tmp);
  sort_tmp = nullptr;
  (void)hipFree(rel);
  rel = nullptr;

  /* 5. final offsets and in-place compaction. */
  GG_TRY(hipMalloc(&off, sizeof(int64_t) * (size_t)(n + 1)), "final offsets");
  if ((rc = scan_counts(cnt, n, off, s))) return cleanup(rc);
  int64_t m = 0;
  GG_TRY(hipMemcpy(&m, off + n, sizeof(int64_t), hipMemcpyDeviceToHost), "m");
  /* The sort batches hold at most max_batch entries with duplicates, so
     their unique entries fit the same buffer. */
  for (size_t i = 0; i + 1 < bounds.size(); ++i) {
    const int64_t r0 = bounds[i], r1 = bounds[i + 1];
    int64_t d0 = 0, d1 = 0;
    GG_TRY(hipMemcpyAsync(&d0, off + r0, sizeof(int64_t), hipMemcpyDeviceToHost, s), "compact");
    GG_TRY(hipMemcpyAsync(&d1, off + r1, sizeof(int64_t), hipMemcpyDeviceToHost, s), "compact");
    GG_TRY(hipStreamSynchronize(s), "compact");
    if (d1 <= d0) continue;
    if (d1 - d0 > max_batch) return cleanup(fail("compaction batch too large", hipErrorInvalidValue));
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for((r1 - r0) * 64)), dim3(kBlock), 0, s, off_dup, off, r0, r1,
                       idx, tmp);
    GG_TRY(hipGetLastError(), "gather");
    GG_TRY(hipMemcpyAsync(idx + d0, tmp, sizeof(int32_t) * (size_t)(d1 - d0), hipMemcpyDeviceToDevice, s),
           "compact copy");
  }
  GG_TRY(hipStreamSynchronize(s), "build");
  *out_off = off;
  *out_idx = idx;
  *out_m = m;
  return cleanup(0);
#undef GG_TRY
}

}  // namespace

extern "C" {

/* Kronecker graph built on the current device.  *offsets (int64[n+1]) and
   *indices (int32, at least m entries) are device allocations released with
   ggd_free.  Returns 0, or -1 (arguments), -3 (out of memory), -4 (device). */
int ggd_kronecker(int scale, int edgefactor, uint64_t seed, const uint32_t thresholds[3], int permute,
                  int64_t** offsets, int32_t** indices, int64_t* n_out, int64_t* m_out, void* stream) {
  g_err.clear();
  if (scale < 1 || scale > 30 || edgefactor < 1 || !thresholds || !offsets || !indices || !n_out || !m_out)
    return -1;
  KronParams p;
  p.key = gg_stream_key(seed, GG_STREAM_EDGES);
  p.pkey = gg_stream_key(seed, GG_STREAM_PERM);
  p.t.a = thresholds[0];
  p.t.ab = thresholds[1];
  p.t.abc = thresholds[2];
  p.scale = scale;
  p.permute = permute;
  const int64_t n = (int64_t)1 << scale;
  const int64_t count = (int64_t)edgefactor << scale;
  *n_out = n;
  KronGen gen;
  gen.p = p;
  return build_csr_dev(gen, n, count, scale, offsets, indices, m_out, reinterpret_cast<hipStream_t>(stream));
}

/* Chung-Lu graph with path tails built on the current device: the graph of
   the host builder's gg_chung_lu for the same arguments.  The alias table
   and the tail anchors are computed on the host (sequential, as there);
   the marks that the anchors need and every edge are generated on the
   device.  Outputs and status as for ggd_kronecker (-2: no anchor). */
int ggd_chung_lu(int64_t n_core, double gamma, double avg_deg, double max_deg, int32_t n_tails, int32_t tail_len,
                 uint64_t seed, int64_t** offsets, int32_t** indices, int64_t* n_out, int64_t* m_out, void* stream) {
  g_err.clear();
  if (n_core < 2 || n_tails < 0 || tail_len < 0 || !offsets || !indices || !n_out || !m_out) return -1;
  const int64_t n = n_core + (int64_t)n_tails * tail_len;
  if (n > 2147483647LL) return -1;
  double i0, c;
  if (gg_cl_weights(n_core, gamma, avg_deg, max_deg, &i0, &c)) return -1;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<uint32_t> thr;
  std::vector<int32_t> alias;
  gg_cl_alias(n_core, i0, c, 1.0 / (gamma - 1.0), thr, alias);
  const int64_t m_core = (int64_t)std::llround((double)n_core * avg_deg / 2.0);
  uint32_t* d_thr = nullptr;
  int32_t* d_alias = nullptr;
  uint32_t* d_anchor = nullptr;
  uint8_t* d_marks = nullptr;
  auto done = [&](int status) {
    (void)hipFree(d_thr);
    (void)hipFree(d_alias);
    (void)hipFree(d_anchor);
    (void)hipFree(d_marks);
    return status;
  };
#define GG_TRY(call, what)                                     \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return done(fail(what, e_));         \
  } while (0)
  GG_TRY(hipMalloc(&d_thr, sizeof(uint32_t) * (size_t)n_core), "alias table");
  GG_TRY(hipMalloc(&d_alias, sizeof(int32_t) * (size_t)n_core), "alias table");
  GG_TRY(hipMemcpyAsync(d_thr, thr.data(), sizeof(uint32_t) * (size_t)n_core, hipMemcpyHostToDevice, s), "table copy");
  GG_TRY(hipMemcpyAsync(d_alias, alias.data(), sizeof(int32_t) * (size_t)n_core, hipMemcpyHostToDevice, s),
         "table copy");
  gg_cl_core_t t;
  t.key = gg_stream_key(seed, GG_STREAM_CL_EDGES);
  t.pkey = gg_stream_key(seed, GG_STREAM_PERM);
  t.n_core = n_core;
  t.pbits = gg_bits_for((uint64_t)n_core);
  t.pad = 0;
  t.thr = d_thr;
  t.alias = d_alias;
  std::vector<uint32_t> anchor((size_t)std::max<int32_t>(n_tails, 1), 0u);
  if (n_tails > 0 && tail_len > 0) {
    GG_TRY(hipMalloc(&d_marks, (size_t)n_core), "marks");
    GG_TRY(hipMemsetAsync(d_marks, 0, (size_t)n_core, s), "marks");
    hipLaunchKernelGGL(k_cl_marks, dim3(grid_for(m_core)), dim3(kBlock), 0, s, t, m_core, d_marks);
    GG_TRY(hipGetLastError(), "marks");
    std::vector<uint8_t> marks((size_t)n_core);
    GG_TRY(hipMemcpyAsync(marks.data(), d_marks, (size_t)n_core, hipMemcpyDeviceToHost, s), "marks copy");
    GG_TRY(hipStreamSynchronize(s), "marks");
    if (gg_cl_anchors(n_core, seed, n_tails, marks.data(), anchor.data())) return done(-2);
  }
  GG_TRY(hipMalloc(&d_anchor, sizeof(uint32_t) * anchor.size()), "anchors");
  GG_TRY(hipMemcpyAsync(d_anchor, anchor.data(), sizeof(uint32_t) * anchor.size(), hipMemcpyHostToDevice, s),
         "anchors");
  GG_TRY(hipStreamSynchronize(s), "anchors");
#undef GG_TRY
  ClGen gen;
  gen.t = t;
  gen.m_core = m_core;
  gen.anchor = d_anchor;
  gen.tail_len = tail_len;
  const int64_t count = m_core + (tail_len > 0 ? (int64_t)n_tails * tail_len : 0);
  *n_out = n;
  return done(build_csr_dev(gen, n, count, gg_bits_for((uint64_t)n), offsets, indices, m_out, s));
}

void ggd_free(void* p) {
  if (p) (void)hipFree(p);
}

const char* ggd_last_error(void) { return g_err.c_str(); }

}  // extern "C"
