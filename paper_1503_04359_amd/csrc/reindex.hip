/*
 * Degree relabelling of a resident graph (locality optimisation of Section
 * 3.4, rethought for one GPU).
 *
 * Internal ID = rank of the vertex by degree class, highest first, ties by
 * caller ID.  The degree class of d >= 1 is its bit length (one class per
 * power of two); degree 0 is class 0.
 * Every adjacency list is rewritten in internal IDs and sorted ascending,
 * which puts neighbours of the highest degree class first (the order the
 * paper uses so that bottom-up scans stop early).  On the device this also
 *   - gathers the hubs into a short ID prefix, so the frontier-bitmap words
 *     probed most often stay in L2,
 *   - makes the vertices of one 64-vertex word similar in degree,
 *   - puts every degree-0 vertex in a suffix that bottom-up steps never
 *     visit,
 *   - keeps caller order inside each class, so mapping results back to
 *     caller IDs reads a few dozen sequential streams instead of random
 *     words.
 * Steps: stable radix sort of (max_class - class, ID) -> new2old; inverse ->
 * old2new; scan of permuted degrees -> offsets; rows copied and mapped
 * (short rows one wavefront each, rows above kLongRow cut into chunks spread
 * over all wavefronts); rows sorted in bounded batches with a segmented
 * radix sort over the ID bits.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include <rocprim/rocprim.hpp>

#include "dobfs_internal.h"

namespace dobfs {
namespace {

constexpr int64_t kLongRow = 4096;
constexpr int64_t kCopyChunk = 2048;
constexpr int64_t kSortBatch = 1ll << 28;  /* entries per segmented-sort batch */
constexpr int64_t kSortRows = 1ll << 24;   /* rows per segmented-sort batch */

struct DegreeOf {
  const int64_t* off;
  __device__ int64_t operator()(int64_t v) const { return off[v + 1] - off[v]; }
};

__device__ __forceinline__ int lane_of() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

__host__ __device__ inline uint32_t degree_class(int64_t d) {
  if (d <= 0) return 0u;
  int bl = 0;
  while (bl < 63 && ((int64_t)1 << bl) <= d) ++bl;  /* bit length */
  return (uint32_t)bl;
}

__global__ void k_sort_keys(const int64_t* off, int64_t n, uint32_t max_class, uint32_t* keys, int32_t* ids) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += nth) {
    keys[v] = max_class - degree_class(off[v + 1] - off[v]);
    ids[v] = (int32_t)v;
  }
}

__global__ void k_inverse_and_degrees(const int64_t* off, const int32_t* new2old, int64_t n, int32_t* old2new,
                                      uint32_t* deg_new) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += nth) {
    const int32_t o = new2old[i];
    old2new[o] = (int32_t)i;
    deg_new[i] = (uint32_t)(off[o + 1] - off[o]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) deg_new[n] = 0u;
}

__global__ void k_last_offset(int64_t* off_new, int64_t n, const uint32_t* deg_new) {
  if (blockIdx.x == 0 && threadIdx.x == 0) off_new[n] = off_new[n - 1] + (int64_t)deg_new[n - 1];
}

/* Rows [r0, n): one wavefront per row. */
__global__ void k_copy_rows(const int64_t* off, const int32_t* idx, const int64_t* off_new, const int32_t* new2old,
                            const int32_t* old2new, int64_t r0, int64_t n, int32_t* idx_new) {
  const int lane = lane_of();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / 64;
  for (int64_t i = r0 + wave; i < n; i += nwaves) {
    const int64_t dst = off_new[i], len = off_new[i + 1] - dst;
    if (len == 0) continue;
    const int64_t src = off[new2old[i]];
    for (int64_t k = lane; k < len; k += 64) idx_new[dst + k] = old2new[idx[src + k]];
  }
}

/* Rows [0, r1) (all longer than kCopyChunk): the flat entry range
   [0, off_new[r1]) cut into chunks, each chunk within at most two rows. */
__global__ void k_copy_long(const int64_t* off, const int32_t* idx, const int64_t* off_new, const int32_t* new2old,
                            const int32_t* old2new, int64_t r1, int32_t* idx_new) {
  const int lane = lane_of();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / 64;
  const int64_t total = off_new[r1];
  for (int64_t c0 = wave * kCopyChunk; c0 < total; c0 += nwaves * kCopyChunk) {
    int64_t lo = 0, hi = r1 - 1;  /* last row with off_new[row] <= c0 */
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (off_new[mid] <= c0) lo = mid; else hi = mid - 1;
    }
    const int64_t c1 = min(total, c0 + kCopyChunk);
    int64_t row = lo;
    for (int64_t e = c0 + lane; e < c1; e += 64) {
      int64_t r = row;
      while (off_new[r + 1] <= e) ++r;
      idx_new[e] = old2new[idx[off[new2old[r]] + (e - off_new[r])]];
    }
  }
}

/* Internal IDs where the degree class changes (classes are non-increasing
   along internal IDs, so each class is one contiguous range). */
__global__ void k_class_bounds(const int64_t* off_new, int64_t n, int32_t* count, int64_t* out, int cap) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += nth) {
    if (degree_class(off_new[v + 1] - off_new[v]) != degree_class(off_new[v] - off_new[v - 1])) {
      const int k = atomicAdd(count, 1);
      if (k < cap) out[k] = v;
    }
  }
}

__global__ void k_rel_offsets(const int64_t* off, int64_t r0, int64_t rows, uint32_t* rel) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= rows) rel[i] = (uint32_t)(off[r0 + i] - off[r0]);
}

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

struct Bufs {
  std::vector<void*> p;
  ~Bufs() {
    for (void* q : p) (void)hipFree(q);
  }
  template <class T>
  hipError_t get(T** out, int64_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(T) * (size_t)(count < 1 ? 1 : count));
    if (e == hipSuccess) {
      p.push_back(q);
      *out = static_cast<T*>(q);
    }
    return e;
  }
  void drop(void* q) {
    for (auto& x : p)
      if (x == q) {
        (void)hipFree(x);
        x = nullptr;
      }
  }
};

int status_of(hipError_t e) { return e == hipErrorOutOfMemory ? DOBFS_ENOMEM : DOBFS_EDEVICE; }

}  // namespace

int build_reindexed(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int grid, hipStream_t s,
                    int64_t** off_new_out, int32_t** idx_new_out, int32_t** new2old_out, int32_t** old2new_out,
                    int64_t** seg_lo_out, int32_t* nseg_out, std::string* err) {
  Bufs tmp;
  int64_t* seg_lo = nullptr;
  int64_t* off_new = nullptr;
  int32_t* idx_new = nullptr;
  int32_t* new2old = nullptr;
  int32_t* old2new = nullptr;
  auto fail = [&](const char* what, hipError_t e) {
    *err = std::string("relabel: ") + what + ": " + hipGetErrorString(e);
    (void)hipFree(off_new);
    (void)hipFree(idx_new);
    (void)hipFree(new2old);
    (void)hipFree(old2new);
    (void)hipFree(seg_lo);
    return status_of(e);
  };
#define RX(call, what)                        \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return fail(what, e_); \
  } while (0)

  /* max degree bounds the sort key */
  int64_t* d_max = nullptr;
  RX(tmp.get(&d_max, 1), "alloc");
  {
    size_t bytes = 0;
    auto deg_it = rocprim::make_transform_iterator(rocprim::make_counting_iterator<int64_t>(0), DegreeOf{off});
    RX(rocprim::reduce(nullptr, bytes, deg_it, d_max, (int64_t)0, (size_t)n, rocprim::maximum<int64_t>(), s),
       "max size");
    char* t = nullptr;
    RX(tmp.get(&t, (int64_t)bytes), "max temp");
    RX(rocprim::reduce(t, bytes, deg_it, d_max, (int64_t)0, (size_t)n, rocprim::maximum<int64_t>(), s), "max");
    tmp.drop(t);
  }
  int64_t max_deg = 0;
  RX(hipMemcpyAsync(&max_deg, d_max, sizeof(int64_t), hipMemcpyDeviceToHost, s), "max copy");
  RX(hipStreamSynchronize(s), "max sync");
  const uint32_t max_class = degree_class(max_deg);
  int bits = 1;
  while (bits < 32 && ((uint32_t)1 << bits) <= max_class) ++bits;

  /* new2old: stable sort by (max_class - class) over ascending IDs */
  RX(hipMalloc(&new2old, sizeof(int32_t) * (size_t)n), "new2old");
  {
    uint32_t *k_in = nullptr, *k_out = nullptr;
    int32_t* v_in = nullptr;
    RX(tmp.get(&k_in, n), "sort keys");
    RX(tmp.get(&k_out, n), "sort keys");
    RX(tmp.get(&v_in, n), "sort ids");
    hipLaunchKernelGGL(k_sort_keys, dim3(grid), dim3(kBlock), 0, s, off, n, max_class, k_in, v_in);
    RX(hipGetLastError(), "keys");
    size_t bytes = 0;
    RX(rocprim::radix_sort_pairs(nullptr, bytes, k_in, k_out, v_in, new2old, (size_t)n, 0u, (unsigned)bits, s),
       "sort size");
    char* t = nullptr;
    RX(tmp.get(&t, (int64_t)bytes), "sort temp");
    RX(rocprim::radix_sort_pairs(t, bytes, k_in, k_out, v_in, new2old, (size_t)n, 0u, (unsigned)bits, s), "sort");
    RX(hipStreamSynchronize(s), "sort sync");
    tmp.drop(t);
    tmp.drop(k_in);
    tmp.drop(k_out);
    tmp.drop(v_in);
  }

  /* old2new and the permuted degrees -> offsets */
  RX(hipMalloc(&old2new, sizeof(int32_t) * (size_t)n), "old2new");
  RX(hipMalloc(&off_new, sizeof(int64_t) * (size_t)(n + 1)), "offsets");
  {
    uint32_t* deg_new = nullptr;
    RX(tmp.get(&deg_new, n + 1), "degrees");
    hipLaunchKernelGGL(k_inverse_and_degrees, dim3(grid), dim3(kBlock), 0, s, off, new2old, n, old2new, deg_new);
    RX(hipGetLastError(), "inverse");
    size_t bytes = 0;
    RX(rocprim::exclusive_scan(nullptr, bytes, deg_new, off_new, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), s),
       "scan size");
    char* t = nullptr;
    RX(tmp.get(&t, (int64_t)bytes), "scan temp");
    RX(rocprim::exclusive_scan(t, bytes, deg_new, off_new, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), s),
       "scan");
    hipLaunchKernelGGL(k_last_offset, dim3(1), dim3(64), 0, s, off_new, n, deg_new);
    RX(hipStreamSynchronize(s), "scan sync");
    tmp.drop(t);
    tmp.drop(deg_new);
  }
  int64_t m_new = 0;
  RX(hipMemcpy(&m_new, off_new + n, sizeof(int64_t), hipMemcpyDeviceToHost), "m");
  if (m_new != m) return fail("entry count changed", hipErrorInvalidValue);

  /* rows copied in internal IDs */
  RX(hipMalloc(&idx_new, sizeof(int32_t) * (size_t)(m > 0 ? m : 1)), "indices");
  int64_t r_long = 0;  /* rows of a class above kLongRow's form a prefix; all longer than kCopyChunk */
  {
    const uint32_t long_class = degree_class(kLongRow);  /* classes above it have degree >= 2 * kLongRow */
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      int64_t o2[2];
      RX(hipMemcpy(o2, off_new + mid, sizeof(o2), hipMemcpyDeviceToHost), "bisect");
      if (degree_class(o2[1] - o2[0]) > long_class) lo = mid + 1; else hi = mid;
    }
    r_long = lo;
  }
  if (r_long > 0) {
    hipLaunchKernelGGL(k_copy_long, dim3(grid), dim3(kBlock), 0, s, off, idx, off_new, new2old, old2new, r_long,
                       idx_new);
    RX(hipGetLastError(), "copy long rows");
  }
  hipLaunchKernelGGL(k_copy_rows, dim3(grid), dim3(kBlock), 0, s, off, idx, off_new, new2old, old2new, r_long, n,
                     idx_new);
  RX(hipGetLastError(), "copy rows");
  RX(hipStreamSynchronize(s), "copy sync");

  /* rows sorted by internal ID, in batches of whole rows bounded in both
     entries and rows.  Rows of degree <= 1 (classes 0 and 1, a suffix)
     need no sorting. */
  int64_t n_sort = 0;
  {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      int64_t o2[2];
      RX(hipMemcpy(o2, off_new + mid, sizeof(o2), hipMemcpyDeviceToHost), "bisect");
      if (degree_class(o2[1] - o2[0]) > degree_class(1)) lo = mid + 1; else hi = mid;
    }
    n_sort = lo;
  }
  if (n_sort > 0) {
    int nbits = 1;
    while (nbits < 31 && ((int64_t)1 << nbits) < n) ++nbits;
    int64_t m_sort = 0;
    RX(hipMemcpy(&m_sort, off_new + n_sort, sizeof(int64_t), hipMemcpyDeviceToHost), "sorted entries");
    const int64_t nb = m_sort / kSortBatch + 1;
    int64_t* d_bounds = nullptr;
    RX(tmp.get(&d_bounds, nb), "bounds");
    hipLaunchKernelGGL(k_bounds, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, off_new, n_sort, kSortBatch,
                       nb, d_bounds);
    std::vector<int64_t> b((size_t)nb);
    RX(hipMemcpyAsync(b.data(), d_bounds, sizeof(int64_t) * (size_t)nb, hipMemcpyDeviceToHost, s), "bounds");
    RX(hipStreamSynchronize(s), "bounds");
    b[0] = 0;
    b.push_back(n_sort);
    std::vector<int64_t> rows;
    for (int64_t x : b) {
      if (!rows.empty() && x <= rows.back()) continue;
      while (!rows.empty() && x - rows.back() > kSortRows) rows.push_back(rows.back() + kSortRows);
      rows.push_back(x);
    }
    std::vector<int64_t> eo(rows.size());
    for (size_t i = 0; i < rows.size(); ++i)
      RX(hipMemcpy(&eo[i], off_new + rows[i], sizeof(int64_t), hipMemcpyDeviceToHost), "batch");
    int64_t max_e = 0, max_r = 0;
    for (size_t i = 0; i + 1 < rows.size(); ++i) {
      max_e = std::max(max_e, eo[i + 1] - eo[i]);
      max_r = std::max(max_r, rows[i + 1] - rows[i]);
    }
    if (max_e >= (int64_t)UINT32_MAX) return fail("sort batch too large", hipErrorInvalidValue);
    int32_t* buf = nullptr;
    uint32_t* rel = nullptr;
    RX(tmp.get(&buf, max_e), "sort buffer");
    RX(tmp.get(&rel, max_r + 1), "relative offsets");
    size_t bytes = 0;
    RX(rocprim::segmented_radix_sort_keys(nullptr, bytes, reinterpret_cast<uint32_t*>(idx_new),
                                          reinterpret_cast<uint32_t*>(buf), (unsigned)max_e, (unsigned)max_r, rel,
                                          rel + 1, 0u, (unsigned)nbits, s),
       "segmented sort size");
    char* t = nullptr;
    RX(tmp.get(&t, (int64_t)bytes), "segmented sort temp");
    for (size_t i = 0; i + 1 < rows.size(); ++i) {
      const int64_t r0 = rows[i], nr = rows[i + 1] - rows[i], e0 = eo[i], ne = eo[i + 1] - eo[i];
      if (ne <= 1) continue;
      hipLaunchKernelGGL(k_rel_offsets, dim3((unsigned)((nr + 1 + 255) / 256)), dim3(256), 0, s, off_new, r0, nr,
                         rel);
      size_t b2 = bytes;
      RX(rocprim::segmented_radix_sort_keys(t, b2, reinterpret_cast<uint32_t*>(idx_new + e0),
                                            reinterpret_cast<uint32_t*>(buf), (unsigned)ne, (unsigned)nr, rel,
                                            rel + 1, 0u, (unsigned)nbits, s),
         "segmented sort");
      RX(hipMemcpyAsync(idx_new + e0, buf, sizeof(int32_t) * (size_t)ne, hipMemcpyDeviceToDevice, s), "sort copy");
    }
    RX(hipStreamSynchronize(s), "sort sync");
  }
  /* degree-class segments of the internal ID space */
  {
    int32_t* d_cnt = nullptr;
    int64_t* d_b = nullptr;
    RX(tmp.get(&d_cnt, 1), "class bounds");
    RX(tmp.get(&d_b, kMaxSeg), "class bounds");
    RX(hipMemsetAsync(d_cnt, 0, sizeof(int32_t), s), "class bounds");
    hipLaunchKernelGGL(k_class_bounds, dim3(grid), dim3(kBlock), 0, s, off_new, n, d_cnt, d_b, kMaxSeg);
    int32_t cnt = 0;
    RX(hipMemcpyAsync(&cnt, d_cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s), "class bounds");
    RX(hipStreamSynchronize(s), "class bounds");
    if (cnt + 2 > kMaxSeg) return fail("too many degree classes", hipErrorInvalidValue);
    std::vector<int64_t> b((size_t)cnt);
    if (cnt) RX(hipMemcpy(b.data(), d_b, sizeof(int64_t) * (size_t)cnt, hipMemcpyDeviceToHost), "class bounds");
    std::sort(b.begin(), b.end());
    b.insert(b.begin(), 0);
    b.push_back(n);
    RX(hipMalloc(&seg_lo, sizeof(int64_t) * (size_t)kMaxSeg), "segments");
    RX(hipMemcpy(seg_lo, b.data(), sizeof(int64_t) * b.size(), hipMemcpyHostToDevice), "segments");
    *nseg_out = (int32_t)b.size() - 1;
  }
  *seg_lo_out = seg_lo;
  *off_new_out = off_new;
  *idx_new_out = idx_new;
  *new2old_out = new2old;
  *old2new_out = old2new;
  return DOBFS_OK;
#undef RX
}

}  // namespace dobfs
