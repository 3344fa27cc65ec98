/*
 * Graph preparation kernels: degree summary and CSR validation.
 */
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dobfs_internal.h"

namespace dobfs {
namespace {

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

/* iso[w] bit i = (vertex 64w+i has degree 0 or lies beyond n).
   counters[0] += vertices of degree >= 1, counters[1] = max degree,
   counters[2] += vertices of degree > kMinHugeCut. */
__global__ void __launch_bounds__(kBlock) k_graph_scan(const int64_t* off, int64_t n, uint64_t* iso,
                                                     int64_t* counters) {
  const int lane = lane_id();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
  const int64_t words = (n + 63) / 64;
  int64_t nonisolated = 0, maxdeg = 0, huge = 0;
  for (int64_t wd = wave; wd < words; wd += nwaves) {
    const int64_t v = wd * kWave + lane;
    int64_t deg = 0;
    if (v < n) deg = off[v + 1] - off[v];
    const uint64_t empty = __ballot(deg == 0);
    if (lane == 0) iso[wd] = empty;
    nonisolated += deg > 0;
    huge += deg > kMinHugeCut;
    maxdeg = deg > maxdeg ? deg : maxdeg;
  }
  for (int o = 32; o > 0; o >>= 1) {
    nonisolated += __shfl_xor(nonisolated, o);
    huge += __shfl_xor(huge, o);
    const int64_t y = __shfl_xor(maxdeg, o);
    maxdeg = y > maxdeg ? y : maxdeg;
  }
  if (lane == 0) {
    if (nonisolated) atomicAdd(reinterpret_cast<unsigned long long*>(&counters[0]), (unsigned long long)nonisolated);
    atomicMax(reinterpret_cast<unsigned long long*>(&counters[1]), (unsigned long long)maxdeg);
    if (huge) atomicAdd(reinterpret_cast<unsigned long long*>(&counters[2]), (unsigned long long)huge);
  }
}

/* bad[0]: first problem found (0 none, 1 offsets, 2 index range,
   3 self-loop, 4 missing reverse edge). */
__global__ void __launch_bounds__(kBlock) k_validate_offsets(const int64_t* off, int64_t n, int64_t m, int32_t* bad) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0 && (off[0] != 0 || off[n] != m)) atomicCAS(bad, 0, 1);
  for (int64_t v = tid; v < n; v += nth) {
    const int64_t b = off[v], e = off[v + 1];
    if (b > e || b < 0 || e > m) atomicCAS(bad, 0, 1);
  }
}

/* Every neighbour ID in [0, n); run only once the offsets passed. */
__global__ void __launch_bounds__(kBlock) k_validate_indices(const int32_t* idx, int64_t n, int64_t m,
                                                           const int32_t* bad_in, int32_t* bad) {
  if (*bad_in) return;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += nth) {
    const int32_t u = idx[e];
    if (u < 0 || (int64_t)u >= n) atomicCAS(bad, 0, 2);
  }
}

/* No self-loop and every (v, u) has (u, v); rows sorted ascending. */
__global__ void __launch_bounds__(kBlock) k_validate_symmetry(const int64_t* off, const int32_t* idx, int64_t n,
                                                            int32_t* bad) {
  if (*bad) return;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += nth) {
    for (int64_t k = off[v]; k < off[v + 1]; ++k) {
      const int32_t u = idx[k];
      if ((int64_t)u == v) {
        atomicCAS(bad, 0, 3);
        break;
      }
      int64_t lo = off[u], hi = off[u + 1];
      bool ok = false;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t x = idx[mid];
        if (x == (int32_t)v) { ok = true; break; }
        if (x < (int32_t)v) lo = mid + 1; else hi = mid;
      }
      if (!ok) {
        atomicCAS(bad, 0, 4);
        break;
      }
    }
  }
}

/* first[v] = the first entry of v's row, -1 for degree 0. */
__global__ void __launch_bounds__(kBlock) k_first_column(const int64_t* off, const int32_t* idx, int64_t n,
                                                       int32_t* first) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += nth) {
    const int64_t b = off[v];
    first[v] = b < off[v + 1] ? idx[b] : -1;
  }
}

/* out[v] = caller ID of first[v] (relabelled graphs). */
__global__ void __launch_bounds__(kBlock) k_first_caller(const int32_t* first, const int32_t* new2old, int64_t n,
                                                       int32_t* out) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += nth) {
    const int32_t u = first[v];
    out[v] = u >= 0 ? new2old[u] : -1;
  }
}

__global__ void k_shift_i64(int64_t* dst, const int64_t* src, int64_t count, int64_t add) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += nth) dst[i] = src[i] + add;
}

__global__ void k_shift_i32(int32_t* dst, const int32_t* src, int64_t count, int32_t add) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += nth) dst[i] = src[i] + add;
}

}  // namespace

/* Graph i of a pack into the union CSR: offsets shifted by the entries
   before it, neighbour IDs by the vertices before it.  Host sources are
   staged through a device buffer. */
hipError_t launch_pack_copy(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int64_t nbase, int64_t mbase,
                            bool src_device, int64_t* uoff, int32_t* uidx, hipStream_t s) {
  const int64_t* doff = off;
  const int32_t* didx = idx;
  int64_t* t_off = nullptr;
  int32_t* t_idx = nullptr;
  hipError_t e = hipSuccess;
  if (!src_device) {
    if ((e = hipMalloc(&t_off, sizeof(int64_t) * (size_t)(n + 1))) != hipSuccess) return e;
    if ((e = hipMalloc(&t_idx, sizeof(int32_t) * (size_t)(m > 0 ? m : 1))) != hipSuccess) {
      (void)hipFree(t_off);
      return e;
    }
    if ((e = hipMemcpyAsync(t_off, off, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (m > 0 && (e = hipMemcpyAsync(t_idx, idx, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice, s)) != hipSuccess)) {
      (void)hipFree(t_off);
      (void)hipFree(t_idx);
      return e;
    }
    doff = t_off;
    didx = t_idx;
  }
  const unsigned blocks_o = (unsigned)std::min<int64_t>((n + 1 + 255) / 256, 4096);
  const unsigned blocks_i = (unsigned)std::min<int64_t>((m + 255) / 256 > 0 ? (m + 255) / 256 : 1, 4096);
  /* the last graph's offsets[n] lands on the union's offsets[N] */
  hipLaunchKernelGGL(k_shift_i64, dim3(blocks_o), dim3(256), 0, s, uoff + nbase, doff, n + 1, mbase);
  if (m > 0) hipLaunchKernelGGL(k_shift_i32, dim3(blocks_i), dim3(256), 0, s, uidx + mbase, didx, m, (int32_t)nbase);
  e = hipGetLastError();
  if (!src_device) {
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(t_off);
    (void)hipFree(t_idx);
    if (e == hipSuccess) e = e2;
  }
  return e;
}

hipError_t launch_first_caller(const int32_t* first, const int32_t* new2old, int64_t n, int32_t* out, int grid,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_first_caller, dim3(grid), dim3(kBlock), 0, s, first, new2old, n, out);
  return hipGetLastError();
}

hipError_t launch_first_column(const int64_t* off, const int32_t* idx, int64_t n, int32_t* first, int grid,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_first_column, dim3(grid), dim3(kBlock), 0, s, off, idx, n, first);
  return hipGetLastError();
}

hipError_t launch_graph_scan(const int64_t* off, int64_t n, uint64_t* iso, int64_t* counters, int grid,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_graph_scan, dim3(grid), dim3(kBlock), 0, s, off, n, iso, counters);
  return hipGetLastError();
}

hipError_t launch_validate(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int symmetry,
                           int32_t* bad, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_offsets, dim3(grid), dim3(kBlock), 0, s, off, n, m, bad);
  hipLaunchKernelGGL(k_validate_indices, dim3(grid), dim3(kBlock), 0, s, idx, n, m, bad, bad);
  if (symmetry) hipLaunchKernelGGL(k_validate_symmetry, dim3(grid), dim3(kBlock), 0, s, off, idx, n, bad);
  return hipGetLastError();
}

}  // namespace dobfs
