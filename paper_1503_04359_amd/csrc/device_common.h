/*
 * Wavefront and workgroup helpers shared by the traversal kernels (wave64,
 * gfx950).
 */
#ifndef DOBFS_DEVICE_COMMON_H
#define DOBFS_DEVICE_COMMON_H

#include <hip/hip_runtime.h>

#include "dobfs_internal.h"

namespace dobfs {
namespace {

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

/* Global wavefront index, made wave-uniform for the compiler so that
   values derived from it live in scalar registers. */
__device__ __forceinline__ int64_t wave_index() {
  return (int64_t)blockIdx.x * (blockDim.x / kWave) + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
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
  unsigned long long bits;  /* batched traversals: slots that found vertices */
};

__device__ __forceinline__ int64_t wave_sum(int64_t x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

template <class T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

/* End of a workgroup's share of a level kernel: its accumulators are summed
   and handed on, and the call returns true in every thread of the last
   workgroup to report.  `nblocks` workgroups report (0: the whole grid);
   with nblocks = 1 the caller is alone and nothing is counted.  Workgroups
   report to one of kGroups group slots (one cache line each) and the last
   of each group forwards the group's sums to the level counters, so no
   address sees more than gridDim/kGroups atomics.

   Every workgroup that reads a level's control state must report before
   the level can close: a workgroup that read the state and left without
   reporting could otherwise be overtaken by the close, and one dispatched
   after the close would read the next level's state inside this launch. */
template <int BT = kBlock>
__device__ bool finish_block_all(Ctl* c, Acc a, uint32_t nblocks = 0) {
  __shared__ int64_t part[4][BT / kWave];
  __shared__ unsigned long long bpart[BT / kWave];
  __shared__ int is_last;
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  for (int o = 32; o > 0; o >>= 1) a.bits |= __shfl_xor(a.bits, o);
  a.found = wave_sum(a.found);
  a.found_deg = wave_sum(a.found_deg);
  a.checked = wave_sum(a.checked);
  a.scanned = wave_sum(a.scanned);
  if (lane == 0) {
    part[0][wv] = a.found;
    part[1][wv] = a.found_deg;
    part[2][wv] = a.checked;
    part[3][wv] = a.scanned;
    bpart[wv] = a.bits;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t sum[4] = {0, 0, 0, 0};
    unsigned long long bits = 0ull;
    for (int k = 0; k < 4; ++k)
      for (int j = 0; j < BT / kWave; ++j) sum[k] += part[k][j];
    for (int j = 0; j < BT / kWave; ++j) bits |= bpart[j];
    const uint32_t nb = nblocks ? nblocks : gridDim.x; /* workgroups taking part */
    if (nb == 1) { /* alone: no other workgroup to wait for or to race with */
      c->nf_next += sum[0];
      c->mf_next += sum[1];
      c->checked += sum[2];
      c->scanned += sum[3];
      c->live_next |= bits;
      is_last = 1;
    } else {
      const uint32_t ng = nb < (uint32_t)kGroups ? nb : (uint32_t)kGroups;
      const uint32_t grp = blockIdx.x % ng;
      const uint32_t gsize = (nb - grp + ng - 1) / ng;
      GroupSlot& gs = c->grp[grp];
      for (int k = 0; k < 4; ++k)
        if (sum[k]) atomicAdd(reinterpret_cast<unsigned long long*>(&gs.sum[k]), (unsigned long long)sum[k]);
      if (bits) atomicOr(&gs.bits, bits);
      __threadfence();
      bool last = false;
      if (atomicAdd(&gs.ticket, 1u) == gsize - 1) {
        __threadfence();
        int64_t* tot[4] = {&c->nf_next, &c->mf_next, &c->checked, &c->scanned};
        for (int k = 0; k < 4; ++k) {
          const int64_t v = ld_agent(&gs.sum[k]);
          gs.sum[k] = 0;
          if (v) atomicAdd(reinterpret_cast<unsigned long long*>(tot[k]), (unsigned long long)v);
        }
        const unsigned long long gb = ld_agent(&gs.bits);
        gs.bits = 0ull;
        if (gb) atomicOr(&c->live_next, gb);
        gs.ticket = 0;
        __threadfence();
        last = atomicAdd(&c->ticket, 1u) == ng - 1;
        if (last) {
          c->ticket = 0;
          __threadfence();
        }
      }
      is_last = last;
    }
  }
  __syncthreads();
  return is_last != 0;
}

/* As finish_block_all, true in thread 0 of the last workgroup only. */
template <int BT = kBlock>
__device__ bool finish_block(Ctl* c, Acc a, uint32_t nblocks = 0) {
  const bool last = finish_block_all<BT>(c, a, nblocks);
  return threadIdx.x == 0 && last;
}

/* Completion groups and the grid ticket back to zero (one workgroup, before
   any level kernel of a traversal). */
__device__ __forceinline__ void reset_groups(Ctl* c) {
  for (int i = threadIdx.x; i < kGroups; i += blockDim.x) {
    GroupSlot& gs = c->grp[i];
    for (int k = 0; k < 4; ++k) gs.sum[k] = 0;
    gs.bits = 0ull;
    gs.ticket = 0u;
  }
  if (threadIdx.x == 0) c->ticket = 0u;
}

/* Inclusive prefix sum over the wavefront. */
__device__ __forceinline__ int wave_incl_scan(int x, int lane) {
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

/* Owner lane of concatenated position p (first lane whose inclusive end
   exceeds p; incl is non-decreasing across lanes). */
__device__ __forceinline__ int owner_of(int incl, int p) {
  int lo = 0;
  for (int step = kWave / 2; step > 0; step >>= 1)
    if (__shfl(incl, lo + step - 1) <= p) lo += step;
  return lo < kWave ? lo : kWave - 1;
}

}  // namespace
}  // namespace dobfs

#endif
