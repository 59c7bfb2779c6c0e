// Device helpers shared by the CPAA kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace cpaa {

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  With remapping, the workgroups that land on one XCD take
// one contiguous range of logical work items, so neighbouring rows (and the
// vector entries they gather) stay in one L2.  Bijective for any total.
__device__ __forceinline__ int xcd_logical(int b, int total, int remap) {
  if (!remap) return b;
  const int x = b & 7, i = b >> 3;
  const int q = total >> 3, r = total & 7;
  return x * q + (x < r ? x : r) + i;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Sum over a 256-thread workgroup; the result is valid in thread 0.
// Every thread of the block must call it (it contains barriers).
__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double red[4];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (threadIdx.x == 0) ? (red[0] + red[1]) + (red[2] + red[3]) : 0.0;
}

__device__ __forceinline__ double block_max256(double v) {
  __shared__ double red[4];
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (threadIdx.x == 0) ? fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) : 0.0;
}

// max of non-negative doubles through the integer ordering of their bits
__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr),
            static_cast<unsigned long long>(__double_as_longlong(v)));
}

__device__ __forceinline__ void atomic_add(double* addr, double v) { unsafeAtomicAdd(addr, v); }
__device__ __forceinline__ void atomic_add(float* addr, float v) { unsafeAtomicAdd(addr, v); }

// Split-row protocols (a row's chunks on several workgroups) exchange their
// partial sums only through device-scope atomics and count arrivals with one
// more atomic.  All that is needed between the two is that this wave's data
// atomics have been performed before its counter atomic is issued: wait for
// every outstanding memory operation, and keep the compiler from moving
// memory operations across the wait.  An agent-scope fence (__threadfence)
// would also write back and invalidate the XCD's whole L2 on this chip,
// which made the tiled term on a power-law graph 2.3x slower.
__device__ __forceinline__ void atomics_done() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Deterministic sum of per-block values over a grid (deterministic plans):
// thread 0 of every block publishes its Q values v (the block's own sums) to
// part[q * nblocks + block]; the last block to count itself in adds them in
// block order (a fixed strided split over its threads, then a fixed tree) and
// returns true, with the grid totals in v of its thread 0.  Every thread of
// every block of the grid calls it once; *counter is zero on entry and is left
// zero.  The values travel through device-scope atomic stores and loads after
// the wave's stores have completed, as in the split-row protocol.
template <int Q>
__device__ __forceinline__ bool ordered_block_sum(double (&v)[Q], int block, int nblocks,
                                                  double* part, int* counter) {
  __shared__ int last;
  if (threadIdx.x == 0) {
    for (int q = 0; q < Q; ++q)
      __hip_atomic_store(&part[static_cast<size_t>(q) * nblocks + block], v[q], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    atomics_done();
    last = atomicAdd(counter, 1) == nblocks - 1 ? 1 : 0;
  }
  __syncthreads();
  if (!last) return false;
  atomics_done();
  for (int q = 0; q < Q; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
      s += __hip_atomic_load(&part[static_cast<size_t>(q) * nblocks + b], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    s = block_sum256(s);
    if (threadIdx.x == 0) v[q] = s;
  }
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

__device__ __forceinline__ int prev_pow2(int v) {
  return v <= 1 ? 1 : (1 << (31 - __clz(v)));
}

}  // namespace cpaa
