// wave64 helpers for CDNA (gfx950): shuffles, ballots and block-level scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ovl {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// bits of lanes strictly below this lane
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  return v;
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint32_t lo = __shfl_xor((unsigned int)(v & 0xffffffffu), d, 64);
    uint32_t hi = __shfl_xor((unsigned int)(v >> 32), d, 64);
    v |= ((uint64_t)hi << 32) | lo;
  }
  return v;
}

// Sum over a block of BS threads.  lds holds BS/64 ints.  All threads get the total.
template <int BS>
__device__ __forceinline__ int block_sum(int v, int* lds) {
  v = wave_sum(v);
  if (lane_id() == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int i = 0; i < BS / 64; ++i) t += lds[i];
  __syncthreads();
  return t;
}

// Exclusive scan over a block of BS threads.  lds holds BS/64 ints.
template <int BS>
__device__ __forceinline__ int block_excl_scan(int v, int* lds, int& total) {
  int incl = wave_incl_scan(v);
  const int wid = threadIdx.x >> 6;
  if (lane_id() == 63) lds[wid] = incl;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < BS / 64; ++i) {
    int x = lds[i];
    pre += i < wid ? x : 0;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return pre + incl - v;
}

template <int BS>
__device__ __forceinline__ float block_max(float v, float* lds) {
  v = wave_max(v);
  if (lane_id() == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = lds[0];
#pragma unroll
  for (int i = 1; i < BS / 64; ++i) t = fmaxf(t, lds[i]);
  __syncthreads();
  return t;
}

// MurmurHash3 32-bit finaliser (Appleby, public domain): colouring priorities.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

}  // namespace ovl
