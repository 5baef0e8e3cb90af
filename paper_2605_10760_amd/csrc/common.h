// Device helpers shared by the kernels: wave64 primitives, segment lookup,
// a single-workgroup scan.
#pragma once

#include "internal.h"

namespace gsr {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// The dispatcher hands workgroup b to XCD (b mod 8).  For a grid of
// 8 * ceil(n/8) workgroups this returns the logical index x*ceil(n/8) + b/8 so
// that every XCD (and its private L2) works through one contiguous eighth of
// the logical range in order; -1 for the surplus workgroups.  Neighbouring
// logical items (adjacent tiles, consecutive sort blocks or binning chunks)
// then share an L2: gathers of the same records hit, and partial-line writes
// to the same output runs merge before they reach HBM.
__host__ __device__ __forceinline__ int xcd_grid(int n) { return 8 * ((n + 7) / 8); }
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int per = (n + 7) / 8;
  const int l = (b & 7) * per + (b >> 3);
  return l < n ? l : -1;
}

// Index s with off[s] <= b < off[s+1] for a non-decreasing off[0..n].
__device__ __forceinline__ int find_seg(const int* off, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane_id() >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Sum over the 64 lanes of a wave (all lanes must be active), returned in
// every lane.  quad_perm [1,0,3,2], [2,3,0,1], row_half_mirror and row_mirror
// give every lane its 16-lane row sum; row_bcast:15 and row_bcast:31 carry
// the row sums up to the last row, whose lane 63 then holds the total.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
  return x + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                                           0, __builtin_bit_cast(int, x), CTRL, ROW_MASK, 0xF,
                                           false));
}
__device__ __forceinline__ float wave_total(float x) {
  x = dpp_add<0xB1, 0xF>(x);
  x = dpp_add<0x4E, 0xF>(x);
  x = dpp_add<0x141, 0xF>(x);
  x = dpp_add<0x140, 0xF>(x);
  x = dpp_add<0x142, 0xA>(x);
  x = dpp_add<0x143, 0xC>(x);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
}

// Exclusive prefix sum of x over a workgroup of NT threads (NT/64 waves).
// `sh` must hold NT/64 + 1 words of LDS.  Returns the prefix; *total gets
// the sum over the workgroup.  Contains __syncthreads().
template <int NT>
__device__ __forceinline__ unsigned long long wg_excl_scan(unsigned long long x,
                                                           unsigned long long* sh,
                                                           unsigned long long* total) {
  constexpr int NW = NT / 64;
  unsigned long long inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    unsigned long long y = __shfl_up(inc, d, 64);
    if (lane_id() >= d) inc += y;
  }
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) sh[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int i = 0; i < NW; ++i) {
      unsigned long long t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[NW] = run;
  }
  __syncthreads();
  unsigned long long r = sh[w] + inc - x;
  *total = sh[NW];
  __syncthreads();
  return r;
}

}  // namespace gsr
