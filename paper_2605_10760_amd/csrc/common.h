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

// FP64 3D covariance Sigma = M M^T, M = R diag(s), of a Gaussian from its
// FP32 log-scales and (unnormalised) quaternion (w, x, y, z).  The scales,
// the normalised quaternion and the rotation are formed in FP32 (a ~1e-7
// relative perturbation of the parameters); the products, where elongated
// splats cancel, run in FP64.  The projection and its backward share this
// code, so the backward maps gradients through the very conic the forward
// rendered with.
__device__ __forceinline__ void cov3_fp64(const float* ls, const float* q, double Sd[3][3]) {
  const float sv[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
  const float qi = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const float qw = q[0] * qi, qx = q[1] * qi, qy = q[2] * qi, qz = q[3] * qi;
  const float R[3][3] = {{1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy)},
                         {2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx)},
                         {2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
  double M[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i][j] = (double)R[i][j] * (double)sv[j];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      Sd[i][j] = M[i][0] * M[j][0] + M[i][1] * M[j][1] + M[i][2] * M[j][2];
      Sd[j][i] = Sd[i][j];
    }
}

// FP64 camera-space mean p, its guard-clamped-free ratios (p_x/p_z, p_y/p_z)
// and the dilated 2D covariance [[a, b], [b, c]] = J (Rc Sigma Rc^T) J^T +
// 0.3 I of a Gaussian in one view (J at the guard-clamped ratios).
struct ScreenCov {
  double p[3];
  double rx, ry;
  double a, b, c;
};
__device__ __forceinline__ ScreenCov screen_cov_fp64(const double Sd[3][3], const float* Rc,
                                                     const float* tc, const float* m, float fxf,
                                                     float fyf, int W, int H) {
  ScreenCov o;
  double Wd[3][3], V[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k)
      Wd[i][k] = (double)Rc[3 * i] * Sd[0][k] + (double)Rc[3 * i + 1] * Sd[1][k] +
                 (double)Rc[3 * i + 2] * Sd[2][k];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      V[i][j] = Wd[i][0] * Rc[3 * j] + Wd[i][1] * Rc[3 * j + 1] + Wd[i][2] * Rc[3 * j + 2];
  for (int i = 0; i < 3; ++i)
    o.p[i] = (double)Rc[3 * i] * m[0] + (double)Rc[3 * i + 1] * m[1] +
             (double)Rc[3 * i + 2] * m[2] + (double)tc[i];
  const double fx = fxf, fy = fyf;
  const double ip2 = 1.0 / o.p[2];
  o.rx = o.p[0] * ip2;
  o.ry = o.p[1] * ip2;
  const double limx = 1.3 * (0.5 * W) / fx, limy = 1.3 * (0.5 * H) / fy;
  const double rxc = fmin(fmax(o.rx, -limx), limx), ryc = fmin(fmax(o.ry, -limy), limy);
  const double j00 = fx * ip2, j02 = -fx * rxc * ip2;
  const double j11 = fy * ip2, j12 = -fy * ryc * ip2;
  const double T00 = j00 * V[0][0] + j02 * V[2][0], T01 = j00 * V[0][1] + j02 * V[2][1];
  const double T02 = j00 * V[0][2] + j02 * V[2][2];
  const double T11 = j11 * V[1][1] + j12 * V[2][1], T12 = j11 * V[1][2] + j12 * V[2][2];
  o.a = T00 * j00 + T02 * j02 + 0.3;
  o.b = T01 * j11 + T02 * j12;
  o.c = T11 * j11 + T12 * j12 + 0.3;
  return o;
}

// Sum of x[0, n) (n a multiple of 4) over a workgroup of NT threads,
// returned in every thread: the carry of a multi-workgroup scan whose
// workgroup reads every element before its own tile (the tiles are few, so
// the redundant reads stay in L2).  Contains __syncthreads().
template <int NT>
__device__ __forceinline__ unsigned long long wg_sum_before(const uint32_t* x, int n,
                                                            unsigned long long* sh) {
  unsigned long long part = 0;
  for (int i = 4 * (int)threadIdx.x; i < n; i += 4 * NT) {
    const uint4 q = *reinterpret_cast<const uint4*>(x + i);
    part += (unsigned long long)q.x + q.y + q.z + q.w;
  }
  unsigned long long tot;
  (void)wg_excl_scan<NT>(part, sh, &tot);
  return tot;
}

}  // namespace gsr
