// Refinement extras of the fused map (Sec. III-C, Eq. (refine_loss)): the
// gradient of the L1 terms on the exposure-compensated render
// I~ = exp(a_k) I^ + b_k, and opacity pruning.
//
// k_l1_grad: a few blocks per view stride over its pixels (a block never
// spans two views): reads the three colour planes, the depth and the targets
// once and writes their gradients once (HBM-bound, 48 B per pixel); the
// per-view sums for (a_k, b_k) are a DPP wave sum, an LDS sum over the
// block's waves and one atomic per block.
// k_prune_*: ordered stream compaction (per-block counts, one-workgroup scan,
// wave-ballot ranks) of the Gaussians whose logit is at least the FP32
// threshold, then a row gather of every parameter array.
#include <algorithm>

#include "common.h"

namespace gsr {

__global__ __launch_bounds__(256) void k_zero_f32(float* p, int n) {
  for (int i = threadIdx.x; i < n; i += 256) p[i] = 0.f;
}

// A view's pixels are spread over blocks_per_view blocks that stride through
// them, so the exposure sums take few atomics per view.  Pixels go four at a
// time (16-byte loads and stores) when the plane size and every pointer
// allow it, one at a time otherwise.
__device__ __forceinline__ float l1_sign(float e, float w) {
  return e > 0.f ? w : (e < 0.f ? -w : 0.f);
}

template <bool VEC>
__global__ __launch_bounds__(256) void k_l1_grad(int HW, int blocks_per_view, const float* color,
                                                 const float* depth, const float* tcol,
                                                 const float* tdep, const float* expo,
                                                 float w_col, float w_dep, float* g_col,
                                                 float* g_dep, float* g_expo) {
  __shared__ float red[2][4];
  const int v = blockIdx.x / blocks_per_view;
  const int b0 = blockIdx.x - v * blocks_per_view;
  const float a = expo ? expo[2 * v] : 0.f, b = expo ? expo[2 * v + 1] : 0.f;
  const float ea = expf(a);
  float sa = 0.f, sb = 0.f;
  if (VEC) {
    const int n4 = HW / 4;
    for (int p = b0 * 256 + (int)threadIdx.x; p < n4; p += blocks_per_view * 256) {
      const size_t base = (size_t)v * 3 * HW + 4 * (size_t)p;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float4 c = *reinterpret_cast<const float4*>(color + base + (size_t)ch * HW);
        const float4 t = *reinterpret_cast<const float4*>(tcol + base + (size_t)ch * HW);
        const float4 g = make_float4(l1_sign(ea * c.x + b - t.x, w_col),
                                     l1_sign(ea * c.y + b - t.y, w_col),
                                     l1_sign(ea * c.z + b - t.z, w_col),
                                     l1_sign(ea * c.w + b - t.w, w_col));
        *reinterpret_cast<float4*>(g_col + base + (size_t)ch * HW) =
            make_float4(ea * g.x, ea * g.y, ea * g.z, ea * g.w);
        sa += c.x * g.x + c.y * g.y + c.z * g.z + c.w * g.w;
        sb += g.x + g.y + g.z + g.w;
      }
      if (g_dep) {
        const size_t q = (size_t)v * HW + 4 * (size_t)p;
        const float4 d = *reinterpret_cast<const float4*>(depth + q);
        const float4 t = *reinterpret_cast<const float4*>(tdep + q);
        *reinterpret_cast<float4*>(g_dep + q) =
            make_float4(l1_sign(d.x - t.x, w_dep), l1_sign(d.y - t.y, w_dep),
                        l1_sign(d.z - t.z, w_dep), l1_sign(d.w - t.w, w_dep));
      }
    }
  } else {
    for (int p = b0 * 256 + (int)threadIdx.x; p < HW; p += blocks_per_view * 256) {
      const size_t base = (size_t)v * 3 * HW + p;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float c = color[base + (size_t)ch * HW];
        const float g = l1_sign(ea * c + b - tcol[base + (size_t)ch * HW], w_col);
        g_col[base + (size_t)ch * HW] = ea * g;
        sa += c * g;
        sb += g;
      }
      if (g_dep) {
        const size_t q = (size_t)v * HW + p;
        g_dep[q] = l1_sign(depth[q] - tdep[q], w_dep);
      }
    }
  }
  if (!g_expo) return;  // uniform
  sa = wave_total(sa);
  sb = wave_total(sb);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    red[0][w] = sa;
    red[1][w] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(&g_expo[2 * v], ea * (red[0][0] + red[0][1] + red[0][2] + red[0][3]));
    atomicAdd(&g_expo[2 * v + 1], red[1][0] + red[1][1] + red[1][2] + red[1][3]);
  }
}

hipError_t launch_l1_grad(int nv, int HW, const float* color, const float* depth,
                          const float* tcol, const float* tdep, const float* expo, float w_col,
                          float w_dep, float* g_col, float* g_dep, float* g_expo, hipStream_t s) {
  if (g_expo) hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(256), 0, s, g_expo, 2 * nv);
  const uintptr_t al = (uintptr_t)color | (uintptr_t)tcol | (uintptr_t)g_col |
                       (g_dep ? ((uintptr_t)depth | (uintptr_t)tdep | (uintptr_t)g_dep) : 0);
  const bool vec = HW % 4 == 0 && (al & 15) == 0;
  // about one pixel group per thread across the batch (every load of the
  // kernel in flight at once); with exposure sums, fewer blocks per view
  // (each adds to the view's two sums with one atomic apiece)
  const int per = vec ? HW / 4 : HW;
  const int bpv = std::min((per + 255) / 256, std::max(64, (g_expo ? 2048 : 16384) / nv));
  if (vec)
    hipLaunchKernelGGL(k_l1_grad<true>, dim3(nv * bpv), dim3(256), 0, s, HW, bpv, color, depth,
                       tcol, tdep, expo, w_col, w_dep, g_col, g_dep, g_expo);
  else
    hipLaunchKernelGGL(k_l1_grad<false>, dim3(nv * bpv), dim3(256), 0, s, HW, bpv, color, depth,
                       tcol, tdep, expo, w_col, w_dep, g_col, g_dep, g_expo);
  return hipGetLastError();
}

// ------------------------------------------------------------------ pruning
__global__ __launch_bounds__(256) void k_prune_count(long n, const float* opac, float thr,
                                                     uint32_t* blk) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const bool keep = i < n && opac[i] >= thr;
  const int c = __syncthreads_count(keep);
  if (threadIdx.x == 0) blk[blockIdx.x] = (uint32_t)c;
}

// One workgroup: exclusive scan of the block counts, in place; total at blk[nb].
__global__ __launch_bounds__(1024) void k_prune_scan(int nb, uint32_t* blk) {
  __shared__ unsigned long long sh[17];
  unsigned long long carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + (int)threadIdx.x;
    const uint32_t x = i < nb ? blk[i] : 0u;
    unsigned long long tot;
    const unsigned long long pre = wg_excl_scan<1024>(x, sh, &tot) + carry;
    if (i < nb) blk[i] = (uint32_t)pre;
    carry += tot;
  }
  if (threadIdx.x == 0) blk[nb] = (uint32_t)carry;
}

hipError_t launch_block_scan(int nb, uint32_t* blk, hipStream_t s) {
  hipLaunchKernelGGL(k_prune_scan, dim3(1), dim3(1024), 0, s, nb, blk);
  return hipGetLastError();
}

// Kept count before each set boundary (one thread per boundary).
__global__ void k_prune_bounds(SimSetTab tab, const float* opac, float thr, const uint32_t* blk,
                               long long* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > tab.ns) return;
  const long e = tab.off[k];
  const long b = e / 256;
  uint32_t c = blk[b];
  for (long i = b * 256; i < e; ++i) c += opac[i] >= thr ? 1u : 0u;
  out[k] = c;
}

__global__ __launch_bounds__(256) void k_prune_gather(long n, float thr, const uint32_t* blk,
                                                      SceneDev in, int color_stride,
                                                      float* m, float* ls, float* q, float* o,
                                                      float* col) {
  __shared__ uint32_t wc[4];
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const bool keep = i < n && in.opac[i] >= thr;
  const unsigned long long bal = __ballot(keep);
  const int lane = lane_id(), w = threadIdx.x >> 6;
  if (lane == 0) wc[w] = (uint32_t)__popcll(bal);
  __syncthreads();
  if (!keep) return;
  uint32_t pos = blk[blockIdx.x] + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
  for (int j = 0; j < w; ++j) pos += wc[j];
  for (int r = 0; r < 3; ++r) {
    m[3 * (size_t)pos + r] = in.means[3 * i + r];
    ls[3 * (size_t)pos + r] = in.log_scales[3 * i + r];
  }
  *reinterpret_cast<float4*>(q + 4 * (size_t)pos) = *reinterpret_cast<const float4*>(in.quats + 4 * i);
  o[pos] = in.opac[i];
  for (int r = 0; r < color_stride; ++r)
    col[(size_t)color_stride * pos + r] = in.colors[(size_t)color_stride * i + r];
}

hipError_t launch_prune(long n, const SceneDev& in, int color_stride, float thr,
                        const SimSetTab& sets, uint32_t* blk, long long* bounds, float* m,
                        float* ls, float* q, float* o, float* col, hipStream_t s) {
  const int nb = (int)((n + 255) / 256);
  if (nb > 0)
    hipLaunchKernelGGL(k_prune_count, dim3(nb), dim3(256), 0, s, n, in.opac, thr, blk);
  hipLaunchKernelGGL(k_prune_scan, dim3(1), dim3(1024), 0, s, nb, blk);
  hipLaunchKernelGGL(k_prune_bounds, dim3(1), dim3(MAXS + 1), 0, s, sets, in.opac, thr, blk,
                     bounds);
  if (nb > 0)
    hipLaunchKernelGGL(k_prune_gather, dim3(nb), dim3(256), 0, s, n, thr, blk, in, color_stride,
                       m, ls, q, o, col);
  return hipGetLastError();
}

}  // namespace gsr
