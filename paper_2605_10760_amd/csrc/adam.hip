// Adam update of the optimisation drivers (the mapping loss, Sec. III-A
// Eq. (map_loss), and the refinement, Sec. III-C Eq. (refine_loss), are
// minimised by first-order steps; the optimiser is Adam with per-array
// learning rates).
//
// One launch updates up to GSR_ADAM_MAX_GROUPS arrays: the arrays are cut
// into chunks of ADAM_CHUNK elements, a workgroup takes one chunk (the
// chunk -> array map travels in the kernel arguments), and every element is
// read once (parameter, gradient, two moments) and written once (parameter,
// two moments): HBM-bound, 28 B per element.  The FP64 bias corrections are
// formed once per workgroup.  The step count lives on the device and is
// advanced by the launch that follows, so a captured step replays with the
// right bias corrections.
#include "common.h"

namespace gsr {

constexpr int ADAM_THREADS = 256;
constexpr int ADAM_CHUNK = 4 * ADAM_THREADS;  // one float4 per thread

struct AdamTab {
  int ng;
  int chunk_off[GSR_ADAM_MAX_GROUPS + 1];  // chunks per array, prefix
  float* p[GSR_ADAM_MAX_GROUPS];
  const float* g[GSR_ADAM_MAX_GROUPS];
  float* m[GSR_ADAM_MAX_GROUPS];
  float* v[GSR_ADAM_MAX_GROUPS];
  long long n[GSR_ADAM_MAX_GROUPS];
  float lr[GSR_ADAM_MAX_GROUPS];
  float b1, c1, b2, c2, eps;  // beta, 1 - beta (rounded once from FP64)
  double b1d, b2d;            // the betas for the bias corrections
};

// The square root and the quotient by the hardware approximations (about
// 1 ulp each), far inside the update's own rounding of m and v.
__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, const AdamTab& t,
                                         float step_size, float inv_sqrt_bc2) {
  m = t.b1 * m + t.c1 * g;
  v = t.b2 * v + t.c2 * (g * g);
  p -= step_size * (m * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v) * inv_sqrt_bc2 + t.eps));
}

__global__ __launch_bounds__(ADAM_THREADS) void k_adam(AdamTab t, const int32_t* step) {
  __shared__ float bc[2];
  const int b = xcd_remap(blockIdx.x, t.chunk_off[t.ng]);
  if (b < 0) return;
  const int a = find_seg(t.chunk_off, t.ng, b);
  const long long n = t.n[a];
  float* P = t.p[a];
  const float* G = t.g[a];
  float* M = t.m[a];
  float* V = t.v[a];
  const bool vec = ((((uintptr_t)P) | ((uintptr_t)G) | ((uintptr_t)M) | ((uintptr_t)V)) & 15) == 0;
  const long long i0 = (long long)(b - t.chunk_off[a]) * ADAM_CHUNK + 4 * (long long)threadIdx.x;
  const bool full = vec && i0 + 4 <= n;
  // the element loads go out before the bias corrections are formed
  float4 p = make_float4(0.f, 0.f, 0.f, 0.f), g = p, m = p, v = p;
  if (full) {
    p = *reinterpret_cast<const float4*>(P + i0);
    g = *reinterpret_cast<const float4*>(G + i0);
    m = *reinterpret_cast<const float4*>(M + i0);
    v = *reinterpret_cast<const float4*>(V + i0);
  }
  // bias corrections of step t = *step + 1, in FP64 (1 - beta^t cancels),
  // by one thread of the workgroup
  if (threadIdx.x == 0) {
    const double tt = (double)(step[0] + 1);
    const double bc1 = 1.0 - pow(t.b1d, tt), bc2 = 1.0 - pow(t.b2d, tt);
    bc[0] = (float)((double)t.lr[a] / bc1);
    bc[1] = (float)(1.0 / sqrt(bc2));
  }
  __syncthreads();
  const float step_size = bc[0], inv_sqrt_bc2 = bc[1];
  if (full) {
    adam_one(p.x, g.x, m.x, v.x, t, step_size, inv_sqrt_bc2);
    adam_one(p.y, g.y, m.y, v.y, t, step_size, inv_sqrt_bc2);
    adam_one(p.z, g.z, m.z, v.z, t, step_size, inv_sqrt_bc2);
    adam_one(p.w, g.w, m.w, v.w, t, step_size, inv_sqrt_bc2);
    *reinterpret_cast<float4*>(P + i0) = p;
    *reinterpret_cast<float4*>(M + i0) = m;
    *reinterpret_cast<float4*>(V + i0) = v;
  } else {
    for (long long i = i0; i < i0 + 4 && i < n; ++i) {
      float pp = P[i], mm = M[i], vv = V[i];
      adam_one(pp, G[i], mm, vv, t, step_size, inv_sqrt_bc2);
      P[i] = pp;
      M[i] = mm;
      V[i] = vv;
    }
  }
}

// The step count advances after the update has read it.
__global__ void k_adam_tick(int32_t* step) {
  if (threadIdx.x == 0) step[0] += 1;
}

hipError_t launch_adam(const gsr_adam_group* gr, int ng, double b1, double b2, double eps,
                       int32_t* step, hipStream_t s) {
  AdamTab t{};
  t.ng = ng;
  t.b1 = (float)b1;
  t.c1 = (float)(1.0 - b1);
  t.b2 = (float)b2;
  t.c2 = (float)(1.0 - b2);
  t.eps = (float)eps;
  t.b1d = b1;
  t.b2d = b2;
  int c = 0;
  for (int k = 0; k < ng; ++k) {
    t.chunk_off[k] = c;
    t.p[k] = gr[k].param;
    t.g[k] = gr[k].grad;
    t.m[k] = gr[k].exp_avg;
    t.v[k] = gr[k].exp_avg_sq;
    t.n[k] = gr[k].n;
    t.lr[k] = gr[k].lr;
    c += (int)((gr[k].n + ADAM_CHUNK - 1) / ADAM_CHUNK);
  }
  t.chunk_off[ng] = c;
  if (c > 0) hipLaunchKernelGGL(k_adam, dim3(xcd_grid(c)), dim3(ADAM_THREADS), 0, s, t, step);
  hipLaunchKernelGGL(k_adam_tick, dim3(1), dim3(64), 0, s, step);
  return hipGetLastError();
}

}  // namespace gsr
