// SSIM term of the refinement loss (Sec. III-C, Eq. (refine_loss)) on the
// exposure-compensated render I~ = exp(a_v) I^ + b_v, and its gradient.
//
// Statistics under an 11 x 11 Gaussian window (sigma 1.5, zero outside the
// image), per colour channel.  Two passes over 16 x 16 pixel tiles, each
// staging the tile plus a 5-pixel halo in LDS and blurring separably
// (horizontal into LDS, then vertical):
//   k_ssim_stats: the five moments of (x, y) -> S and the three gradient
//     maps f1 = dS/dmx - 2 mx dS/dsxx - my dS/dsxy, f2 = dS/dsxx,
//     f3 = dS/dsxy (12 B per pixel and channel to the workspace), and the sum
//     of S;
//   k_ssim_grad: blurs of f1..f3 -> d mean(S)/dx = (w*f1 + 2 x w*f2 +
//     y w*f3) / N, chained through the exposure into d_color (accumulated);
//   k_ssim_reduce: per-block partial sums (S, and the exposure gradients)
//     summed per view in a fixed order: no float atomics on a few hot
//     addresses.
#include "common.h"

namespace gsr {

constexpr int SS_T = 16, SS_R = 5, SS_E = SS_T + 2 * SS_R;  // tile, radius, staged edge
constexpr float SS_C1 = 0.01f * 0.01f, SS_C2 = 0.03f * 0.03f;

struct SsimArgs {
  float w[2 * SS_R + 1];
  int W, H, TX, nv;
  float weight_over_n;  // weight / (3 V H W)
};

__device__ __forceinline__ float block_sum_256(float x, float* red) {
  x = wave_total(x);
  if (lane_id() == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  const float t = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void k_ssim_stats(SsimArgs A, const float* color,
                                                    const float* target, const float* expo,
                                                    float* f, float* ssim_part) {
  __shared__ float sx[SS_E][SS_E + 1], sy[SS_E][SS_E + 1];
  __shared__ float hm[5][SS_E][SS_T];
  __shared__ float red[4];
  const int vc = blockIdx.y, v = vc / 3;
  const int ty = blockIdx.x / A.TX, tx = blockIdx.x - ty * A.TX;
  const int X0 = tx * SS_T - SS_R, Y0 = ty * SS_T - SS_R;
  const float ea = expo ? expf(expo[2 * v]) : 1.f, eb = expo ? expo[2 * v + 1] : 0.f;
  const size_t plane = (size_t)A.W * A.H;
  const float* ci = color + (size_t)vc * plane;
  const float* ti = target + (size_t)vc * plane;
  for (int i = threadIdx.x; i < SS_E * SS_E; i += 256) {
    const int r = i / SS_E, c = i - r * SS_E;
    const int gx = X0 + c, gy = Y0 + r;
    const bool in = gx >= 0 && gx < A.W && gy >= 0 && gy < A.H;
    const size_t q = (size_t)gy * A.W + gx;
    sx[r][c] = in ? ea * ci[q] + eb : 0.f;
    sy[r][c] = in ? ti[q] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SS_E * SS_T; i += 256) {
    const int r = i / SS_T, c = i - r * SS_T;
    float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
    for (int d = 0; d <= 2 * SS_R; ++d) {
      const float x = sx[r][c + d], y = sy[r][c + d], w = A.w[d];
      m0 += w * x;
      m1 += w * y;
      m2 += w * x * x;
      m3 += w * y * y;
      m4 += w * x * y;
    }
    hm[0][r][c] = m0; hm[1][r][c] = m1; hm[2][r][c] = m2; hm[3][r][c] = m3; hm[4][r][c] = m4;
  }
  __syncthreads();
  const int i = threadIdx.x / SS_T, j = threadIdx.x - i * SS_T;
  float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int d = 0; d <= 2 * SS_R; ++d) {
#pragma unroll
    for (int k = 0; k < 5; ++k) m[k] += A.w[d] * hm[k][i + d][j];
  }
  const int gx = tx * SS_T + j, gy = ty * SS_T + i;
  float s = 0.f;
  if (gx < A.W && gy < A.H) {
    const float mx = m[0], my = m[1];
    const float sxx = m[2] - mx * mx, syy = m[3] - my * my, sxy = m[4] - mx * my;
    const float a1 = 2.f * mx * my + SS_C1, a2 = 2.f * sxy + SS_C2;
    const float b1 = mx * mx + my * my + SS_C1, b2 = sxx + syy + SS_C2;
    const float ib = 1.f / (b1 * b2);
    s = a1 * a2 * ib;
    const float d_mx = 2.f * my * a2 * ib - 2.f * mx * s / b1;
    const float d_sxx = -s / b2;
    const float d_sxy = 2.f * a1 * ib;
    const size_t q = (size_t)vc * plane + (size_t)gy * A.W + gx;
    const size_t all = (size_t)3 * A.nv * plane;
    f[q] = d_mx - 2.f * mx * d_sxx - my * d_sxy;
    f[all + q] = d_sxx;
    f[2 * all + q] = d_sxy;
  }
  const float t = block_sum_256(s, red);
  if (threadIdx.x == 0) ssim_part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_ssim_grad(SsimArgs A, const float* color,
                                                   const float* target, const float* expo,
                                                   const float* f, float* d_color,
                                                   float* e_part) {
  __shared__ float sf[3][SS_E][SS_E + 1];
  __shared__ float hf[3][SS_E][SS_T];
  __shared__ float red[4];
  const int vc = blockIdx.y, v = vc / 3;
  const int ty = blockIdx.x / A.TX, tx = blockIdx.x - ty * A.TX;
  const int X0 = tx * SS_T - SS_R, Y0 = ty * SS_T - SS_R;
  const size_t plane = (size_t)A.W * A.H, all = (size_t)3 * A.nv * plane;
  const float* fv = f + (size_t)vc * plane;
  for (int i = threadIdx.x; i < SS_E * SS_E; i += 256) {
    const int r = i / SS_E, c = i - r * SS_E;
    const int gx = X0 + c, gy = Y0 + r;
    const bool in = gx >= 0 && gx < A.W && gy >= 0 && gy < A.H;
    const size_t q = (size_t)gy * A.W + gx;
#pragma unroll
    for (int k = 0; k < 3; ++k) sf[k][r][c] = in ? fv[k * all + q] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SS_E * SS_T; i += 256) {
    const int r = i / SS_T, c = i - r * SS_T;
    float h0 = 0.f, h1 = 0.f, h2 = 0.f;
#pragma unroll
    for (int d = 0; d <= 2 * SS_R; ++d) {
      const float w = A.w[d];
      h0 += w * sf[0][r][c + d];
      h1 += w * sf[1][r][c + d];
      h2 += w * sf[2][r][c + d];
    }
    hf[0][r][c] = h0; hf[1][r][c] = h1; hf[2][r][c] = h2;
  }
  __syncthreads();
  const int i = threadIdx.x / SS_T, j = threadIdx.x - i * SS_T;
  float b0 = 0.f, b1 = 0.f, b2 = 0.f;
#pragma unroll
  for (int d = 0; d <= 2 * SS_R; ++d) {
    const float w = A.w[d];
    b0 += w * hf[0][i + d][j];
    b1 += w * hf[1][i + d][j];
    b2 += w * hf[2][i + d][j];
  }
  const int gx = tx * SS_T + j, gy = ty * SS_T + i;
  const float ea = expo ? expf(expo[2 * v]) : 1.f, eb = expo ? expo[2 * v + 1] : 0.f;
  float sa = 0.f, sb = 0.f;
  if (gx < A.W && gy < A.H) {
    const size_t q = (size_t)vc * plane + (size_t)gy * A.W + gx;
    const float c = color[q];
    const float x = ea * c + eb, y = target[q];
    // loss = weight (1 - mean S): dL/dx~ = -weight/N (w*f1 + 2 x w*f2 + y w*f3)
    const float g = -A.weight_over_n * (b0 + 2.f * x * b1 + y * b2);
    d_color[q] += ea * g;
    sa = g * c;
    sb = g;
  }
  if (!e_part) return;  // uniform
  const float ta = block_sum_256(sa, red);
  const float tb = block_sum_256(sb, red);
  if (threadIdx.x == 0) {
    const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    e_part[2 * b] = ea * ta;
    e_part[2 * b + 1] = tb;
  }
}

// One workgroup per view: the view's block partials of the exposure sums
// (added to d_expo) and of S (to s_view[v]).  Sums run in a fixed order
// (deterministic).
__global__ __launch_bounds__(256) void k_ssim_reduce(int nb_view, const float* s_part,
                                                     const float* e_part, float* d_expo,
                                                     float* s_view) {
  __shared__ float red[4];
  const int v = blockIdx.x;
  const size_t k0 = (size_t)v * 3 * nb_view;
  float a = 0.f, b = 0.f, t = 0.f;
  for (int i = threadIdx.x; i < 3 * nb_view; i += 256) {
    t += s_part[k0 + i];
    if (e_part) {
      a += e_part[2 * (k0 + i)];
      b += e_part[2 * (k0 + i) + 1];
    }
  }
  t = block_sum_256(t, red);
  if (e_part) {
    a = block_sum_256(a, red);
    b = block_sum_256(b, red);
  }
  if (threadIdx.x == 0) {
    s_view[v] = t;
    if (e_part) {
      d_expo[2 * v] += a;
      d_expo[2 * v + 1] += b;
    }
  }
}

__global__ __launch_bounds__(64) void k_ssim_mean(int nv, const float* s_view, float inv_n,
                                                  float* out) {
  float t = 0.f;
  for (int v = threadIdx.x; v < nv; v += 64) t += s_view[v];
  t = wave_total(t);
  if (threadIdx.x == 0) out[0] = t * inv_n;
}

static size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

size_t ssim_workspace_bytes(int nv, int W, int H) {
  const size_t nb = (size_t)((W + SS_T - 1) / SS_T) * ((H + SS_T - 1) / SS_T) * 3 * nv;
  return align_up(nb * 4) + align_up(nb * 8) + align_up((size_t)nv * 4) +
         (size_t)3 * 3 * nv * (size_t)W * H * sizeof(float);
}

hipError_t launch_ssim(int nv, int W, int H, float weight, const float* color,
                       const float* target, const float* expo, void* ws, float* d_color,
                       float* d_expo, float* ssim_out, hipStream_t s) {
  SsimArgs A{};
  double g[2 * SS_R + 1], tot = 0.0;
  for (int d = -SS_R; d <= SS_R; ++d) tot += g[d + SS_R] = exp(-(double)(d * d) / (2.0 * 1.5 * 1.5));
  for (int d = 0; d <= 2 * SS_R; ++d) A.w[d] = (float)(g[d] / tot);
  A.W = W;
  A.H = H;
  A.TX = (W + SS_T - 1) / SS_T;
  A.nv = nv;
  const double n = 3.0 * nv * (double)W * H;
  A.weight_over_n = (float)(weight / n);
  const int TY = (H + SS_T - 1) / SS_T;
  const int nb_view = A.TX * TY;
  const size_t nb = (size_t)nb_view * 3 * nv;
  char* w8 = (char*)ws;
  float* s_part = (float*)w8;
  float* e_part = (float*)(w8 + align_up(nb * 4));
  float* s_view = (float*)(w8 + align_up(nb * 4) + align_up(nb * 8));
  float* f = (float*)(w8 + align_up(nb * 4) + align_up(nb * 8) + align_up((size_t)nv * 4));
  const dim3 grid(nb_view, 3 * nv);
  hipLaunchKernelGGL(k_ssim_stats, grid, dim3(256), 0, s, A, color, target, expo, f, s_part);
  hipLaunchKernelGGL(k_ssim_grad, grid, dim3(256), 0, s, A, color, target, expo, f, d_color,
                     d_expo ? e_part : (float*)nullptr);
  if (d_expo || ssim_out)
    hipLaunchKernelGGL(k_ssim_reduce, dim3(nv), dim3(256), 0, s, nb_view, s_part,
                       d_expo ? e_part : (const float*)nullptr, d_expo, s_view);
  if (ssim_out)
    hipLaunchKernelGGL(k_ssim_mean, dim3(1), dim3(64), 0, s, nv, s_view, (float)(1.0 / n),
                       ssim_out);
  return hipGetLastError();
}

}  // namespace gsr
