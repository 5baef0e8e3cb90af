// SSIM term of the refinement loss (Sec. III-C, Eq. (refine_loss)) on the
// exposure-compensated render I~ = exp(a_v) I^ + b_v, and its gradient.
//
// Statistics under an 11 x 11 Gaussian window (sigma 1.5, zero outside the
// image), per colour channel.  Two passes over 32 x 32 pixel tiles, each
// staging the tile plus a 5-pixel halo in LDS and blurring separably
// (horizontal into LDS, then vertical), every thread producing four
// consecutive outputs of a row (horizontal) or a column (vertical) from 14
// staged values held in registers, so each staged value is read from LDS
// once per four outputs instead of once per tap:
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

constexpr int SS_T = 32, SS_R = 5, SS_E = SS_T + 2 * SS_R;  // tile, radius, staged edge
constexpr int SS_K = 2 * SS_R + 1;                           // taps
constexpr int SS_P = 4;                                      // outputs per thread and pass
constexpr int SS_L = SS_P + 2 * SS_R;                        // staged values they read
constexpr int SS_RUNS = SS_T / SS_P;                         // runs of outputs per row
static_assert(SS_T * SS_T == 256 * SS_P, "the vertical pass: SS_P outputs per thread");
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

// Horizontal blur of NM staged maps (rows of SS_E values) into NM maps of
// SS_E rows x SS_T columns: item (row r, run u) reads SS_L values of each map
// and writes SS_P outputs.  PRODUCTS: the maps are (x, y) and the blurred
// quantities are x, y, x^2, y^2, x y.
template <int NM, bool PRODUCTS>
__device__ __forceinline__ void ss_hblur(const SsimArgs& A, const float (*src)[SS_E][SS_E + 1],
                                         float (*dst)[SS_E][SS_T + 1]) {
  constexpr int NO = PRODUCTS ? 5 : NM;
  for (int it = threadIdx.x; it < SS_E * SS_RUNS; it += 256) {
    const int r = it / SS_RUNS, c0 = (it - r * SS_RUNS) * SS_P;
    float acc[NO][SS_P];
#pragma unroll
    for (int k = 0; k < NO; ++k)
#pragma unroll
      for (int o = 0; o < SS_P; ++o) acc[k][o] = 0.f;
    float val[NM][SS_L];
#pragma unroll
    for (int k = 0; k < NM; ++k)
#pragma unroll
      for (int t = 0; t < SS_L; ++t) val[k][t] = src[k][r][c0 + t];
#pragma unroll
    for (int t = 0; t < SS_L; ++t) {
      float q[NO];
      if constexpr (PRODUCTS) {
        const float x = val[0][t], y = val[1][t];
        q[0] = x; q[1] = y; q[2] = x * x; q[3] = y * y; q[4] = x * y;
      } else {
#pragma unroll
        for (int k = 0; k < NO; ++k) q[k] = val[k % NM][t];
      }
#pragma unroll
      for (int o = 0; o < SS_P; ++o) {
        const int d = t - o;
        if (d >= 0 && d < SS_K) {
#pragma unroll
          for (int k = 0; k < NO; ++k) acc[k][o] += A.w[d] * q[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NO; ++k)
#pragma unroll
      for (int o = 0; o < SS_P; ++o) dst[k][r][c0 + o] = acc[k][o];
  }
}

// Vertical blur of map k of hm at column j, rows i0 .. i0 + SS_P - 1 of the
// tile (staged rows i0 .. i0 + SS_L - 1).
__device__ __forceinline__ void ss_vblur(const SsimArgs& A, const float (*m)[SS_T + 1], int i0,
                                         int j, float (&out)[SS_P]) {
  float val[SS_L];
#pragma unroll
  for (int t = 0; t < SS_L; ++t) val[t] = m[i0 + t][j];
#pragma unroll
  for (int o = 0; o < SS_P; ++o) {
    float a = 0.f;
#pragma unroll
    for (int d = 0; d < SS_K; ++d) a += A.w[d] * val[o + d];
    out[o] = a;
  }
}

__global__ __launch_bounds__(256) void k_ssim_stats(SsimArgs A, const float* color,
                                                    const float* target, const float* expo,
                                                    float* f, float* ssim_part) {
  __shared__ float sxy[2][SS_E][SS_E + 1];
  __shared__ float hm[5][SS_E][SS_T + 1];
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
    sxy[0][r][c] = in ? ea * ci[q] + eb : 0.f;
    sxy[1][r][c] = in ? ti[q] : 0.f;
  }
  __syncthreads();
  ss_hblur<2, true>(A, sxy, hm);
  __syncthreads();
  // thread: column j, rows i0 .. i0 + 3 of the tile
  const int j = threadIdx.x % SS_T, i0 = (threadIdx.x / SS_T) * SS_P;
  float m[5][SS_P];
#pragma unroll
  for (int k = 0; k < 5; ++k) ss_vblur(A, hm[k], i0, j, m[k]);
  const int gx = tx * SS_T + j;
  const size_t all = (size_t)3 * A.nv * plane;
  float s = 0.f;
#pragma unroll
  for (int o = 0; o < SS_P; ++o) {
    const int gy = ty * SS_T + i0 + o;
    if (gx < A.W && gy < A.H) {
      const float mx = m[0][o], my = m[1][o];
      const float sxx = m[2][o] - mx * mx, syy = m[3][o] - my * my, sxy = m[4][o] - mx * my;
      const float a1 = 2.f * mx * my + SS_C1, a2 = 2.f * sxy + SS_C2;
      const float b1 = mx * mx + my * my + SS_C1, b2 = sxx + syy + SS_C2;
      const float ib = 1.f / (b1 * b2);
      const float so = a1 * a2 * ib;
      const float d_mx = 2.f * my * a2 * ib - 2.f * mx * so / b1;
      const float d_sxx = -so / b2;
      const float d_sxy = 2.f * a1 * ib;
      const size_t q = (size_t)vc * plane + (size_t)gy * A.W + gx;
      f[q] = d_mx - 2.f * mx * d_sxx - my * d_sxy;
      f[all + q] = d_sxx;
      f[2 * all + q] = d_sxy;
      s += so;
    }
  }
  const float t = block_sum_256(s, red);
  if (threadIdx.x == 0) ssim_part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_ssim_grad(SsimArgs A, const float* color,
                                                   const float* target, const float* expo,
                                                   const float* f, float* d_color,
                                                   float* e_part) {
  __shared__ float sf[3][SS_E][SS_E + 1];
  __shared__ float hf[3][SS_E][SS_T + 1];
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
  ss_hblur<3, false>(A, sf, hf);
  __syncthreads();
  const int j = threadIdx.x % SS_T, i0 = (threadIdx.x / SS_T) * SS_P;
  float b[3][SS_P];
#pragma unroll
  for (int k = 0; k < 3; ++k) ss_vblur(A, hf[k], i0, j, b[k]);
  const int gx = tx * SS_T + j;
  const float ea = expo ? expf(expo[2 * v]) : 1.f, eb = expo ? expo[2 * v + 1] : 0.f;
  float sa = 0.f, sb = 0.f;
#pragma unroll
  for (int o = 0; o < SS_P; ++o) {
    const int gy = ty * SS_T + i0 + o;
    if (gx < A.W && gy < A.H) {
      const size_t q = (size_t)vc * plane + (size_t)gy * A.W + gx;
      const float c = color[q];
      const float x = ea * c + eb, y = target[q];
      // loss = weight (1 - mean S): dL/dx~ = -weight/N (w*f1 + 2 x w*f2 + y w*f3)
      const float g = -A.weight_over_n * (b[0][o] + 2.f * x * b[1][o] + y * b[2][o]);
      d_color[q] += ea * g;
      sa += g * c;
      sb += g;
    }
  }
  if (!e_part) return;  // uniform
  const float ta = block_sum_256(sa, red);
  const float tb = block_sum_256(sb, red);
  if (threadIdx.x == 0) {
    const size_t bb = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    e_part[2 * bb] = ea * ta;
    e_part[2 * bb + 1] = tb;
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
