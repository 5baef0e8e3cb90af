// SSIM term of the refinement loss (Sec. III-C, Eq. (refine_loss)) on the
// exposure-compensated render I~ = exp(a_v) I^ + b_v, and its gradient.
//
// Statistics under an 11 x 11 Gaussian window (sigma 1.5, zero outside the
// image), per colour channel, in one pass over 32 x 32 pixel tiles (k_ssim):
// the five moments of (x, y) -> S and the gradient maps f1 = dS/dmx -
// 2 mx dS/dsxx - my dS/dsxy, f2 = dS/dsxx, f3 = dS/dsxy on the tile plus a
// 5-pixel halo, then blurs of f1..f3 -> d mean(S)/dx = (w*f1 + 2 x w*f2 +
// y w*f3) / N at the tile's pixels, chained through the exposure into
// d_color (accumulated); the maps never leave LDS.  k_ssim_reduce: per-block
// partial sums (S, and the exposure gradients) summed per view in a fixed
// order: no float atomics on a few hot addresses.
#include "common.h"

namespace gsr {

constexpr int SS_T = 32, SS_R = 5;   // tile, window radius
constexpr int SS_K = 2 * SS_R + 1;     // taps
constexpr int SS_P = 4;                // outputs per thread and blur
constexpr int SS_L = SS_P + 2 * SS_R;  // the values they read
static_assert(SS_T * SS_T == 256 * SS_P, "the tile's blur: SS_P outputs per thread");
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

// One workgroup per 32 x 32 tile of one channel of one view, in LDS only:
//  A  x~ = exp(a) I^ + b and the target, on the tile plus a 10-pixel halo
//     (zero outside the image), SS_X x SS_X staged;
//  B/C the five window moments on the SS_S x SS_S statistics region (the tile
//     plus a 5-pixel halo, two spare rows and columns): horizontal blurs into
//     LDS, then vertical blurs into registers, in two groups (x, y, xy; then
//     xx, yy) so that one buffer of three maps serves both;
//  D  S and the gradient maps f1..f3 of the region (zero outside the image)
//     into the staging buffer, S summed over the tile;
//  E/F the blurred maps at the tile's pixels, chained through the exposure
//     into d_color.
// Each thread blurs SS_P consecutive outputs of a row or column from SS_L
// values held in registers.
constexpr int SS_S = 44, SS_X = SS_S + 2 * SS_R;  // statistics region, staged edge
constexpr int SS_SG = SS_S / SS_P;                // row groups of the region
static_assert(SS_S >= SS_T + 2 * SS_R && SS_S % SS_P == 0, "statistics region");

// Horizontal blur of rows [0, nrow) of NM maps (or of the products of (x, y)
// when PROD > 0: PROD = 1 blurs x, y, xy; PROD = 2 blurs xx, yy) into NO maps
// of nout columns (a multiple of SS_P).
template <int NM, int NO, int PROD, int SW, int DW, int NROW>
__device__ __forceinline__ void ss_hblur(const SsimArgs& A, const float (*src)[NROW][SW],
                                         float (*dst)[NROW][DW], int nout) {
  const int runs = nout / SS_P;
  for (int it = threadIdx.x; it < NROW * runs; it += 256) {
    const int r = it / runs, c0 = (it - r * runs) * SS_P;
    float acc[NO][SS_P];
#pragma unroll
    for (int k = 0; k < NO; ++k)
#pragma unroll
      for (int o = 0; o < SS_P; ++o) acc[k][o] = 0.f;
#pragma unroll
    for (int t = 0; t < SS_L; ++t) {
      float q[NO];
      if constexpr (PROD == 1) {
        const float x = src[0][r][c0 + t], y = src[1][r][c0 + t];
        q[0] = x; q[1] = y; q[2 % NO] = x * y;
      } else if constexpr (PROD == 2) {
        const float x = src[0][r][c0 + t], y = src[1][r][c0 + t];
        q[0] = x * x; q[1 % NO] = y * y;
      } else {
#pragma unroll
        for (int k = 0; k < NO; ++k) q[k] = src[k % NM][r][c0 + t];
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

// Vertical blur of one map at column j, output rows i0 .. i0 + SS_P - 1
// (input rows i0 .. i0 + SS_L - 1).
template <int DW, int NROW>
__device__ __forceinline__ void ss_vblur(const SsimArgs& A, const float (*m)[DW], int i0, int j,
                                         float (&out)[SS_P]) {
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

struct SsimSmem {
  union {
    float sxy[2][SS_X][SS_X + 1];  // A-B: x~ and the target
    float f[3][SS_S][SS_S + 1];    // D-E: f1, f2, f3 on the statistics region
  } u0;
  union {
    float hm[3][SS_X][SS_S + 1];   // B-C: horizontal moment blurs
    float hf[3][SS_S][SS_T + 1];   // E-F: horizontal blurs of f1..f3
  } u1;
  float red[4];
};

constexpr int SS_ITEMS = SS_S * SS_SG;                     // vertical statistics items
constexpr int SS_IPT = (SS_ITEMS + 255) / 256;              // per thread

__global__ __launch_bounds__(256) void k_ssim(SsimArgs A, const float* color, const float* target,
                                              const float* expo, float* d_color,
                                              float* ssim_part, float* e_part) {
  __shared__ SsimSmem sm;
  const int vc = blockIdx.y, v = vc / 3;
  const int ty = blockIdx.x / A.TX, tx = blockIdx.x - ty * A.TX;
  // pixel of staged (0, 0) and of statistics-region (0, 0)
  const int XS = tx * SS_T - 2 * SS_R, YS = ty * SS_T - 2 * SS_R;
  const int XR = tx * SS_T - SS_R, YR = ty * SS_T - SS_R;
  const float ea = expo ? expf(expo[2 * v]) : 1.f, eb = expo ? expo[2 * v + 1] : 0.f;
  const size_t plane = (size_t)A.W * A.H;
  const float* ci = color + (size_t)vc * plane;
  const float* ti = target + (size_t)vc * plane;
  for (int i = threadIdx.x; i < SS_X * SS_X; i += 256) {
    const int r = i / SS_X, c = i - r * SS_X;
    const int gx = XS + c, gy = YS + r;
    const bool in = gx >= 0 && gx < A.W && gy >= 0 && gy < A.H;
    const size_t q = (size_t)gy * A.W + gx;
    sm.u0.sxy[0][r][c] = in ? ea * ci[q] + eb : 0.f;
    sm.u0.sxy[1][r][c] = in ? ti[q] : 0.f;
  }
  __syncthreads();
  // moments of the statistics items: item = (column c, row group g)
  float mom[SS_IPT][5][SS_P];
  ss_hblur<2, 3, 1, SS_X + 1, SS_S + 1, SS_X>(A, sm.u0.sxy, sm.u1.hm, SS_S);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < SS_IPT; ++u) {
    const int it = (int)threadIdx.x + 256 * u;
    if (it < SS_ITEMS) {
      const int c = it % SS_S, g = it / SS_S;
      ss_vblur<SS_S + 1, SS_X>(A, sm.u1.hm[0], g * SS_P, c, mom[u][0]);  // x
      ss_vblur<SS_S + 1, SS_X>(A, sm.u1.hm[1], g * SS_P, c, mom[u][1]);  // y
      ss_vblur<SS_S + 1, SS_X>(A, sm.u1.hm[2], g * SS_P, c, mom[u][4]);  // xy
    }
  }
  __syncthreads();
  ss_hblur<2, 2, 2, SS_X + 1, SS_S + 1, SS_X>(A, sm.u0.sxy, sm.u1.hm, SS_S);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < SS_IPT; ++u) {
    const int it = (int)threadIdx.x + 256 * u;
    if (it < SS_ITEMS) {
      const int c = it % SS_S, g = it / SS_S;
      ss_vblur<SS_S + 1, SS_X>(A, sm.u1.hm[0], g * SS_P, c, mom[u][2]);  // xx
      ss_vblur<SS_S + 1, SS_X>(A, sm.u1.hm[1], g * SS_P, c, mom[u][3]);  // yy
    }
  }
  __syncthreads();  // the staging buffer becomes the f maps
  float s = 0.f;
#pragma unroll
  for (int u = 0; u < SS_IPT; ++u) {
    const int it = (int)threadIdx.x + 256 * u;
    if (it < SS_ITEMS) {
      const int c = it % SS_S, g = it / SS_S;
      const int gx = XR + c;
#pragma unroll
      for (int o = 0; o < SS_P; ++o) {
        const int r = g * SS_P + o, gy = YR + r;
        float f1 = 0.f, f2 = 0.f, f3 = 0.f;
        if (gx >= 0 && gx < A.W && gy >= 0 && gy < A.H) {
          const float mx = mom[u][0][o], my = mom[u][1][o];
          const float sxx = mom[u][2][o] - mx * mx, syy = mom[u][3][o] - my * my;
          const float sxy = mom[u][4][o] - mx * my;
          const float a1 = 2.f * mx * my + SS_C1, a2 = 2.f * sxy + SS_C2;
          const float b1 = mx * mx + my * my + SS_C1, b2 = sxx + syy + SS_C2;
          // b1, b2 >= C1, C2 > 0: reciprocals by the hardware (about 1 ulp)
          const float rb1 = __builtin_amdgcn_rcpf(b1), rb2 = __builtin_amdgcn_rcpf(b2);
          const float ib = rb1 * rb2;
          const float so = a1 * a2 * ib;
          const float d_mx = 2.f * my * a2 * ib - 2.f * mx * so * rb1;
          const float d_sxx = -so * rb2;
          const float d_sxy = 2.f * a1 * ib;
          f1 = d_mx - 2.f * mx * d_sxx - my * d_sxy;
          f2 = d_sxx;
          f3 = d_sxy;
          // the tile's own pixels carry S
          if (r >= SS_R && r < SS_R + SS_T && c >= SS_R && c < SS_R + SS_T) s += so;
        }
        sm.u0.f[0][r][c] = f1;
        sm.u0.f[1][r][c] = f2;
        sm.u0.f[2][r][c] = f3;
      }
    }
  }
  __syncthreads();
  ss_hblur<3, 3, 0, SS_S + 1, SS_T + 1, SS_S>(A, sm.u0.f, sm.u1.hf, SS_T);
  __syncthreads();
  // thread: column j, rows i0 .. i0 + SS_P - 1 of the tile
  const int j = threadIdx.x % SS_T, i0 = (threadIdx.x / SS_T) * SS_P;
  float bl[3][SS_P];
#pragma unroll
  for (int k = 0; k < 3; ++k) ss_vblur<SS_T + 1, SS_S>(A, sm.u1.hf[k], i0, j, bl[k]);
  const int gx = tx * SS_T + j;
  float sa = 0.f, sb = 0.f;
#pragma unroll
  for (int o = 0; o < SS_P; ++o) {
    const int gy = ty * SS_T + i0 + o;
    if (gx < A.W && gy < A.H) {
      const size_t q = (size_t)gy * A.W + gx;
      const float c = ci[q];
      const float x = ea * c + eb, y = ti[q];
      // loss = weight (1 - mean S): dL/dx~ = -weight/N (w*f1 + 2 x w*f2 + y w*f3)
      const float g = -A.weight_over_n * (bl[0][o] + 2.f * x * bl[1][o] + y * bl[2][o]);
      d_color[(size_t)vc * plane + q] += ea * g;
      sa += g * c;
      sb += g;
    }
  }
  const size_t bb = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
  const float t = block_sum_256(s, sm.red);
  if (threadIdx.x == 0) ssim_part[bb] = t;
  if (!e_part) return;  // uniform
  const float ta = block_sum_256(sa, sm.red);
  const float tb = block_sum_256(sb, sm.red);
  if (threadIdx.x == 0) {
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
  return align_up(nb * 4) + align_up(nb * 8) + align_up((size_t)nv * 4);
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
  const dim3 grid(nb_view, 3 * nv);
  hipLaunchKernelGGL(k_ssim, grid, dim3(256), 0, s, A, color, target, expo, d_color, s_part,
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
