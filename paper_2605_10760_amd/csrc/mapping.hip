// Mapping-loss extras (Sec. III-A, Eq. (map_loss)) and Gaussian seeding of
// new keyframes.
//
// k_iso_grad: one thread per Gaussian, the gradient of the isotropy term
// sum_c |s_c - mean(s)| (s = exp(log-scale)) with respect to the log-scales,
// added into the caller's gradient (HBM-bound: 12 B read, 12 B read-modify-
// written per Gaussian).
// k_normal_grad: one 16 x 16 output tile per workgroup.  The depth of the
// tile plus a two-pixel halo goes to LDS; every pixel of the tile plus a
// one-pixel halo computes its depth-induced normal (central differences of
// back-projected points) and the gradients of its cosine loss with respect
// to its two difference vectors, also to LDS; each output pixel then gathers
// the four difference-vector gradients that involve it and projects them on
// its ray.  The difference vectors are formed from depth differences and the
// exact ray differences (2 / f), which keeps FP32 cancellation small.
// k_seed_*: ordered compaction (per-block counts, one-workgroup scan,
// wave-ballot ranks) of the pixels with positive depth on a stride grid,
// each writing one isotropic Gaussian at its back-projected point.
// The allocation-free seeding variant keeps the per-block counts in a
// file-scope device array instead of a temporary allocation.
#include <mutex>

#include "common.h"

namespace gsr {

__global__ __launch_bounds__(256) void k_iso_grad(long n, const float* ls, float w, float* g) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float s0 = expf(ls[3 * i]), s1 = expf(ls[3 * i + 1]), s2 = expf(ls[3 * i + 2]);
  // sign(s_c - mean) = sign(2 s_c - s_a - s_b): equal components give an
  // exact 0, and three equal components give a zero gradient either way
  const float e0 = 2.f * s0 - (s1 + s2), e1 = 2.f * s1 - (s0 + s2), e2 = 2.f * s2 - (s0 + s1);
  const float q0 = e0 > 0.f ? 1.f : (e0 < 0.f ? -1.f : 0.f);
  const float q1 = e1 > 0.f ? 1.f : (e1 < 0.f ? -1.f : 0.f);
  const float q2 = e2 > 0.f ? 1.f : (e2 < 0.f ? -1.f : 0.f);
  const float m = (q0 + q1 + q2) * (1.f / 3.f);
  g[3 * i] += w * s0 * (q0 - m);
  g[3 * i + 1] += w * s1 * (q1 - m);
  g[3 * i + 2] += w * s2 * (q2 - m);
}

hipError_t launch_iso_grad(long n, const float* ls, float w, float* g, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_iso_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ls, w,
                       g);
  return hipGetLastError();
}

// ------------------------------------------------------------ normal loss
constexpr int NT = 16;       // output tile edge
constexpr int NG = NT + 2;   // pixels whose normals the tile needs
constexpr int ND = NT + 4;   // depth samples those normals read

struct F3 {
  float x, y, z;
};
__device__ __forceinline__ F3 cross3(F3 a, F3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__global__ __launch_bounds__(256) void k_normal_grad(int W, int H, int tiles_x, int tiles_y,
                                                     const float* depth, const float* prior,
                                                     const float* intr, float w, float* g_dep) {
  __shared__ float sd[ND][ND];
  __shared__ float sg[6][NG][NG];  // (ga, gb) of every pixel of the tile + halo
  const int tpv = tiles_x * tiles_y;
  const int v = blockIdx.x / tpv;
  const int t = blockIdx.x - v * tpv;
  const int j0 = (t / tiles_x) * NT, i0 = (t % tiles_x) * NT;
  const size_t HW = (size_t)H * W;
  const float* dv = depth + v * HW;
  for (int k = threadIdx.x; k < ND * ND; k += 256) {
    const int j = j0 - 2 + k / ND, i = i0 - 2 + k % ND;
    sd[k / ND][k % ND] = (j >= 0 && j < H && i >= 0 && i < W) ? dv[(size_t)j * W + i] : 0.f;
  }
  const float fx = intr[4 * v], fy = intr[4 * v + 1], cx = intr[4 * v + 2], cy = intr[4 * v + 3];
  const float ifx = 1.f / fx, ify = 1.f / fy;
  __syncthreads();
  for (int k = threadIdx.x; k < NG * NG; k += 256) {
    const int lj = k / NG, li = k % NG;
    const int j = j0 - 1 + lj, i = i0 - 1 + li;
    F3 ga{0.f, 0.f, 0.f}, gb{0.f, 0.f, 0.f};
    if (j >= 1 && j < H - 1 && i >= 1 && i < W - 1) {
      const float du = sd[lj + 2][li + 1], dd = sd[lj][li + 1];
      const float dr = sd[lj + 1][li + 2], dl = sd[lj + 1][li];
      if (du > 0.f && dd > 0.f && dr > 0.f && dl > 0.f) {
        const float xi = ((float)i + 0.5f - cx) * ifx, yj = ((float)j + 0.5f - cy) * ify;
        const float xr = ((float)(i + 1) + 0.5f - cx) * ifx;
        const float yu = ((float)(j + 1) + 0.5f - cy) * ify;
        // a = P(i, j+1) - P(i, j-1), b = P(i+1, j) - P(i-1, j)
        const float ev = du - dd, eh = dr - dl;
        const F3 a{ev * xi, ev * yu + dd * (2.f * ify), ev};
        const F3 b{eh * xr + dl * (2.f * ifx), eh * yj, eh};
        const F3 c = cross3(a, b);
        const float n2 = c.x * c.x + c.y * c.y + c.z * c.z;
        if (n2 > 0.f) {
          const float inr = rsqrtf(n2);
          const F3 n{c.x * inr, c.y * inr, c.z * inr};
          const size_t q = v * 3 * HW + (size_t)j * W + i;
          const F3 p{prior[q], prior[q + HW], prior[q + 2 * HW]};
          const float dot = n.x * p.x + n.y * p.y + n.z * p.z;
          const float sc = w * inr;
          const F3 gc{sc * (dot * n.x - p.x), sc * (dot * n.y - p.y), sc * (dot * n.z - p.z)};
          ga = cross3(b, gc);
          gb = cross3(gc, a);
        }
      }
    }
    sg[0][lj][li] = ga.x;
    sg[1][lj][li] = ga.y;
    sg[2][lj][li] = ga.z;
    sg[3][lj][li] = gb.x;
    sg[4][lj][li] = gb.y;
    sg[5][lj][li] = gb.z;
  }
  __syncthreads();
  const int lj = threadIdx.x / NT, li = threadIdx.x % NT;
  const int j = j0 + lj, i = i0 + li;
  if (j >= H || i >= W) return;
  // the point P(i, j) is the "+" end of the vertical difference of (i, j-1),
  // the "-" end of that of (i, j+1), and likewise horizontally
  const int gj = lj + 1, gi = li + 1;
  const float px = sg[0][gj - 1][gi] - sg[0][gj + 1][gi] + sg[3][gj][gi - 1] - sg[3][gj][gi + 1];
  const float py = sg[1][gj - 1][gi] - sg[1][gj + 1][gi] + sg[4][gj][gi - 1] - sg[4][gj][gi + 1];
  const float pz = sg[2][gj - 1][gi] - sg[2][gj + 1][gi] + sg[5][gj][gi - 1] - sg[5][gj][gi + 1];
  const float rx = ((float)i + 0.5f - cx) * ifx, ry = ((float)j + 0.5f - cy) * ify;
  g_dep[v * HW + (size_t)j * W + i] += rx * px + ry * py + pz;
}

hipError_t launch_normal_grad(int nv, int W, int H, const float* depth, const float* prior,
                              const float* intr, float w, float* g_dep, hipStream_t s) {
  const int tx = (W + NT - 1) / NT, ty = (H + NT - 1) / NT;
  hipLaunchKernelGGL(k_normal_grad, dim3((unsigned)(nv * tx * ty)), dim3(256), 0, s, W, H, tx,
                     ty, depth, prior, intr, w, g_dep);
  return hipGetLastError();
}

// ---------------------------------------------------------------- seeding
struct SeedGrid {
  int W, H, stride, gw;  // gw grid columns
  long m;                // grid points
};

__device__ __forceinline__ bool seed_valid(const SeedGrid& sgd, const float* d, long k, int* pj,
                                           int* pi) {
  if (k >= sgd.m) return false;
  const int gj = (int)(k / sgd.gw), gi = (int)(k - (long)gj * sgd.gw);
  *pj = gj * sgd.stride;
  *pi = gi * sgd.stride;
  return d[(size_t)*pj * sgd.W + *pi] > 0.f;
}

__global__ __launch_bounds__(256) void k_seed_count(SeedGrid sgd, const float* d, uint32_t* blk) {
  int j, i;
  const bool ok = seed_valid(sgd, d, (long)blockIdx.x * 256 + threadIdx.x, &j, &i);
  const int c = __syncthreads_count(ok);
  if (threadIdx.x == 0) blk[blockIdx.x] = (uint32_t)c;
}

__global__ __launch_bounds__(256) void k_seed_write(SeedGrid sgd, const float* d,
                                                    const float* col, const float* vm,
                                                    const float* intr, float opac_logit,
                                                    long max_out, const uint32_t* blk, float* m,
                                                    float* ls, float* q, float* o, float* c) {
  __shared__ uint32_t wc[4];
  int j = 0, i = 0;
  const bool ok = seed_valid(sgd, d, (long)blockIdx.x * 256 + threadIdx.x, &j, &i);
  const unsigned long long bal = __ballot(ok);
  const int lane = lane_id(), w = threadIdx.x >> 6;
  if (lane == 0) wc[w] = (uint32_t)__popcll(bal);
  __syncthreads();
  if (!ok) return;
  long pos = blk[blockIdx.x] + __popcll(bal & ((1ull << lane) - 1ull));
  for (int k = 0; k < w; ++k) pos += wc[k];
  if (pos >= max_out) return;
  const float fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
  const float ifx = 1.f / fx, ify = 1.f / fy;
  const int W = sgd.W, H = sgd.H, s = sgd.stride;
  const float z = d[(size_t)j * W + i];
  const float xi = ((float)i + 0.5f - cx) * ifx, yj = ((float)j + 0.5f - cy) * ify;
  // mean distance to the grid neighbours with positive depth; a neighbour's
  // offset is (z' - z) ray' + z (ray' - ray), the ray step being s / f
  float sum = 0.f;
  int cnt = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int dj = e < 2 ? 0 : (e == 2 ? -s : s), di = e < 2 ? (e == 0 ? -s : s) : 0;
    const int jj = j + dj, ii = i + di;
    if (jj < 0 || jj >= H || ii < 0 || ii >= W) continue;
    const float zn = d[(size_t)jj * W + ii];
    if (!(zn > 0.f)) continue;
    const float xn = ((float)ii + 0.5f - cx) * ifx, yn = ((float)jj + 0.5f - cy) * ify;
    const float dz = zn - z;
    const float ox = dz * xn + z * ((float)di * ifx), oy = dz * yn + z * ((float)dj * ify);
    sum += sqrtf(ox * ox + oy * oy + dz * dz);
    ++cnt;
  }
  const float sc = cnt ? sum / (float)cnt : z * (float)s * ifx;
  const float p0 = z * xi - vm[3], p1 = z * yj - vm[7], p2 = z - vm[11];
#pragma unroll
  for (int a = 0; a < 3; ++a) m[3 * pos + a] = vm[a] * p0 + vm[4 + a] * p1 + vm[8 + a] * p2;
  const float lsc = logf(sc);
  ls[3 * pos] = lsc;
  ls[3 * pos + 1] = lsc;
  ls[3 * pos + 2] = lsc;
  *reinterpret_cast<float4*>(q + 4 * pos) = make_float4(1.f, 0.f, 0.f, 0.f);
  o[pos] = opac_logit;
  const size_t HW = (size_t)H * W, px = (size_t)j * W + i;
  c[3 * pos] = col[px];
  c[3 * pos + 1] = col[HW + px];
  c[3 * pos + 2] = col[2 * HW + px];
}

// ------------------------------------------------- allocation-free seeding
// Block counts of gsr_seed_noalloc: one word per 256 grid points plus the
// total, at most SEED_NOALLOC_MAX_POINTS points.  Every GPU the library runs
// on holds its own copy until the process ends; every call on a GPU shares
// it, so calls that overlap on one GPU race.  Nothing in it needs clearing:
// the count kernel writes every word the scan reads.
static __device__ __align__(256) uint32_t scratch[SEED_NOALLOC_MAX_POINTS / 256 + 64];

// Device address of `scratch` on the current device, looked up once per
// device with that device current (the array's name is a host-side stand-in
// in host code and must never reach a kernel).
hipError_t seed_scratch(uint32_t** out) {
  static std::mutex mu;
  static uint32_t* addr[GSR_MAX_DEVICES] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= GSR_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = (uint32_t*)p;
  }
  *out = addr[dev];
  return hipSuccess;
}

// The grid total (blk[nb] after the scan) as a device int64.
__global__ void k_seed_total(const uint32_t* blk, int nb, int64_t* n_out) {
  if (threadIdx.x == 0) n_out[0] = (int64_t)blk[nb];
}

hipError_t launch_seed_total(const uint32_t* blk, int nb, int64_t* n_out, hipStream_t s) {
  hipLaunchKernelGGL(k_seed_total, dim3(1), dim3(64), 0, s, blk, nb, n_out);
  return hipGetLastError();
}

hipError_t launch_seed(int W, int H, int stride, const float* depth, const float* color,
                       const float* vm, const float* intr, float opac_logit, long max_out,
                       uint32_t* blk, float* m, float* ls, float* q, float* o, float* c,
                       hipStream_t s) {
  SeedGrid g;
  g.W = W;
  g.H = H;
  g.stride = stride;
  g.gw = (W + stride - 1) / stride;
  g.m = (long)g.gw * ((H + stride - 1) / stride);
  const int nb = (int)((g.m + 255) / 256);
  hipLaunchKernelGGL(k_seed_count, dim3(nb), dim3(256), 0, s, g, depth, blk);
  hipError_t e = launch_block_scan(nb, blk, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_seed_write, dim3(nb), dim3(256), 0, s, g, depth, color, vm, intr,
                     opac_logit, max_out, blk, m, ls, q, o, c);
  return hipGetLastError();
}

}  // namespace gsr
