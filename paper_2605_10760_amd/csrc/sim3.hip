// Sim(3) correction of Gaussian sets and the lift of keyframe poses into the
// global frame (Sec. III-C, Eq. (gauss_update); Sec. III-B, Eq. (mapgba_lift)).
//
// A similarity is stored as 8 floats (s, qw, qx, qy, qz, tx, ty, tz).  Each
// Gaussian of set k moves by sims[k]: mean -> s R mean + t, log-scales +
// ln s, rotation q -> q_R * q (Hamilton product); opacity and colour stay.
// A keyframe [Rk | tk] of set k becomes [Rk R^T | s tk - Rk R^T t], the rigid
// form of Tk o C^{-1} (the camera's length unit scaled by s).  One thread per
// Gaussian or view; the products run in FP64 and are rounded once.
// Elementwise: 40 B read and 40 B written per Gaussian.
#include "common.h"

namespace gsr {

struct Sim3 {
  double s, R[3][3], q[4], t[3];
};

__device__ __forceinline__ Sim3 load_sim3(const float* p) {
  Sim3 c;
  c.s = p[0];
  double w = p[1], x = p[2], y = p[3], z = p[4];
  const double n = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  w *= n; x *= n; y *= n; z *= n;
  c.q[0] = w; c.q[1] = x; c.q[2] = y; c.q[3] = z;
  c.R[0][0] = 1 - 2 * (y * y + z * z); c.R[0][1] = 2 * (x * y - w * z); c.R[0][2] = 2 * (x * z + w * y);
  c.R[1][0] = 2 * (x * y + w * z); c.R[1][1] = 1 - 2 * (x * x + z * z); c.R[1][2] = 2 * (y * z - w * x);
  c.R[2][0] = 2 * (x * z - w * y); c.R[2][1] = 2 * (y * z + w * x); c.R[2][2] = 1 - 2 * (x * x + y * y);
  c.t[0] = p[5]; c.t[1] = p[6]; c.t[2] = p[7];
  return c;
}

__global__ __launch_bounds__(256) void k_sim3_gaussians(SimSetTab tab, const float* m_in,
                                                        const float* ls_in, const float* q_in,
                                                        const float* sims, float* m_out,
                                                        float* ls_out, float* q_out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= tab.off[tab.ns]) return;
  int lo = 0, hi = tab.ns;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (tab.off[mid] <= i) lo = mid; else hi = mid;
  }
  const Sim3 c = load_sim3(sims + 8 * lo);
  const double m[3] = {m_in[3 * i], m_in[3 * i + 1], m_in[3 * i + 2]};
  const double ls[3] = {ls_in[3 * i], ls_in[3 * i + 1], ls_in[3 * i + 2]};
  const float4 qf = *reinterpret_cast<const float4*>(q_in + 4 * i);
  const double w2 = qf.x, x2 = qf.y, y2 = qf.z, z2 = qf.w;
  const double w1 = c.q[0], x1 = c.q[1], y1 = c.q[2], z1 = c.q[3];
  const double lns = log(c.s);
  for (int r = 0; r < 3; ++r) {
    m_out[3 * i + r] = (float)(c.s * (c.R[r][0] * m[0] + c.R[r][1] * m[1] + c.R[r][2] * m[2]) + c.t[r]);
    ls_out[3 * i + r] = (float)(ls[r] + lns);
  }
  *reinterpret_cast<float4*>(q_out + 4 * i) =
      make_float4((float)(w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2),
                  (float)(w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2),
                  (float)(w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2),
                  (float)(w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2));
}

__global__ void k_sim3_views(SimViewTab tab, const float* vin, const float* sims, float* vout) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= tab.nv) return;
  const Sim3 c = load_sim3(sims + 8 * tab.view_set[v]);
  double Rk[3][3], tk[3];
  for (int r = 0; r < 3; ++r) {
    for (int j = 0; j < 3; ++j) Rk[r][j] = vin[12 * v + 4 * r + j];
    tk[r] = vin[12 * v + 4 * r + 3];
  }
  double M[3][3];  // Rk R^T
  for (int r = 0; r < 3; ++r)
    for (int j = 0; j < 3; ++j)
      M[r][j] = Rk[r][0] * c.R[j][0] + Rk[r][1] * c.R[j][1] + Rk[r][2] * c.R[j][2];
  for (int r = 0; r < 3; ++r) {
    for (int j = 0; j < 3; ++j) vout[12 * v + 4 * r + j] = (float)M[r][j];
    vout[12 * v + 4 * r + 3] =
        (float)(c.s * tk[r] - (M[r][0] * c.t[0] + M[r][1] * c.t[1] + M[r][2] * c.t[2]));
  }
}

hipError_t launch_sim3_gaussians(const SimSetTab& tab, const float* m_in, const float* ls_in,
                                 const float* q_in, const float* sims, float* m_out,
                                 float* ls_out, float* q_out, hipStream_t s) {
  const long n = tab.off[tab.ns];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sim3_gaussians, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab,
                     m_in, ls_in, q_in, sims, m_out, ls_out, q_out);
  return hipGetLastError();
}

hipError_t launch_sim3_views(const SimViewTab& tab, const float* vin, const float* sims,
                             float* vout, hipStream_t s) {
  hipLaunchKernelGGL(k_sim3_views, dim3((tab.nv + 63) / 64), dim3(64), 0, s, tab, vin, sims, vout);
  return hipGetLastError();
}

}  // namespace gsr
