// Projection of (view, Gaussian) pairs, visible-pair compaction and the
// pose-delta update.
//
// Key pass: one thread per Gaussian, looping over the views of its set; each
// pair evaluates the key path in FP32 with no fused multiply-add and a fixed
// operation order (it decides culling, the tile rectangle and the depth key
// and must match an FP32 re-evaluation bit for bit) and writes a 4-byte key,
// with one visible count per 256-pair block for the ordered compaction that
// follows.  Record pass: for visible pairs, the rect again and the
// screen-space record in FP64 rounded once to FP32 (the 2D conic of an
// elongated splat loses digits to cancellation in FP32), one pair per lane
// from a per-wave queue of the wave's visible pairs.  The parameters are
// read once per Gaussian in each pass (coalesced AoS rows); the record pass
// writes one 48-byte record and one 8-byte rect per visible pair.
#include <algorithm>

#include "common.h"

namespace gsr {

// Real spherical harmonic normalisation constants (Condon-Shortley phase):
// 1/(2 sqrt(pi)), sqrt(3/(4 pi)), sqrt(15/pi)/2, sqrt(5/pi)/4, sqrt(15/pi)/4,
// sqrt(35/(2 pi))/4, sqrt(105/pi)/2, sqrt(21/(2 pi))/4, sqrt(7/pi)/4,
// sqrt(105/pi)/4.
#define SHK0 0.28209479177387814f
#define SHK1 0.4886025119029199f
#define SHK2A 1.0925484305920792f
#define SHK2B 0.31539156525252005f
#define SHK2C 0.5462742152960396f
#define SHK3A 0.5900435899266435f
#define SHK3B 2.890611442640554f
#define SHK3C 0.4570457994644658f
#define SHK3D 0.3731763325901154f
#define SHK3E 1.445305721320277f

// Basis values Y[k], k < (D+1)^2, at a unit direction.
template <int D>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float* Y) {
  Y[0] = SHK0;
  if (D >= 1) { Y[1] = -SHK1 * y; Y[2] = SHK1 * z; Y[3] = -SHK1 * x; }
  if (D >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SHK2A * x * y; Y[5] = -SHK2A * y * z; Y[6] = SHK2B * (2.f * zz - xx - yy);
    Y[7] = -SHK2A * x * z; Y[8] = SHK2C * (xx - yy);
    if (D >= 3) {
      Y[9] = -SHK3A * y * (3.f * xx - yy);
      Y[10] = SHK3B * x * y * z;
      Y[11] = -SHK3C * y * (4.f * zz - xx - yy);
      Y[12] = SHK3D * z * (2.f * zz - 3.f * xx - 3.f * yy);
      Y[13] = -SHK3C * x * (4.f * zz - xx - yy);
      Y[14] = SHK3E * z * (xx - yy);
      Y[15] = -SHK3A * x * (xx - 3.f * yy);
    }
  }
}

// Camera-space depth of a mean, in the key path's FP32 order.
__device__ __forceinline__ float cam_depth32(const float* m, const float* Rc, const float* tc) {
#pragma clang fp contract(off)
  return ((Rc[6] * m[0] + Rc[7] * m[1]) + Rc[8] * m[2]) + tc[2];
}

struct KeyResult {
  float p2;
  uint32_t x0, y0, x1, y1;
};

// The FP32 key path.  Every +, -, *, / and sqrt is one IEEE FP32 operation
// in the order written (contraction disabled); exp and log run in FP64 on
// the FP32 inputs and are rounded once.  The part that depends on the
// Gaussian alone (3D covariance, opacity threshold) is evaluated once per
// Gaussian; the part that depends on the view once per pair.
struct KeyGauss {
  float S00, S01, S02, S11, S12, S22;  // 3D covariance
  float k2;                            // 2 ln(255 sigma)
  bool ok;                             // unit quaternion defined, 255 sigma > 1
};

__device__ __forceinline__ KeyGauss key_gauss(const float* ls, const float* q, float o) {
#pragma clang fp contract(off)
  KeyGauss g;
  const float s0 = (float)exp((double)ls[0]);
  const float s1 = (float)exp((double)ls[1]);
  const float s2 = (float)exp((double)ls[2]);
  const float qn = sqrtf(((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3]);
  const float w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  const float R00 = 1.f - 2.f * (yy + zz), R01 = 2.f * (xy - wz), R02 = 2.f * (xz + wy);
  const float R10 = 2.f * (xy + wz), R11 = 1.f - 2.f * (xx + zz), R12 = 2.f * (yz - wx);
  const float R20 = 2.f * (xz - wy), R21 = 2.f * (yz + wx), R22 = 1.f - 2.f * (xx + yy);
  const float M00 = R00 * s0, M01 = R01 * s1, M02 = R02 * s2;
  const float M10 = R10 * s0, M11 = R11 * s1, M12 = R12 * s2;
  const float M20 = R20 * s0, M21 = R21 * s1, M22 = R22 * s2;
  g.S00 = (M00 * M00 + M01 * M01) + M02 * M02;
  g.S01 = (M00 * M10 + M01 * M11) + M02 * M12;
  g.S02 = (M00 * M20 + M01 * M21) + M02 * M22;
  g.S11 = (M10 * M10 + M11 * M11) + M12 * M12;
  g.S12 = (M10 * M20 + M11 * M21) + M12 * M22;
  g.S22 = (M20 * M20 + M21 * M21) + M22 * M22;
  const float sigma = (float)(1.0 / (1.0 + exp(-(double)o)));
  const double t = 255.0 * (double)sigma;
  g.ok = qn > 0.f && t > 1.0;
  g.k2 = g.ok ? (float)(2.0 * log(t)) : 0.f;
  return g;
}

// Returns false when the pair is culled.
__device__ __forceinline__ bool key_view(const float* m, const KeyGauss& g, const float* Rc,
                                         const float* tc, float fx, float fy, float cx, float cy,
                                         int W, int H, int TW, int TH, int TX, int TY,
                                         float z_near, KeyResult& kr) {
#pragma clang fp contract(off)
  const float p0 = ((Rc[0] * m[0] + Rc[1] * m[1]) + Rc[2] * m[2]) + tc[0];
  const float p1 = ((Rc[3] * m[0] + Rc[4] * m[1]) + Rc[5] * m[2]) + tc[1];
  const float p2 = cam_depth32(m, Rc, tc);
  if (!(p2 > z_near) || !g.ok) return false;
  const float S[3][3] = {{g.S00, g.S01, g.S02}, {g.S01, g.S11, g.S12}, {g.S02, g.S12, g.S22}};
  float Wm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      Wm[i][k] = (Rc[3 * i] * S[0][k] + Rc[3 * i + 1] * S[1][k]) + Rc[3 * i + 2] * S[2][k];
  float V[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j)
      V[i][j] = (Wm[i][0] * Rc[3 * j] + Wm[i][1] * Rc[3 * j + 1]) + Wm[i][2] * Rc[3 * j + 2];
  const float rx = p0 / p2, ry = p1 / p2;
  const float u = fx * rx + cx;
  const float v = fy * ry + cy;
  const float limx = 1.3f * ((0.5f * (float)W) / fx);
  const float limy = 1.3f * ((0.5f * (float)H) / fy);
  const float rxc = rx < -limx ? -limx : (rx > limx ? limx : rx);
  const float ryc = ry < -limy ? -limy : (ry > limy ? limy : ry);
  const float j00 = fx / p2, j02 = -(fx * rxc) / p2;
  const float j11 = fy / p2, j12 = -(fy * ryc) / p2;
  const float T00 = j00 * V[0][0] + j02 * V[0][2];
  const float T01 = j00 * V[0][1] + j02 * V[1][2];
  const float T02 = j00 * V[0][2] + j02 * V[2][2];
  const float T11 = j11 * V[1][1] + j12 * V[1][2];
  const float T12 = j11 * V[1][2] + j12 * V[2][2];
  const float a = (T00 * j00 + T02 * j02) + 0.3f;
  const float b = T01 * j11 + T02 * j12;
  const float c = (T11 * j11 + T12 * j12) + 0.3f;
  const float det = a * c - b * b;
  if (!(det > 0.f)) return false;
  const float ex = sqrtf(g.k2 * a);
  const float ey = sqrtf(g.k2 * c);
  if (!(isfinite(u) && isfinite(v) && isfinite(ex) && isfinite(ey))) return false;
  const float itw = 1.0f / (float)TW, ith = 1.0f / (float)TH;
  const float fX = (float)TX, fY = (float)TY;
  float fx0 = floorf((u - ex) * itw);
  float fx1 = floorf((u + ex) * itw) + 1.f;
  float fy0 = floorf((v - ey) * ith);
  float fy1 = floorf((v + ey) * ith) + 1.f;
  fx0 = fx0 < 0.f ? 0.f : (fx0 > fX ? fX : fx0);
  fx1 = fx1 < 0.f ? 0.f : (fx1 > fX ? fX : fx1);
  fy0 = fy0 < 0.f ? 0.f : (fy0 > fY ? fY : fy0);
  fy1 = fy1 < 0.f ? 0.f : (fy1 > fY ? fY : fy1);
  kr.x0 = (uint32_t)fx0; kr.x1 = (uint32_t)fx1;
  kr.y0 = (uint32_t)fy0; kr.y1 = (uint32_t)fy1;
  if (kr.x1 <= kr.x0 || kr.y1 <= kr.y0) return false;
  kr.p2 = p2;
  return true;
}

// Key pass: one thread per Gaussian of a rendered set; it projects its
// Gaussian into every view of the set in turn (views are uniform across the
// workgroup, whose Gaussians all belong to one set).  The parameters are read
// once and the view-independent part of the key path (3D covariance,
// opacity threshold) is done once, instead of once per view.  Pair p of view
// v is Gaussian p - pair_off[v] of the set, so the workgroup's 256 Gaussians
// are the 256-pair block (blk_off[v] + its block index in the set) of each
// view.  Writes the depth key (or CULLED) of every pair and the visible
// count of every 256-pair block, for the ordered compaction that follows.
__global__ __launch_bounds__(PROJ_BLOCK) void k_project(ProjTab t, SceneDev sc, CamDev cam,
                                                        StateDev st, uint32_t* blk_cnt) {
  const int b = xcd_remap(blockIdx.x, t.set_gblk[t.ns]);
  if (b < 0) return;
  const int s = find_seg(t.set_gblk, t.ns, b);
  const int lb = b - t.set_gblk[s];
  const int local = lb * PROJ_BLOCK + (int)threadIdx.x;
  const bool valid = local < t.set_goff[s + 1] - t.set_goff[s];
  const long gi = (long)t.set_goff[s] + (valid ? local : 0);
  float m[3] = {0.f, 0.f, 0.f}, ls[3] = {0.f, 0.f, 0.f}, q[4] = {1.f, 0.f, 0.f, 0.f}, o = 0.f;
  if (valid) {
    m[0] = sc.means[3 * gi]; m[1] = sc.means[3 * gi + 1]; m[2] = sc.means[3 * gi + 2];
    ls[0] = sc.log_scales[3 * gi]; ls[1] = sc.log_scales[3 * gi + 1];
    ls[2] = sc.log_scales[3 * gi + 2];
    const float4 q4 = *reinterpret_cast<const float4*>(sc.quats + 4 * gi);
    q[0] = q4.x; q[1] = q4.y; q[2] = q4.z; q[3] = q4.w;
    o = sc.opac[gi];
  }
  KeyGauss kg = key_gauss(ls, q, o);
  kg.ok = kg.ok && valid;
  for (int vi = t.set_voff[s]; vi < t.set_voff[s + 1]; ++vi) {
    const int v = t.vset[vi];
    const int pair = t.pair_off[v] + local;
    const float* vm = cam.viewmats + 12 * v;
    const float Rc[9] = {vm[0], vm[1], vm[2], vm[4], vm[5], vm[6], vm[8], vm[9], vm[10]};
    const float tc[3] = {vm[3], vm[7], vm[11]};
    const float4 in = *reinterpret_cast<const float4*>(cam.intrinsics + 4 * v);
    KeyResult kr;
    const bool vis = key_view(m, kg, Rc, tc, in.x, in.y, in.z, in.w, t.W, t.H, t.TW, t.TH, t.TX,
                              t.TY, cam.z_near, kr);
    if (valid) st.zkey[pair] = vis ? __float_as_uint(kr.p2) : CULLED;
    const int cnt = __syncthreads_count(vis);
    if (threadIdx.x == 0) blk_cnt[t.blk_off[v] + lb] = (uint32_t)cnt;
  }
}

// Record pass (after the compaction): for every visible pair, the tile rect
// (the key path again, same code and inputs, so the same rect) and the FP64
// screen-space record, written at the pair's position in the compacted
// visible list, so that a view's records are consecutive lines (written in
// full, read densely by the binning and compositing).
//
// One wave per 64 Gaussians of a set.  Each lane loads its Gaussian once and
// puts the view-independent quantities (mean, FP32 key covariance and
// threshold, FP64 covariance, opacity, threshold of the record extents,
// degree-0 colour) in the wave's LDS slot.  The wave then walks the set's
// views, appending its visible pairs (lane, view) to a queue in LDS, and
// computes records 64 at a time from the queue, one pair per lane, so that
// no lane idles on a culled pair.
constexpr int RQ = 128;  // queue slots per wave (at most 63 + 64 held)
struct RecSlot {
  float m[3][64];
  float S[6][64];      // FP32 key-path covariance
  float k2[64];        // key-path 2 ln(255 sigma), negative: not renderable
  double Sd[6][64];    // FP64 covariance (00, 01, 02, 11, 12, 22)
  float sig[64], k2f[64];
  float col[3][64];
  uint32_t item[RQ], row[RQ];
};

template <int SHD>
__device__ __forceinline__ void record_one(const ProjTab& t, const SceneDev& sc,
                                           const CamDev& cam, const StateDev& st,
                                           const RecSlot& L, long g0, uint32_t item,
                                           uint32_t row) {
  const int l = (int)(item & 63u), v = (int)(item >> 6);
  const float m[3] = {L.m[0][l], L.m[1][l], L.m[2][l]};
  KeyGauss kg;
  kg.S00 = L.S[0][l]; kg.S01 = L.S[1][l]; kg.S02 = L.S[2][l];
  kg.S11 = L.S[3][l]; kg.S12 = L.S[4][l]; kg.S22 = L.S[5][l];
  kg.k2 = L.k2[l];
  kg.ok = true;  // visible in the key pass
  const float* vm = cam.viewmats + 12 * v;
  const float Rc[9] = {vm[0], vm[1], vm[2], vm[4], vm[5], vm[6], vm[8], vm[9], vm[10]};
  const float tc[3] = {vm[3], vm[7], vm[11]};
  const float4 in = *reinterpret_cast<const float4*>(cam.intrinsics + 4 * v);
  KeyResult kr;
  // visible in the key pass, so visible here (the same pure function of the
  // same inputs); an empty rect would only drop the pair
  if (!key_view(m, kg, Rc, tc, in.x, in.y, in.z, in.w, t.W, t.H, t.TW, t.TH, t.TX, t.TY,
                cam.z_near, kr))
    kr.x0 = kr.x1 = kr.y0 = kr.y1 = 0u;
  st.rect[row] = make_uint2(kr.x0 | (kr.y0 << 16), kr.x1 | (kr.y1 << 16));
  double Sd[3][3];
  Sd[0][0] = L.Sd[0][l]; Sd[0][1] = Sd[1][0] = L.Sd[1][l]; Sd[0][2] = Sd[2][0] = L.Sd[2][l];
  Sd[1][1] = L.Sd[3][l]; Sd[1][2] = Sd[2][1] = L.Sd[4][l]; Sd[2][2] = L.Sd[5][l];
  ScreenCov sc2 = screen_cov_fp64(Sd, Rc, tc, m, in.x, in.y, t.W, t.H);
  const double fx = in.x, fy = in.y;
  const double* p = sc2.p;
  const double rx = sc2.rx, ry = sc2.ry;
  const double a = sc2.a, bb = sc2.b, c = sc2.c;
  const double det = a * c - bb * bb;
  const double u = fx * rx + (double)in.z, vv = fy * ry + (double)in.w;
  float cv[3] = {L.col[0][l], L.col[1][l], L.col[2][l]};
  if (SHD > 0) {
    // camera centre o_cam = -Rc^T tc; direction d = (mu - o_cam)/|mu - o_cam|
    const float ox = -(Rc[0] * tc[0] + Rc[3] * tc[1] + Rc[6] * tc[2]);
    const float oy = -(Rc[1] * tc[0] + Rc[4] * tc[1] + Rc[7] * tc[2]);
    const float oz = -(Rc[2] * tc[0] + Rc[5] * tc[1] + Rc[8] * tc[2]);
    float dx = m[0] - ox, dy = m[1] - oy, dz = m[2] - oz;
    const float inv = 1.f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= inv; dy *= inv; dz *= inv;
    constexpr int NB = (SHD + 1) * (SHD + 1);
    float Y[16];
    sh_eval<SHD>(dx, dy, dz, Y);
    const float* k = sc.colors + (long)3 * sc.sh_stride * (g0 + l);
    float r = 0.5f, g = 0.5f, bl = 0.5f;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      r += Y[i] * k[3 * i]; g += Y[i] * k[3 * i + 1]; bl += Y[i] * k[3 * i + 2];
    }
    cv[0] = fmaxf(r, 0.f); cv[1] = fmaxf(g, 0.f); cv[2] = fmaxf(bl, 0.f);
  }
  const float k2f = L.k2f[l];
  const float exr = sqrtf(k2f * (float)a) * (1.f + 1e-4f) + 1e-2f;
  const float eyr = sqrtf(k2f * (float)c) * (1.f + 1e-4f) + 1e-2f;
  float4* rp = st.rec + 3 * (long)row;
  // conic (A, B, C) = (c, -b, a)/det, stored pre-scaled so that the exponent
  // in base 2 is A' dx^2 + B' dx dy + C' dy^2:
  // A' = -A log2(e)/2, B' = -B log2(e), C' = -C log2(e)/2
  const double L2E = 1.4426950408889634;
  const double h = L2E / det;
  rp[0] = make_float4((float)u, (float)vv, (float)(-0.5 * h * c), (float)(h * bb));
  rp[1] = make_float4((float)(-0.5 * h * a), L.sig[l], (float)p[2], exr);
  rp[2] = make_float4(cv[0], cv[1], cv[2], eyr);
}

template <int SHD>
__global__ __launch_bounds__(PROJ_BLOCK) void k_records(ProjTab t, SceneDev sc, CamDev cam,
                                                        StateDev st) {
  __shared__ RecSlot slots[PROJ_BLOCK / 64];
  const int b = xcd_remap(blockIdx.x, t.set_gblk[t.ns]);
  if (b < 0) return;
  const int s = find_seg(t.set_gblk, t.ns, b);
  const int lb = b - t.set_gblk[s];
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  RecSlot& L = slots[wv];
  const int local = lb * PROJ_BLOCK + (int)threadIdx.x;
  const bool valid = local < t.set_goff[s + 1] - t.set_goff[s];
  const long gi = (long)t.set_goff[s] + (valid ? local : 0);
  const long g0 = (long)t.set_goff[s] + lb * PROJ_BLOCK + 64 * wv;  // the wave's lane-0 Gaussian
  {
    float m[3] = {0.f, 0.f, 0.f}, ls[3] = {0.f, 0.f, 0.f}, q[4] = {1.f, 0.f, 0.f, 0.f}, o = 0.f;
    if (valid) {
      m[0] = sc.means[3 * gi]; m[1] = sc.means[3 * gi + 1]; m[2] = sc.means[3 * gi + 2];
      ls[0] = sc.log_scales[3 * gi]; ls[1] = sc.log_scales[3 * gi + 1];
      ls[2] = sc.log_scales[3 * gi + 2];
      const float4 q4 = *reinterpret_cast<const float4*>(sc.quats + 4 * gi);
      q[0] = q4.x; q[1] = q4.y; q[2] = q4.z; q[3] = q4.w;
      o = sc.opac[gi];
    }
    const KeyGauss kg = key_gauss(ls, q, o);
    // ---- view-independent part of the FP64 record.  Scales, rotation and
    // opacity are formed in FP32 first: their rounding perturbs the
    // parameters by ~1e-7 relative, while the products, where elongated
    // splats cancel, run in FP64.
    double Sd[3][3];
    cov3_fp64(ls, q, Sd);
    const float sigf = 1.f / (1.f + expf(-o));
    // half-extents of the alpha >= 1/255 ellipse use k2f, widened by a
    // margin far above FP32 rounding: every pixel outside that box has
    // alpha < 1/255, so the compositing kernels may skip the splat there
    // without changing any result
    const float t255 = 255.f * sigf;
    L.m[0][lane] = m[0]; L.m[1][lane] = m[1]; L.m[2][lane] = m[2];
    L.S[0][lane] = kg.S00; L.S[1][lane] = kg.S01; L.S[2][lane] = kg.S02;
    L.S[3][lane] = kg.S11; L.S[4][lane] = kg.S12; L.S[5][lane] = kg.S22;
    L.k2[lane] = kg.k2;
    L.Sd[0][lane] = Sd[0][0]; L.Sd[1][lane] = Sd[0][1]; L.Sd[2][lane] = Sd[0][2];
    L.Sd[3][lane] = Sd[1][1]; L.Sd[4][lane] = Sd[1][2]; L.Sd[5][lane] = Sd[2][2];
    L.sig[lane] = sigf;
    L.k2f[lane] = t255 > 1.f ? 2.f * logf(t255) : 0.f;
    float col[3] = {0.f, 0.f, 0.f};
    if (SHD == 0 && valid) {
      col[0] = sc.colors[3 * gi]; col[1] = sc.colors[3 * gi + 1]; col[2] = sc.colors[3 * gi + 2];
    }
    L.col[0][lane] = col[0]; L.col[1][lane] = col[1]; L.col[2][lane] = col[2];
  }
  uint32_t head = 0u, tail = 0u;
  for (int vi = t.set_voff[s]; vi < t.set_voff[s + 1]; ++vi) {
    const int v = t.vset[vi];
    const uint32_t row = valid ? st.vidx[t.pair_off[v] + local] : CULLED;
    const bool vis = row != CULLED;
    const unsigned long long mk = __ballot(vis);
    if (vis) {
      const uint32_t k = (tail + __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u))) &
                         (RQ - 1);
      L.item[k] = (uint32_t)lane | ((uint32_t)v << 6);
      L.row[k] = row;
    }
    tail += (uint32_t)__popcll(mk);
    __builtin_amdgcn_wave_barrier();
    if (tail - head >= 64u) {
      const uint32_t k = (head + (uint32_t)lane) & (RQ - 1);
      record_one<SHD>(t, sc, cam, st, L, g0, L.item[k], L.row[k]);
      head += 64u;
      __builtin_amdgcn_wave_barrier();
    }
  }
  if ((uint32_t)lane < tail - head) {
    const uint32_t k = (head + (uint32_t)lane) & (RQ - 1);
    record_one<SHD>(t, sc, cam, st, L, g0, L.item[k], L.row[k]);
  }
}

// Exclusive scan of the per-block visible counts and the per-view offsets
// of the compacted, view-major visible-pair list, over ceil(nb / 4096)
// workgroups: workgroup b scans tile b after summing every count before it,
// writes the offset of each view whose first block falls in its tile, and
// the last workgroup writes the total.
constexpr int SB_TILE = 4096;  // 1024 threads x 4 counts
__global__ __launch_bounds__(1024) void k_scan_blocks(ProjTab t, const uint32_t* blk,
                                                     uint32_t* scan, StateHeader* hdr) {
  __shared__ unsigned long long sh[17];
  const int nb = t.blk_off[t.nv];
  const int base = (int)blockIdx.x * SB_TILE;
  const unsigned long long carry = wg_sum_before<1024>(blk, base, sh);
  const int i0 = base + 4 * (int)threadIdx.x;
  uint32_t x[4];
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = (i0 + k < nb) ? blk[i0 + k] : 0u;
    s += x[k];
  }
  unsigned long long tot;
  unsigned long long pre = wg_excl_scan<1024>(s, sh, &tot) + carry;
  // the prefix goes to its own array: later workgroups still read the counts
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i0 + k < nb) scan[i0 + k] = (uint32_t)pre;
    pre += x[k];
  }
  const bool last = blockIdx.x == gridDim.x - 1;
  const unsigned long long all = carry + tot;
  if (last && threadIdx.x == 0) {
    hdr->vis_total = (uint32_t)all;
    hdr->vis_off[t.nv] = (uint32_t)all;
  }
  __syncthreads();
  // view offsets: the scanned value of the view's first block, or the total
  // for views whose blocks start at nb (empty views at the end)
  for (int v = threadIdx.x; v < t.nv; v += 1024) {
    const int f = t.blk_off[v];
    if (f >= base && f < base + SB_TILE && f < nb) hdr->vis_off[v] = scan[f];
    else if (f >= nb && last) hdr->vis_off[v] = (uint32_t)all;
  }
}

// Ordered compaction: visible pairs keep their (view-major, id) order.  A
// workgroup takes CP_SUB consecutive 256-pair blocks (their keys loaded
// together, then compacted block by block).
constexpr int CP_SUB = 4;
__global__ __launch_bounds__(PROJ_BLOCK) void k_compact(ProjTab t, StateDev st,
                                                        const uint32_t* blk_scan,
                                                        uint32_t* kout) {
  const int nb = t.blk_off[t.nv];
  const int g = xcd_remap(blockIdx.x, (nb + CP_SUB - 1) / CP_SUB);
  if (g < 0) return;
  __shared__ int wc[CP_SUB][PROJ_BLOCK / 64];
  const int lane = lane_id(), w = threadIdx.x >> 6;
  uint32_t key[CP_SUB];
  int pair[CP_SUB];
  bool in[CP_SUB];
#pragma unroll
  for (int k = 0; k < CP_SUB; ++k) {
    const int b = g * CP_SUB + k;
    in[k] = false;
    key[k] = CULLED;
    pair[k] = 0;
    if (b < nb) {
      const int v = find_seg(t.blk_off, t.nv, b);
      const int local = (b - t.blk_off[v]) * PROJ_BLOCK + (int)threadIdx.x;
      pair[k] = t.pair_off[v] + local;
      in[k] = local < t.pair_off[v + 1] - t.pair_off[v];
      if (in[k]) key[k] = st.zkey[pair[k]];
    }
  }
  unsigned long long m[CP_SUB];
#pragma unroll
  for (int k = 0; k < CP_SUB; ++k) {
    m[k] = __ballot(key[k] != CULLED);
    if (lane == 0) wc[k][w] = __popcll(m[k]);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < CP_SUB; ++k) {
    const int b = g * CP_SUB + k;
    if (b >= nb) break;
    uint32_t pos = CULLED;
    if (key[k] != CULLED) {
      pos = blk_scan[b] + (uint32_t)__popcll(m[k] & ((1ull << lane) - 1ull));
      for (int i = 0; i < w; ++i) pos += wc[k][i];
      // the sort carries the visible position (its first pass takes each
      // key's index as its value)
      kout[pos] = key[k];
    }
    // position of the pair in the compacted visible list (the row of its
    // screen-space gradient), CULLED for culled pairs
    if (in[k]) st.vidx[pair[k]] = pos;
  }
}

// viewmats_out[v] = Exp(xi_v) [R|t] with xi = (rho, phi) (FP64 internally).
__global__ void k_pose_delta(const float* vin, const float* delta, float* vout, int nv) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const double r0 = delta[6 * v], r1 = delta[6 * v + 1], r2 = delta[6 * v + 2];
  const double w0 = delta[6 * v + 3], w1 = delta[6 * v + 4], w2 = delta[6 * v + 5];
  const double th2 = w0 * w0 + w1 * w1 + w2 * w2, th = sqrt(th2);
  double A, B, C;  // sin(th)/th, (1-cos th)/th^2, (th - sin th)/th^3
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  const double K[3][3] = {{0, -w2, w1}, {w2, 0, -w0}, {-w1, w0, 0}};
  double K2[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K2[i][j] = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
  double Rm[3][3], Vm[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double I = (i == j) ? 1.0 : 0.0;
      Rm[i][j] = I + A * K[i][j] + B * K2[i][j];
      Vm[i][j] = I + B * K[i][j] + C * K2[i][j];
    }
  const double rho[3] = {r0, r1, r2};
  double tt[3];
  for (int i = 0; i < 3; ++i) tt[i] = Vm[i][0] * rho[0] + Vm[i][1] * rho[1] + Vm[i][2] * rho[2];
  double in[3][4];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 4; ++j) in[i][j] = vin[12 * v + 4 * i + j];
  double out[3][4];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 4; ++j)
      out[i][j] = Rm[i][0] * in[0][j] + Rm[i][1] * in[1][j] + Rm[i][2] * in[2][j] +
                  (j == 3 ? tt[i] : 0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 4; ++j) vout[12 * v + 4 * i + j] = (float)out[i][j];
}

hipError_t launch_project_keys(const ProjTab& t, const SceneDev& sc, const CamDev& cam,
                               StateDev st, uint32_t* blk_cnt, hipStream_t s) {
  const int nb = t.set_gblk[t.ns];
  if (nb == 0) return hipSuccess;
  // the key path does not read colours: one kernel for every degree
  hipLaunchKernelGGL(k_project, dim3(xcd_grid(nb)), dim3(PROJ_BLOCK), 0, s, t, sc, cam, st,
                     blk_cnt);
  return hipGetLastError();
}

hipError_t launch_project_records(const ProjTab& t, const SceneDev& sc, const CamDev& cam,
                                  StateDev st, hipStream_t s) {
  const int nb = t.set_gblk[t.ns];
  if (nb == 0) return hipSuccess;
  const dim3 g(xcd_grid(nb)), b(PROJ_BLOCK);
  switch (sc.sh_degree) {
    case 0: hipLaunchKernelGGL(k_records<0>, g, b, 0, s, t, sc, cam, st); break;
    case 1: hipLaunchKernelGGL(k_records<1>, g, b, 0, s, t, sc, cam, st); break;
    case 2: hipLaunchKernelGGL(k_records<2>, g, b, 0, s, t, sc, cam, st); break;
    default: hipLaunchKernelGGL(k_records<3>, g, b, 0, s, t, sc, cam, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_compact(const ProjTab& t, StateDev st, const uint32_t* blk_cnt,
                          uint32_t* blk_scan, uint32_t* kout, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_blocks, dim3(std::max(1, (t.blk_off[t.nv] + SB_TILE - 1) / SB_TILE)),
                     dim3(1024), 0, s, t, blk_cnt, blk_scan, st.hdr);
  const int nb = t.blk_off[t.nv];
  if (nb > 0)
    hipLaunchKernelGGL(k_compact, dim3(xcd_grid((nb + CP_SUB - 1) / CP_SUB)), dim3(PROJ_BLOCK), 0,
                       s, t, st, blk_scan, kout);
  return hipGetLastError();
}

hipError_t launch_pose_delta(const float* vin, const float* delta, float* vout, int nv,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_pose_delta, dim3((nv + 63) / 64), dim3(64), 0, s, vin, delta, vout, nv);
  return hipGetLastError();
}

}  // namespace gsr
