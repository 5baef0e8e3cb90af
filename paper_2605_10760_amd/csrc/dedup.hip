// Occupancy-aware deduplication of borrowed Gaussians (Sec. III-C, Eqs.
// (envelope), (free_carve), (dedup)).
//
// One open-addressing hash set of 64-bit voxel keys (21 bits per axis,
// offset 2^20) with a flag word per slot (bit 0 occupied, bit 1 free):
//   k_dd_clear   empty every slot (a fill kernel, capturable);
//   k_dd_occ     one thread per target Gaussian inserts every voxel of its
//                box [mu - k s, mu + k s];
//   k_dd_free    one thread per keyframe pixel walks the voxels of the
//                segment from the camera centre to the back-projected depth
//                (t in [0, 1)) and inserts them, through a workgroup-local
//                LDS set that drops the repeats of neighbouring rays;
//   k_dd_probe   one thread per borrowed Gaussian looks up the voxel of its
//                mean: kept only when absent.
// Voxel indices are floor(x / v) in FP64 from the FP32 inputs; segment
// crossings are computed per plane as (plane - c) / (r - c) (no incremental
// sums) and walked in increasing t, ties to the lower axis, with no fused
// multiply-add, so every index is reproducible.  Inserts use 64-bit CAS with
// linear probing, bounded by DD_MAX_PROBE; an insert that finds no slot
// raises the overflow flag (bit 0).  Indices outside the key range (+-2^20
// voxels per axis, NaN included) or a box / segment of more than 2^22 voxels
// raise bit 1 and are skipped, so every thread's loop is bounded.
#include "common.h"

namespace gsr {

constexpr unsigned long long DD_EMPTY = ~0ull;
constexpr int DD_MAX_PROBE = 1 << 14;
constexpr long long DD_OFF = 1ll << 20;
constexpr long long DD_MAX_CELLS = 1ll << 22;  // voxels of one box or one segment

struct DedupTable {
  unsigned long long* keys;
  unsigned int* flags;
  unsigned int* counters;  // [0] overflow flag, [1] distinct voxels
  unsigned long long mask;
};

__device__ __forceinline__ unsigned long long dd_pack(long long x, long long y, long long z) {
  return (unsigned long long)((x + DD_OFF) & 0x1FFFFF) |
         ((unsigned long long)((y + DD_OFF) & 0x1FFFFF) << 21) |
         ((unsigned long long)((z + DD_OFF) & 0x1FFFFF) << 42);
}

// splitmix64 finaliser
__device__ __forceinline__ unsigned long long dd_mix(unsigned long long k) {
  k ^= k >> 30;
  k *= 0xbf58476d1ce4e5b9ull;
  k ^= k >> 27;
  k *= 0x94d049bb133111ebull;
  k ^= k >> 31;
  return k;
}

// A slot's key only ever goes from empty to its final value, so a plain
// read that already shows the key (or the flag) settles the insert without
// an atomic: many rays of one keyframe share the voxels near its camera, and
// their CASes would otherwise queue on the same slot.  A stale read of an
// empty slot falls through to the CAS, which decides.
__device__ void dd_insert(const DedupTable& T, unsigned long long key, unsigned int flag) {
  unsigned long long h = dd_mix(key) & T.mask;
  for (int probe = 0; probe < DD_MAX_PROBE && probe <= (long long)T.mask; ++probe) {
    unsigned long long cur = T.keys[h];
    if (cur == DD_EMPTY) {
      cur = atomicCAS(&T.keys[h], DD_EMPTY, key);
      if (cur == DD_EMPTY) {
        atomicAdd(&T.counters[1], 1u);
        atomicOr(&T.flags[h], flag);
        return;
      }
    }
    if (cur == key) {
      if ((T.flags[h] & flag) == 0u) atomicOr(&T.flags[h], flag);
      return;
    }
    h = (h + 1) & T.mask;
  }
  atomicOr(&T.counters[0], 1u);
}

// Workgroup-local filter in front of dd_insert: the rays of one workgroup
// (neighbouring pixels of one keyframe) cross mostly the same voxels, so a
// key goes to the global set only from the thread that first places it in
// this LDS set (bounded probing; a key that finds no LDS slot goes straight
// to the global set).  Every key still reaches the global set, once per
// workgroup at most.
constexpr int DD_LSLOTS = 4096;
constexpr int DD_LPROBE = 8;
__device__ void dd_insert_local(const DedupTable& T, unsigned long long* lk,
                                unsigned long long key, unsigned int flag) {
  unsigned int h = (unsigned int)(dd_mix(key) >> 40) & (DD_LSLOTS - 1);
  for (int probe = 0; probe < DD_LPROBE; ++probe) {
    unsigned long long cur = lk[h];
    if (cur == DD_EMPTY) {
      cur = atomicCAS(&lk[h], DD_EMPTY, key);
      if (cur == DD_EMPTY) {
        dd_insert(T, key, flag);
        return;
      }
    }
    if (cur == key) return;
    h = (h + 1) & (DD_LSLOTS - 1);
  }
  dd_insert(T, key, flag);
}

__global__ __launch_bounds__(256) void k_dd_clear(DedupTable T) {
  const unsigned long long i = (unsigned long long)blockIdx.x * 256 + threadIdx.x;
  if (i <= T.mask) {
    T.keys[i] = DD_EMPTY;
    T.flags[i] = 0u;
  }
  if (i < 2) T.counters[i] = 0u;
}

__global__ __launch_bounds__(256) void k_dd_occ(DedupTable T, const float* means,
                                                const float* log_scales, long long n, double v,
                                                double kenv) {
#pragma clang fp contract(off)
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  long long lo[3], hi[3];
  double cells = 1.0;
  for (int a = 0; a < 3; ++a) {
    const double m = means[3 * i + a];
    const double s = exp((double)log_scales[3 * i + a]);
    const double l = floor((m - kenv * s) / v), h = floor((m + kenv * s) / v);
    // indices must fit the key, and a box must stay bounded
    if (!(l > -(double)DD_OFF && h < (double)DD_OFF)) {
      atomicOr(&T.counters[0], 2u);
      return;
    }
    lo[a] = (long long)l;
    hi[a] = (long long)h;
    cells *= (double)(hi[a] - lo[a] + 1);
  }
  if (cells > (double)DD_MAX_CELLS) {
    atomicOr(&T.counters[0], 2u);
    return;
  }
  for (long long x = lo[0]; x <= hi[0]; ++x)
    for (long long y = lo[1]; y <= hi[1]; ++y)
      for (long long z = lo[2]; z <= hi[2]; ++z) dd_insert(T, dd_pack(x, y, z), 1u);
}

__global__ __launch_bounds__(256) void k_dd_free(DedupTable T, const float* depth,
                                                 const float* viewmats, const float* intr,
                                                 int W, int H, long long npix, double v) {
#pragma clang fp contract(off)
  __shared__ unsigned long long lk[DD_LSLOTS];
  for (int k = threadIdx.x; k < DD_LSLOTS; k += 256) lk[k] = DD_EMPTY;
  __syncthreads();  // the only barrier: threads may leave after it
  const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
  if (g >= npix) return;
  const int kf = (int)(g / ((long long)W * H));
  const long long p = g - (long long)kf * W * H;
  const int j = (int)(p / W), i = (int)(p - (long long)j * W);
  const double dd = depth[g];
  if (!(dd > 0.0)) return;
  const float* vm = viewmats + 12 * kf;
  double R[3][3], t[3];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) R[r][c] = vm[4 * r + c];
    t[r] = vm[4 * r + 3];
  }
  const double fx = intr[4 * kf], fy = intr[4 * kf + 1], cx = intr[4 * kf + 2],
               cy = intr[4 * kf + 3];
  const double ray[3] = {((double)i + 0.5 - cx) / fx, ((double)j + 0.5 - cy) / fy, 1.0};
  double c[3], d[3];
  long long cur[3], end[3];
  double steps = 0.0;
  for (int a = 0; a < 3; ++a) {
    c[a] = -((R[0][a] * t[0] + R[1][a] * t[1]) + R[2][a] * t[2]);
    const double r = c[a] + dd * ((R[0][a] * ray[0] + R[1][a] * ray[1]) + R[2][a] * ray[2]);
    d[a] = r - c[a];
    const double fc = floor(c[a] / v), fr = floor(r / v);
    // indices must fit the key, and a segment's walk must stay bounded
    if (!(fc > -(double)DD_OFF && fc < (double)DD_OFF && fr > -(double)DD_OFF &&
          fr < (double)DD_OFF)) {
      atomicOr(&T.counters[0], 2u);
      return;
    }
    cur[a] = (long long)fc;
    end[a] = (long long)fr;
    steps += fabs(fr - fc);
  }
  if (steps > (double)DD_MAX_CELLS) {
    atomicOr(&T.counters[0], 2u);
    return;
  }
  dd_insert_local(T, lk, dd_pack(cur[0], cur[1], cur[2]), 2u);
  // next plane index per axis (the walk stops at the end voxel's planes)
  long long nxt[3];
  int step[3];
  for (int a = 0; a < 3; ++a) {
    step[a] = d[a] > 0.0 ? 1 : -1;
    nxt[a] = d[a] > 0.0 ? cur[a] + 1 : cur[a];
  }
  for (;;) {
    int best = -1;
    double tb = 1.0;
    for (int a = 0; a < 3; ++a) {
      if (d[a] == 0.0 || cur[a] == end[a]) continue;
      const double ta = ((double)nxt[a] * v - c[a]) / d[a];
      // ta = 0: a start on the plane, moving down, leaves its voxel at once
      if (ta >= 0.0 && ta < tb) {
        tb = ta;
        best = a;
      }
    }
    if (best < 0) break;
    cur[best] += step[best];
    nxt[best] += step[best];
    dd_insert_local(T, lk, dd_pack(cur[0], cur[1], cur[2]), 2u);
  }
}

__global__ __launch_bounds__(256) void k_dd_probe(DedupTable T, const float* means, long long n,
                                                  double v, uint8_t* keep) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  long long q[3];
  for (int a = 0; a < 3; ++a) {
    const double f = floor((double)means[3 * i + a] / v);
    if (!(f > -(double)DD_OFF && f < (double)DD_OFF)) {
      atomicOr(&T.counters[0], 2u);
      keep[i] = 0;
      return;
    }
    q[a] = (long long)f;
  }
  const unsigned long long key = dd_pack(q[0], q[1], q[2]);
  unsigned long long h = dd_mix(key) & T.mask;
  bool found = false;
  for (long long probe = 0; probe <= (long long)T.mask; ++probe) {
    const unsigned long long k = T.keys[h];
    if (k == key) {
      found = T.flags[h] != 0u;
      break;
    }
    if (k == DD_EMPTY) break;
    h = (h + 1) & T.mask;
  }
  keep[i] = found ? 0 : 1;
}

size_t dedup_workspace_bytes(long long slots) {
  return (size_t)slots * 12 + 256;
}

hipError_t launch_dedup(long long slots, void* ws, double v, double kenv, const float* tm,
                        const float* tls, long long n_tgt, const float* depth, const float* vms,
                        const float* intr, int nk, int W, int H, const float* sm, long long n_src,
                        uint8_t* keep, hipStream_t s, unsigned int** counters) {
  DedupTable T;
  char* b = (char*)ws;
  T.counters = (unsigned int*)b;
  T.keys = (unsigned long long*)(b + 256);
  T.flags = (unsigned int*)(b + 256 + 8 * (size_t)slots);
  T.mask = (unsigned long long)slots - 1;
  *counters = T.counters;
  const auto blocks = [](long long n) { return dim3((unsigned)((n + 255) / 256)); };
  hipLaunchKernelGGL(k_dd_clear, blocks(slots), dim3(256), 0, s, T);
  if (n_tgt > 0)
    hipLaunchKernelGGL(k_dd_occ, blocks(n_tgt), dim3(256), 0, s, T, tm, tls, n_tgt, v, kenv);
  const long long npix = (long long)nk * W * H;
  if (npix > 0)
    hipLaunchKernelGGL(k_dd_free, blocks(npix), dim3(256), 0, s, T, depth, vms, intr, W, H, npix,
                       v);
  if (n_src > 0)
    hipLaunchKernelGGL(k_dd_probe, blocks(n_src), dim3(256), 0, s, T, sm, n_src, v, keep);
  return hipGetLastError();
}

}  // namespace gsr
