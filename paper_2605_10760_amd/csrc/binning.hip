// Tile binning: the last (most significant) digit of the (tile, depth) key
// sort, done as a stable counting sort whose bucket is the tile.
//
// Input: each view's visible pairs in (depth, id) order and their tile
// rectangles.  The pairs are cut into chunks of C consecutive entries.
//   count   : per chunk, per-tile instance counts from a 2D difference array
//             in LDS (4 atomics per pair) and a 2D prefix sum
//   colscan : per tile, exclusive prefix over the view's chunks
//   tilescan: exclusive prefix over all tiles -> tile ranges, total count,
//             capacity check
//   scatter : one wave per chunk walks its pairs in order and writes the
//             pair id to every tile of the rect at that tile's LDS cursor
// Because chunks are in depth order and a chunk's pairs are visited in
// order, each tile's list comes out in (depth, id) order - the stable pass
// of an LSD radix sort - and the 64-bit keys are never materialised.
#include "common.h"

namespace gsr {

__device__ __forceinline__ void chunk_range(const BinTab& t, const StateHeader* hdr, int b,
                                            int& v, int& lo, int& hi) {
  v = find_seg(t.cblk_off, t.nv, b);
  const int lc = b - t.cblk_off[v];
  lo = (int)hdr->vis_off[v] + lc * t.chunk;
  hi = min((int)hdr->vis_off[v + 1], lo + t.chunk);
}

__global__ __launch_bounds__(256) void k_bin_count(BinTab t, StateDev st, uint32_t* counts) {
  extern __shared__ int dif[];  // (TY+1) x (TX+1)
  const int b = xcd_remap(blockIdx.x, t.cblk_off[t.nv]);
  if (b < 0) return;
  int v, lo, hi;
  chunk_range(t, st.hdr, b, v, lo, hi);
  if (lo >= hi) return;
  const int TX = t.TX, TY = t.TY, SX = TX + 1;
  const int nd = (TY + 1) * SX;
  for (int i = threadIdx.x; i < nd; i += 256) dif[i] = 0;
  __syncthreads();
  for (int i = lo + (int)threadIdx.x; i < hi; i += 256) {
    const uint32_t pair = st.order[i];
    const uint2 r = st.rect[pair];
    const int x0 = r.x & 0xFFFF, y0 = r.x >> 16, x1 = r.y & 0xFFFF, y1 = r.y >> 16;
    atomicAdd(&dif[y0 * SX + x0], 1);
    atomicSub(&dif[y0 * SX + x1], 1);
    atomicSub(&dif[y1 * SX + x0], 1);
    atomicAdd(&dif[y1 * SX + x1], 1);
  }
  __syncthreads();
  for (int y = threadIdx.x; y < TY; y += 256) {
    int run = 0;
    for (int x = 0; x < TX; ++x) {
      run += dif[y * SX + x];
      dif[y * SX + x] = run;
    }
  }
  __syncthreads();
  uint32_t* out = counts + (size_t)b * t.T;
  for (int x = threadIdx.x; x < TX; x += 256) {
    int run = 0;
    for (int y = 0; y < TY; ++y) {
      run += dif[y * SX + x];
      out[y * TX + x] = (uint32_t)run;
    }
  }
}

// Exclusive prefix of each tile's counts over its view's active chunks (in
// place) and the tile's total.  A workgroup covers 64 consecutive tiles
// (lanes: coalesced rows) x 16 segments of the chunk range (waves), so the
// dependent walk down a column is 16x shorter.
constexpr int CS_TILES = 64, CS_SEGS = 16;
__global__ __launch_bounds__(CS_TILES* CS_SEGS) void k_bin_colscan(BinTab t,
                                                                  const StateHeader* hdr,
                                                                  uint32_t* counts,
                                                                  uint32_t* tile_cnt) {
  __shared__ uint32_t part[CS_SEGS][CS_TILES];
  const int lane = threadIdx.x & (CS_TILES - 1), seg = threadIdx.x / CS_TILES;
  const int g = blockIdx.x * CS_TILES + lane;
  const bool ok = g < t.nv * t.T;
  int nc = 0, k0 = 0, k1 = 0;
  uint32_t* c = counts;
  if (ok) {
    const int v = g / t.T, tl = g - v * t.T;
    const int n = (int)(hdr->vis_off[v + 1] - hdr->vis_off[v]);
    nc = (n + t.chunk - 1) / t.chunk;
    k0 = (int)((long)nc * seg / CS_SEGS);
    k1 = (int)((long)nc * (seg + 1) / CS_SEGS);
    c = counts + (size_t)t.cblk_off[v] * t.T + tl;
  }
  uint32_t sum = 0;
  int k = k0;
  for (; k + 4 <= k1; k += 4) {
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = c[(size_t)(k + j) * t.T];
#pragma unroll
    for (int j = 0; j < 4; ++j) sum += x[j];
  }
  for (; k < k1; ++k) sum += c[(size_t)k * t.T];
  part[seg][lane] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (int s2 = 0; s2 < seg; ++s2) run += part[s2][lane];
  if (ok && seg == CS_SEGS - 1) tile_cnt[g] = run + sum;
  k = k0;
  for (; k + 4 <= k1; k += 4) {
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = c[(size_t)(k + j) * t.T];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c[(size_t)(k + j) * t.T] = run;
      run += x[j];
    }
  }
  for (; k < k1; ++k) {
    const uint32_t x = c[(size_t)k * t.T];
    c[(size_t)k * t.T] = run;
    run += x;
  }
}

// One workgroup: tile ranges from the per-tile totals; total instance count
// and the capacity flag go to the state header.
__global__ __launch_bounds__(1024) void k_tile_scan(BinTab t, StateDev st,
                                                   const uint32_t* tile_cnt) {
  __shared__ unsigned long long sh[17];
  const int n = t.nv * t.T;
  unsigned long long carry = 0;
  for (int base = 0; base < n; base += 4096) {
    const int i0 = base + 4 * (int)threadIdx.x;
    uint32_t x[4];
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[k] = (i0 + k < n) ? tile_cnt[i0 + k] : 0u;
      s += x[k];
    }
    unsigned long long tot;
    unsigned long long pre = wg_excl_scan<1024>(s, sh, &tot) + carry;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (i0 + k < n) {
        const uint32_t a = (uint32_t)min(pre, 0xFFFFFFFFull);
        const uint32_t e = (uint32_t)min(pre + x[k], 0xFFFFFFFFull);
        st.ranges[i0 + k] = x[k] ? make_uint2(a, e) : make_uint2(0u, 0u);
      }
      pre += x[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    st.hdr->inst_total = carry;
    st.hdr->overflow = carry > st.cap ? 1u : 0u;
  }
}

// One wave per chunk.  cursor[t] starts at the tile's range start plus the
// instances of earlier chunks; the chunk's pairs are visited in order and
// the lanes cover the current pair's rectangle (one entry per tile).
__global__ __launch_bounds__(64) void k_bin_scatter(BinTab t, StateDev st,
                                                    const uint32_t* counts) {
  extern __shared__ uint32_t cur[];  // [T]
  const int b = xcd_remap(blockIdx.x, t.cblk_off[t.nv]);
  if (b < 0) return;
  int v, lo, hi;
  chunk_range(t, st.hdr, b, v, lo, hi);
  if (lo >= hi) return;
  if (st.hdr->overflow) return;
  const int lane = threadIdx.x, TX = t.TX, T = t.T;
  const uint32_t* cb = counts + (size_t)b * T;
  const uint2* rg = st.ranges + (size_t)v * T;
  for (int i = lane; i < T; i += 64) cur[i] = rg[i].x + cb[i];
  __syncthreads();
  for (int base = lo; base < hi; base += 64) {
    const int i = base + lane;
    const bool valid = i < hi;
    const uint32_t pair = valid ? st.order[i] : 0u;
    const uint2 r = valid ? st.rect[pair] : make_uint2(0u, 0u);
    const int cnt = min(64, hi - base);
    for (int j = 0; j < cnt; ++j) {
      const uint32_t pj = __builtin_amdgcn_readlane(pair, j);
      const uint32_t rx = __builtin_amdgcn_readlane(r.x, j);
      const uint32_t ry = __builtin_amdgcn_readlane(r.y, j);
      const int x0 = rx & 0xFFFF, y0 = rx >> 16, x1 = ry & 0xFFFF, y1 = ry >> 16;
      const int w = x1 - x0, area = w * (y1 - y0);
      for (int k = lane; k < area; k += 64) {
        const int dy = k / w;
        const int tile = (y0 + dy) * TX + x0 + (k - dy * w);
        const uint32_t pos = cur[tile];
        if (pos < st.cap) st.inst[pos] = pj;
        cur[tile] = pos + 1;
      }
      // The next pair may read cursors this pair's lanes wrote.  LDS
      // operations of one wave execute in issue order, and the compiler keeps
      // these possibly-aliasing accesses in program order.
    }
  }
}

hipError_t launch_binning(const BinTab& t, StateDev st, uint32_t* counts, uint32_t* tile_cnt,
                          hipStream_t s) {
  const int nc = t.cblk_off[t.nv];
  const size_t dif_bytes = (size_t)(t.TX + 1) * (t.TY + 1) * sizeof(int);
  if (nc > 0)
    hipLaunchKernelGGL(k_bin_count, dim3(xcd_grid(nc)), dim3(256), dif_bytes, s, t, st, counts);
  const int ntile = t.nv * t.T;
  hipLaunchKernelGGL(k_bin_colscan, dim3((ntile + CS_TILES - 1) / CS_TILES),
                     dim3(CS_TILES * CS_SEGS), 0, s, t, st.hdr, counts, tile_cnt);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, t, st, tile_cnt);
  if (nc > 0)
    hipLaunchKernelGGL(k_bin_scatter, dim3(xcd_grid(nc)), dim3(64), (size_t)t.T * sizeof(uint32_t), s, t,
                       st, counts);
  return hipGetLastError();
}

}  // namespace gsr
