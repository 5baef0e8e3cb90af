// Tile binning: the last (most significant) digit of the (tile, depth) key
// sort, done as a stable counting sort on tile rows; the per-tile lists are
// the row lists filtered by column, which the compositing kernels do as they
// walk (a tile reads only the prefix of its row list that it needs).
//
// Input: each view's visible pairs in (depth, id) order and their tile
// rectangles.  The depth-ordered pairs are cut into chunks; per chunk the
// number of pairs spanning each tile row (1D difference array in LDS), an
// exclusive scan down each row's chunks, a scan over all (view, row) buckets
// (the row ranges), and a scatter where one wave per chunk holds its pairs in
// registers, 64 per step, and appends (visible position, x0 | x1 << 16) to
// every row the rect spans, ranked inside each row by a wave ballot (lane
// order = depth order), row by row so each row's stores are issued back to
// back.  The counting pass also sums the (pair, tile) copies the rects stand
// for (reported, never stored).
#include <algorithm>

#include "common.h"

namespace gsr {

__device__ __forceinline__ void chunk_range(const BinTab& t, const StateHeader* hdr, int b,
                                            int& v, int& lo, int& hi) {
  v = find_seg(t.cblk_off, t.nv, b);
  const int lc = b - t.cblk_off[v];
  lo = (int)hdr->vis_off[v] + lc * t.chunk;
  hi = min((int)hdr->vis_off[v + 1], lo + t.chunk);
}

__device__ __forceinline__ void unpack_rect(uint2 r, int& x0, int& y0, int& x1, int& y1) {
  x0 = r.x & 0xFFFF;
  y0 = r.x >> 16;
  x1 = r.y & 0xFFFF;
  y1 = r.y >> 16;
}

// Per chunk: pairs spanning each row (rows[y] for y < TY).  A workgroup
// takes RC_SUB chunks: their rects are loaded together, counted into one 1D
// difference array per chunk in LDS, and wave k scans chunk k's array.
__global__ __launch_bounds__(256) void k_row_count(BinTab t, StateDev st, uint32_t* counts,
                                                   uint32_t* area_part) {
  __shared__ int dif[RC_SUB][MAX_ROWS + 1];
  __shared__ uint32_t wsum[4];
  const int nc = t.cblk_off[t.nv];
  const int g = xcd_remap(blockIdx.x, (nc + RC_SUB - 1) / RC_SUB);
  if (g < 0) return;
  const int TY = t.TY;
  int lo[RC_SUB], hi[RC_SUB];
  uint2 rc[RC_SUB];
#pragma unroll
  for (int k = 0; k < RC_SUB; ++k) {
    const int b = g * RC_SUB + k;
    lo[k] = hi[k] = 0;
    if (b < nc) {
      int v;
      chunk_range(t, st.hdr, b, v, lo[k], hi[k]);
    }
    // a chunk holds at most 256 pairs: one per thread
    const int i = lo[k] + (int)threadIdx.x;
    rc[k] = i < hi[k] ? st.rect[st.order[i]] : make_uint2(0u, 0u);
  }
  for (int i = threadIdx.x; i < RC_SUB * (MAX_ROWS + 1); i += 256) (&dif[0][0])[i] = 0;
  __syncthreads();
  uint32_t area = 0;
#pragma unroll
  for (int k = 0; k < RC_SUB; ++k) {
    if (lo[k] + (int)threadIdx.x < hi[k]) {
      int x0, y0, x1, y1;
      unpack_rect(rc[k], x0, y0, x1, y1);
      atomicAdd(&dif[k][y0], 1);
      atomicSub(&dif[k][y1], 1);
      area += (uint32_t)((x1 - x0) * (y1 - y0));
    }
  }
  // (pair, tile) copies of the workgroup's pairs (at most 1024 x 512 x 512),
  // one partial per workgroup: the row range scan adds them up
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) area += (uint32_t)__shfl_xor((int)area, d, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = area;
  __syncthreads();
  if (threadIdx.x == 0) area_part[g] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  // wave k: inclusive scan of chunk k's difference array, 64 rows at a time
  const int k = threadIdx.x >> 6;
  const int b = g * RC_SUB + k;
  if (b < nc && lo[k] < hi[k]) {
    int carry = 0;
    for (int base = 0; base < TY; base += 64) {
      const int y = base + lane_id();
      const int x = y < TY ? dif[k][y] : 0;
      const int inc = (int)wave_incl_scan((uint32_t)x) + carry;
      if (y < TY) counts[(size_t)b * TY + y] = (uint32_t)inc;
      carry = __shfl(inc, 63, 64);
    }
  }
}

// Exclusive prefix of a [chunk][cols] count matrix down each column over the
// view's active chunks (in place), and the column totals.  A workgroup covers
// 16 consecutive columns (16 lanes: a 64-byte row piece) x 64 segments of the
// chunk range (four per wave), so the walk down a column is 64x shorter and
// there are few columns per workgroup (a view has one column per tile row).
constexpr int CS_COLS = 16, CS_SEGS = 64;
__global__ __launch_bounds__(CS_COLS* CS_SEGS) void k_colscan(BinTab t, const StateHeader* hdr,
                                                             int cols, uint32_t* counts,
                                                             uint32_t* totals) {
  __shared__ uint32_t part[CS_SEGS][CS_COLS];
  const int lane = threadIdx.x & (CS_COLS - 1), seg = threadIdx.x / CS_COLS;
  const int g = blockIdx.x * CS_COLS + lane;
  const bool ok = g < t.nv * cols;
  int k0 = 0, k1 = 0;
  uint32_t* c = counts;
  if (ok) {
    const int v = g / cols, col = g - v * cols;
    const int n = (int)(hdr->vis_off[v + 1] - hdr->vis_off[v]);
    const int nc = (n + t.chunk - 1) / t.chunk;
    k0 = (int)((long)nc * seg / CS_SEGS);
    k1 = (int)((long)nc * (seg + 1) / CS_SEGS);
    c = counts + (size_t)t.cblk_off[v] * cols + col;
  }
  uint32_t sum = 0;
  int k = k0;
  for (; k + 4 <= k1; k += 4) {
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = c[(size_t)(k + j) * cols];
#pragma unroll
    for (int j = 0; j < 4; ++j) sum += x[j];
  }
  for (; k < k1; ++k) sum += c[(size_t)k * cols];
  part[seg][lane] = sum;
  __syncthreads();
  uint32_t run = 0;
  for (int s2 = 0; s2 < seg; ++s2) run += part[s2][lane];
  if (ok && seg == CS_SEGS - 1) totals[g] = run + sum;
  k = k0;
  for (; k + 4 <= k1; k += 4) {
    uint32_t x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = c[(size_t)(k + j) * cols];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c[(size_t)(k + j) * cols] = run;
      run += x[j];
    }
  }
  for (; k < k1; ++k) {
    const uint32_t x = c[(size_t)k * cols];
    c[(size_t)k * cols] = run;
    run += x;
  }
}

// Exclusive scan of n bucket totals into [first, last+1) ranges ((0, 0)
// when empty), over ceil(n / RS_TILE) workgroups: workgroup b scans tile b
// after summing every total before it; the last workgroup writes the grand
// total into *total and the capacity flag into *flag (set when the total
// exceeds cap), and the sum of the np partials in part into *part_total.
constexpr int RS_TILE = 4096;  // 1024 threads x 4 totals
__global__ __launch_bounds__(1024) void k_range_scan(int n, const uint32_t* cnt, uint2* ranges,
                                                    unsigned long long cap,
                                                    unsigned long long* total,
                                                    unsigned int* flag, int np,
                                                    const uint32_t* part,
                                                    unsigned long long* part_total) {
  __shared__ unsigned long long sh[17];
  const int base = (int)blockIdx.x * RS_TILE;
  const unsigned long long carry = wg_sum_before<1024>(cnt, base, sh);
  const int i0 = base + 4 * (int)threadIdx.x;
  uint32_t x[4];
  unsigned long long s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = (i0 + k < n) ? cnt[i0 + k] : 0u;
    s += x[k];
  }
  unsigned long long tot;
  unsigned long long pre = wg_excl_scan<1024>(s, sh, &tot) + carry;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i0 + k < n) {
      const uint32_t a = (uint32_t)min(pre, 0xFFFFFFFFull);
      const uint32_t e = (uint32_t)min(pre + x[k], 0xFFFFFFFFull);
      ranges[i0 + k] = x[k] ? make_uint2(a, e) : make_uint2(0u, 0u);
    }
    pre += x[k];
  }
  if (blockIdx.x == gridDim.x - 1) {
    unsigned long long ps = 0;
    for (int i = threadIdx.x; i < np; i += 1024) ps += part[i];
    unsigned long long pall;
    (void)wg_excl_scan<1024>(ps, sh, &pall);
    if (threadIdx.x == 0) {
      const unsigned long long all = carry + tot;
      *total = all;
      *flag = all > cap ? 1u : 0u;
      *part_total = pall;
    }
  }
}

// Wave-wide minimum / maximum (every lane active), returned in every lane.
__device__ __forceinline__ int wave_min_i(int x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = min(x, __shfl_xor(x, d, 64));
  return x;
}
__device__ __forceinline__ int wave_max_i(int x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = max(x, __shfl_xor(x, d, 64));
  return x;
}

// One wave per chunk: append every pair, in order, to each row it spans.
// Row entries are (pair id, x0 | x1 << 16).  The chunk's pairs sit in
// registers, 64 per step (lane order = depth order); for every row the chunk
// spans, a ballot per step gives the lanes spanning it, so lane l's slot in
// that row is the row cursor plus the number of lower lanes in the mask.
// The row cursors sit in the wave's row of LDS (no barriers: one wave).
__global__ __launch_bounds__(256) void k_row_scatter(BinTab t, StateDev st, const uint32_t* counts) {
  constexpr int STEPS = MAX_CHUNK / 64;
  __shared__ uint32_t curs[4][MAX_ROWS];
  const int nc = t.cblk_off[t.nv];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int b = xcd_remap(blockIdx.x, (nc + 3) / 4) * 4 + wave;
  if (b < 0 || b >= nc) return;
  int v, lo, hi;
  chunk_range(t, st.hdr, b, v, lo, hi);
  if (lo >= hi || st.hdr->overflow) return;
  const int lane = threadIdx.x & 63, TY = t.TY;
  const int nsteps = (hi - lo + 63) / 64;
  // the chunk's pairs and rects, every load issued before the first use
  uint32_t pid[STEPS];
#pragma unroll
  for (int k = 0; k < STEPS; ++k) pid[k] = st.order[min(lo + k * 64 + lane, hi - 1)];
  uint2 rc[STEPS];
#pragma unroll
  for (int k = 0; k < STEPS; ++k) rc[k] = st.rect[pid[k]];
  int y0[STEPS], span[STEPS];
  uint32_t xs[STEPS];
  int ymin = TY, ymax = 0;
#pragma unroll
  for (int k = 0; k < STEPS; ++k) {
    const bool valid = lo + k * 64 + lane < hi;
    y0[k] = (int)(rc[k].x >> 16);
    const int y1 = (int)(rc[k].y >> 16);
    span[k] = valid ? y1 - y0[k] : 0;
    xs[k] = (rc[k].x & 0xFFFF) | (rc[k].y << 16);
    if (valid && y1 > y0[k]) {
      ymin = min(ymin, y0[k]);
      ymax = max(ymax, y1);
    }
  }
  ymin = __builtin_amdgcn_readfirstlane(wave_min_i(ymin));
  ymax = __builtin_amdgcn_readfirstlane(wave_max_i(ymax));
  uint32_t* cw = curs[wave];
  for (int y = ymin + lane; y < ymax; y += 64)
    cw[y] = st.row_rg[(size_t)v * TY + y].x + counts[(size_t)b * TY + y];
  __builtin_amdgcn_wave_barrier();
  // row by row: a ballot per 64 pairs; the row's stores of the chunk are
  // issued back to back onto consecutive entries.  They stay inside the row's
  // range: the counts used the same y0 <= y < y1 rule, and an overflowing
  // row level returned above.
#pragma unroll 1
  for (int y = ymin; y < ymax; ++y) {
    uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane((int)cw[y]);
#pragma unroll
    for (int k = 0; k < STEPS; ++k) {
      if (k < nsteps) {
        const bool cov = (unsigned)(y - y0[k]) < (unsigned)span[k];
        const unsigned long long m = __ballot(cov);
        if (cov) {
          const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
              (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          st.rows[c + rank] = make_uint2(pid[k], xs[k]);
        }
        c += (uint32_t)__popcll(m);
      }
    }
  }
}

hipError_t launch_binning(const BinTab& t, StateDev st, const BinWork& w, hipStream_t s) {
  const int nc = t.cblk_off[t.nv];
  const int nrows = t.nv * t.TY;
  const int nparts = (nc + RC_SUB - 1) / RC_SUB;
  if (nc > 0)
    hipLaunchKernelGGL(k_row_count, dim3(xcd_grid(nparts)), dim3(256), 0, s, t, st, w.counts,
                       w.area_part);
  hipLaunchKernelGGL(k_colscan, dim3((nrows + CS_COLS - 1) / CS_COLS), dim3(CS_COLS * CS_SEGS),
                     0, s, t, st.hdr, t.TY, w.counts, w.row_tot);
  const int nb = std::max(1, (nrows + RS_TILE - 1) / RS_TILE);
  hipLaunchKernelGGL(k_range_scan, dim3(nb), dim3(1024), 0, s, nrows, w.row_tot, st.row_rg,
                     st.cap, &st.hdr->row_total, &st.hdr->overflow, nparts, w.area_part,
                     &st.hdr->inst_total);
  if (nc > 0)
    hipLaunchKernelGGL(k_row_scatter, dim3(xcd_grid((nc + 3) / 4)), dim3(256), 0, s, t, st,
                       w.counts);
  return hipGetLastError();
}

}  // namespace gsr
