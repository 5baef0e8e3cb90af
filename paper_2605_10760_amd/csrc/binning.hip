// Tile binning: the last (most significant) digit of the (tile, depth) key
// sort, done as a stable two-level counting sort - rows, then tiles - that
// writes each tile's list in (depth, pair id) order without ever forming the
// 64-bit keys.
//
// Input: each view's visible pairs in (depth, id) order and their tile
// rectangles.
//   row level  : the depth-ordered pairs are cut into chunks; per chunk the
//                number of pairs spanning each tile row (1D difference array
//                in LDS), an exclusive scan down each row's chunks, a scan
//                over all (view, row) buckets, and a scatter where one wave
//                per chunk takes its pairs 64 at a time and appends
//                (pair id, x0, x1) to every row the rect spans, ranked inside
//                each row by a wave ballot (lane order = depth order).
//   Both scatters hold their chunk / segment in registers and walk it
//   bucket by bucket, so each bucket's stores are issued back to back.
//   tile level : each row list (still in depth order) is cut into segments
//                of SEG entries; per segment the number of entries covering
//                each tile of the row, an exclusive scan down each tile's
//                segments, a scan over all tiles (the tile ranges), and a
//                scatter where one wave per segment holds the segment in
//                registers and, column by column, ranks the entries covering
//                the column by a wave ballot per 64 entries.
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
constexpr int RC_SUB = 4;
__global__ __launch_bounds__(256) void k_row_count(BinTab t, StateDev st, uint32_t* counts) {
  __shared__ int dif[RC_SUB][MAX_ROWS + 1];
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
#pragma unroll
  for (int k = 0; k < RC_SUB; ++k) {
    if (lo[k] + (int)threadIdx.x < hi[k]) {
      int x0, y0, x1, y1;
      unpack_rect(rc[k], x0, y0, x1, y1);
      atomicAdd(&dif[k][y0], 1);
      atomicSub(&dif[k][y1], 1);
    }
  }
  __syncthreads();
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
// 64 consecutive columns (lanes: coalesced rows) x 16 segments of the chunk
// range (waves), so the dependent walk down a column is 16x shorter.
constexpr int CS_COLS = 64, CS_SEGS = 16;
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
// total into *total (if given) and the capacity flag into *flag (set when
// the total exceeds cap).
constexpr int RS_TILE = 4096;  // 1024 threads x 4 totals
__global__ __launch_bounds__(1024) void k_range_scan(int n, const uint32_t* cnt, uint2* ranges,
                                                    unsigned long long cap,
                                                    unsigned long long* total,
                                                    unsigned int* flag,
                                                    const unsigned int* prior_flag,
                                                    const unsigned long long* prior_total) {
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
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    unsigned long long all = carry + tot;
    // an earlier level that overflowed leaves this level's counts empty: keep
    // the flag and report the earlier level's total as a lower bound
    const bool prior = prior_flag && *prior_flag;
    if (prior && prior_total && *prior_total > all) all = *prior_total;
    if (total) *total = all;
    *flag = (prior || all > cap) ? 1u : 0u;
  }
}

static void range_scan(int n, const uint32_t* cnt, uint2* ranges, unsigned long long cap,
                       unsigned long long* total, unsigned int* flag,
                       const unsigned int* prior_flag, const unsigned long long* prior_total,
                       hipStream_t s) {
  const int nb = std::max(1, (n + RS_TILE - 1) / RS_TILE);
  hipLaunchKernelGGL(k_range_scan, dim3(nb), dim3(1024), 0, s, n, cnt, ranges, cap, total, flag,
                     prior_flag, prior_total);
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
__global__ __launch_bounds__(256) void k_row_scatter(BinTab t, StateDev st, const uint32_t* counts,
                                                     const uint2* row_rg, uint2* rows,
                                                     const unsigned int* row_flag) {
  constexpr int STEPS = MAX_CHUNK / 64;
  __shared__ uint32_t curs[4][MAX_ROWS];
  const int nc = t.cblk_off[t.nv];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int b = xcd_remap(blockIdx.x, (nc + 3) / 4) * 4 + wave;
  if (b < 0 || b >= nc) return;
  int v, lo, hi;
  chunk_range(t, st.hdr, b, v, lo, hi);
  if (lo >= hi || *row_flag) return;
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
    cw[y] = row_rg[(size_t)v * TY + y].x + counts[(size_t)b * TY + y];
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
          rows[c + rank] = make_uint2(pid[k], xs[k]);
        }
        c += (uint32_t)__popcll(m);
      }
    }
  }
}

// Level 2 works on segments of SEG consecutive entries of a row list, so a
// long row is spread over many workgroups; segment s of row r covers
// entries [row_rg[r].x + (s - seg_off[r]) * SEG, ...) of that row.

// One workgroup: segment offsets of the row lists (zero segments when the
// row level overflowed).
__global__ __launch_bounds__(1024) void k_seg_scan(int n, const uint2* row_rg, uint32_t* seg_off,
                                                  const unsigned int* row_flag) {
  __shared__ unsigned long long sh[17];
  const bool off = *row_flag != 0u;
  unsigned long long carry = 0;
  for (int base = 0; base < n; base += 1024) {
    const int r = base + (int)threadIdx.x;
    uint32_t ns = 0;
    if (r < n && !off) {
      const uint2 rg = row_rg[r];
      ns = (rg.y - rg.x + SEG - 1) / SEG;
    }
    unsigned long long tot;
    const unsigned long long pre = wg_excl_scan<1024>(ns, sh, &tot) + carry;
    if (r < n) seg_off[r] = (uint32_t)pre;
    carry += tot;
  }
  if (threadIdx.x == 0) seg_off[n] = (uint32_t)carry;
}

// One workgroup per row list: the row of each of its segments.
__global__ __launch_bounds__(256) void k_seg_rows(const uint32_t* seg_off, uint32_t* seg_row) {
  const int r = blockIdx.x;
  const uint32_t s0 = seg_off[r], s1 = seg_off[r + 1];
  for (uint32_t k = s0 + threadIdx.x; k < s1; k += 256) seg_row[k] = (uint32_t)r;
}

// Row r and entry range [lo, hi) of segment s.
__device__ __forceinline__ void seg_range(const uint32_t* seg_off, const uint32_t* seg_row,
                                          const uint2* row_rg, uint32_t s, int& r, uint32_t& lo,
                                          uint32_t& hi) {
  r = (int)seg_row[s];
  const uint2 rg = row_rg[r];
  lo = rg.x + (s - seg_off[r]) * (uint32_t)SEG;
  hi = min(rg.y, lo + (uint32_t)SEG);
}

// Per segment: entries covering each tile of the row (1D difference array
// over the columns).  Grid-stride over the device-side segment count.
__global__ __launch_bounds__(256) void k_tile_count(int nrows, int TX, const uint32_t* seg_off,
                                                    const uint32_t* seg_row, const uint2* row_rg,
                                                    const uint2* rows, uint32_t* seg_cnt) {
  __shared__ int dif[MAX_COLS + 1];
  const uint32_t nseg = seg_off[nrows];
  for (uint32_t s = (uint32_t)xcd_remap(blockIdx.x, gridDim.x); s < nseg; s += gridDim.x) {
    int r;
    uint32_t lo, hi;
    seg_range(seg_off, seg_row, row_rg, s, r, lo, hi);
    for (int i = threadIdx.x; i <= TX; i += 256) dif[i] = 0;
    __syncthreads();
    for (uint32_t i = lo + threadIdx.x; i < hi; i += 256) {
      const uint32_t xs = rows[i].y;
      atomicAdd(&dif[xs & 0xFFFF], 1);
      atomicSub(&dif[xs >> 16], 1);
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      int carry = 0;
      for (int base = 0; base < TX; base += 64) {
        const int x = base + (int)threadIdx.x;
        const int d = x < TX ? dif[x] : 0;
        const int inc = (int)wave_incl_scan((uint32_t)d) + carry;
        if (x < TX) seg_cnt[(size_t)s * TX + x] = (uint32_t)inc;
        carry = __shfl(inc, 63, 64);
      }
    }
    __syncthreads();
  }
}

// One thread per (row, column): exclusive scan of the column's counts down
// the row's segments (in place) and the tile's total.
__global__ __launch_bounds__(256) void k_seg_colscan(int nrows, int TX, const uint32_t* seg_off,
                                                     uint32_t* seg_cnt, uint32_t* tile_cnt) {
  const int g = blockIdx.x * 256 + (int)threadIdx.x;
  if (g >= nrows * TX) return;
  const int r = g / TX, x = g - r * TX;
  const uint32_t s0 = seg_off[r], s1 = seg_off[r + 1];
  uint32_t* c = seg_cnt + (size_t)s0 * TX + x;
  const int n = (int)(s1 - s0);
  uint32_t run = 0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {
    uint32_t v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = c[(size_t)(k + j) * TX];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c[(size_t)(k + j) * TX] = run;
      run += v[j];
    }
  }
  for (; k < n; ++k) {
    const uint32_t v = c[(size_t)k * TX];
    c[(size_t)k * TX] = run;
    run += v;
  }
  tile_cnt[g] = run;
}

// One wave per segment (grid-stride over the device-side segment count).
// The segment's SEG entries are loaded into registers at once, 64 per step in
// list order; the cursors of the columns it covers go to the wave's row of
// LDS.  Column by column, a ballot per step gives the lanes whose entry
// covers the column; lane l stores its pair at the column's cursor plus the
// number of lower lanes in the mask, and the cursor advances by the mask's
// count.  A column's stores of the whole segment are issued back to back and
// land on consecutive words, so its cache lines are filled before the next
// column starts (walking step-major instead interleaves every column's short
// runs, and partly filled lines reach HBM about twice over).  The step loop
// is unrolled so that the entries are addressed statically.
constexpr int TS_WAVES = 4;
constexpr int TS_STEPS = SEG / 64;
// Lanes whose entry covers column x store their pair at c plus their rank
// among the covering lanes; c advances by the number of covering lanes.
__device__ __forceinline__ void scatter_step(int x, int x0, int span, uint32_t pid, uint32_t& c,
                                             uint32_t* inst) {
  const bool cov = (unsigned)(x - x0) < (unsigned)span;
  const unsigned long long m = __ballot(cov);
  if (cov) {
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    inst[c + rank] = pid;
  }
  c += (uint32_t)__popcll(m);
}

__global__ __launch_bounds__(64 * TS_WAVES) void k_tile_scatter(BinTab t, StateDev st,
                                                                const uint32_t* seg_off,
                                                                const uint32_t* seg_row,
                                                                const uint32_t* seg_cnt,
                                                                const uint2* row_rg,
                                                                const uint2* rows) {
  __shared__ uint32_t curs[TS_WAVES][MAX_COLS];
  if (st.hdr->overflow) return;
  const int nrows = t.nv * t.TY;
  const uint32_t nseg = seg_off[nrows];
  const int lane = threadIdx.x & 63, TX = t.TX;
  const uint32_t nw = gridDim.x * TS_WAVES;
  const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  uint32_t* cw = curs[wave];
  for (uint32_t s = (uint32_t)xcd_remap(blockIdx.x, gridDim.x) * TS_WAVES + wave; s < nseg;
       s += nw) {
    int r;
    uint32_t lo, hi;
    seg_range(seg_off, seg_row, row_rg, s, r, lo, hi);
    const int nsteps = (int)((hi - lo + 63) / 64);
    uint32_t pid[TS_STEPS];
    int x0[TS_STEPS], span[TS_STEPS];
    int xmin = TX, xmax = 0;
    // unconditional loads (clamped into the segment) so that all of them are
    // in flight together
#pragma unroll
    for (int k = 0; k < TS_STEPS; ++k) {
      const uint32_t i = lo + (uint32_t)(k * 64 + lane);
      const uint2 e = rows[min(i, hi - 1u)];
      const bool valid = i < hi;
      pid[k] = e.x;
      x0[k] = (int)(e.y & 0xFFFF);
      span[k] = valid ? (int)(e.y >> 16) - x0[k] : 0;
      if (valid) {
        xmin = min(xmin, x0[k]);
        xmax = max(xmax, (int)(e.y >> 16));
      }
    }
    xmin = __builtin_amdgcn_readfirstlane(wave_min_i(xmin));
    xmax = __builtin_amdgcn_readfirstlane(wave_max_i(xmax));
    // the cursors of the covered columns go to this wave's LDS row
    for (int x = xmin + lane; x < xmax; x += 64)
      cw[x] = st.ranges[(size_t)r * TX + x].x + seg_cnt[(size_t)s * TX + x];
    __builtin_amdgcn_wave_barrier();
    // Stores stay inside the tile's range: the column's cursor plus the
    // covering entries of this segment end at the next segment's cursor
    // (the counts used the same x0 <= x < x1 rule), and the ranges fit the
    // capacity (checked above through the overflow flag).
    if (nsteps == TS_STEPS) {
#pragma unroll 1
      for (int x = xmin; x < xmax; ++x) {
        uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane((int)cw[x]);
#pragma unroll
        for (int k = 0; k < TS_STEPS; ++k) scatter_step(x, x0[k], span[k], pid[k], c, st.inst);
      }
    } else {
#pragma unroll 1
      for (int x = xmin; x < xmax; ++x) {
        uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane((int)cw[x]);
#pragma unroll
        for (int k = 0; k < TS_STEPS; ++k)
          if (k < nsteps) scatter_step(x, x0[k], span[k], pid[k], c, st.inst);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

hipError_t launch_binning(const BinTab& t, StateDev st, const BinWork& w, hipStream_t s) {
  const int nc = t.cblk_off[t.nv];
  const int nrows = t.nv * t.TY;
  // level 1: rows
  if (nc > 0)
    hipLaunchKernelGGL(k_row_count, dim3(xcd_grid((nc + RC_SUB - 1) / RC_SUB)), dim3(256), 0, s,
                       t, st, w.counts);
  hipLaunchKernelGGL(k_colscan, dim3((nrows + CS_COLS - 1) / CS_COLS), dim3(CS_COLS * CS_SEGS),
                     0, s, t, st.hdr, t.TY, w.counts, w.row_tot);
  range_scan(nrows, w.row_tot, w.row_rg, w.row_cap, &st.hdr->row_total, w.row_flag,
             (const unsigned int*)nullptr, (const unsigned long long*)nullptr, s);
  if (nc > 0)
    hipLaunchKernelGGL(k_row_scatter, dim3(xcd_grid((nc + 3) / 4)), dim3(256), 0, s, t, st,
                       w.counts, w.row_rg, w.rows, w.row_flag);
  // level 2: tiles, per row segment
  hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, s, nrows, w.row_rg, w.seg_off,
                     w.row_flag);
  if (nrows > 0)
    hipLaunchKernelGGL(k_seg_rows, dim3(nrows), dim3(256), 0, s, w.seg_off, w.seg_row);
  hipLaunchKernelGGL(k_tile_count, dim3(w.seg_grid), dim3(256), 0, s, nrows, t.TX, w.seg_off,
                     w.seg_row, w.row_rg, w.rows, w.seg_cnt);
  hipLaunchKernelGGL(k_seg_colscan, dim3((nrows * t.TX + 255) / 256), dim3(256), 0, s, nrows,
                     t.TX, w.seg_off, w.seg_cnt, w.tile_cnt);
  range_scan(t.nv * t.T, w.tile_cnt, st.ranges, st.cap, &st.hdr->inst_total, &st.hdr->overflow,
             w.row_flag, &st.hdr->row_total, s);
  hipLaunchKernelGGL(k_tile_scatter, dim3(w.seg_grid), dim3(64 * TS_WAVES), 0, s, t, st,
                     w.seg_off, w.seg_row, w.seg_cnt, w.row_rg, w.rows);
  return hipGetLastError();
}

}  // namespace gsr
