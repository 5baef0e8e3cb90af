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
//                per chunk walks its pairs in order and appends
//                (pair id, x0, x1) to every row the rect spans.  A chunk's
//                run in a row bucket is long (tens of entries), so these
//                writes are coalesced.
//   tile level : per (view, row), the row list (still in depth order) gives
//                the per-tile counts (difference array over columns); a scan
//                over all tiles gives the tile ranges; then four waves per
//                row, each owning a quarter of the row's tiles, walk the row
//                list 64 entries at a time, rank each entry inside every tile
//                it covers by a wave ballot (lanes are list order, so ranks
//                are stable) and write the pair id at the tile's cursor.
//                Each tile's list is written front to back by one wave, so
//                partial cache lines fill up in L2 before they are evicted.
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

// Per chunk: pairs spanning each row (rows[y] for y < TY).
__global__ __launch_bounds__(256) void k_row_count(BinTab t, StateDev st, uint32_t* counts) {
  __shared__ int dif[MAX_ROWS + 1];
  const int b = xcd_remap(blockIdx.x, t.cblk_off[t.nv]);
  if (b < 0) return;
  int v, lo, hi;
  chunk_range(t, st.hdr, b, v, lo, hi);
  if (lo >= hi) return;
  const int TY = t.TY;
  for (int i = threadIdx.x; i <= TY; i += 256) dif[i] = 0;
  __syncthreads();
  for (int i = lo + (int)threadIdx.x; i < hi; i += 256) {
    int x0, y0, x1, y1;
    unpack_rect(st.rect[st.order[i]], x0, y0, x1, y1);
    atomicAdd(&dif[y0], 1);
    atomicSub(&dif[y1], 1);
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    // wave-wide inclusive scan of the difference array, 64 rows at a time
    int carry = 0;
    for (int base = 0; base < TY; base += 64) {
      const int y = base + (int)threadIdx.x;
      const int x = y < TY ? dif[y] : 0;
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

// One workgroup: exclusive scan of n bucket totals into [first, last+1)
// ranges ((0, 0) when empty), the grand total into *total (if given) and the
// capacity flag into *flag (set when the total exceeds cap).
__global__ __launch_bounds__(1024) void k_range_scan(int n, const uint32_t* cnt, uint2* ranges,
                                                    unsigned long long cap,
                                                    unsigned long long* total,
                                                    unsigned int* flag,
                                                    const unsigned int* prior_flag,
                                                    const unsigned long long* prior_total) {
  __shared__ unsigned long long sh[17];
  unsigned long long carry = 0;
  for (int base = 0; base < n; base += 4096) {
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
    carry += tot;
  }
  if (threadIdx.x == 0) {
    // an earlier level that overflowed leaves this level's counts empty: keep
    // the flag and report the earlier level's total as a lower bound
    const bool prior = prior_flag && *prior_flag;
    if (prior && prior_total && *prior_total > carry) carry = *prior_total;
    if (total) *total = carry;
    *flag = (prior || carry > cap) ? 1u : 0u;
  }
}

// One wave per chunk: append every pair, in order, to each row it spans.
// Row entries are (pair id, x0 | x1 << 16).
__global__ __launch_bounds__(64) void k_row_scatter(BinTab t, StateDev st, const uint32_t* counts,
                                                    const uint2* row_rg, uint2* rows,
                                                    unsigned long long row_cap,
                                                    const unsigned int* row_flag) {
  __shared__ uint32_t cur[MAX_ROWS];
  const int b = xcd_remap(blockIdx.x, t.cblk_off[t.nv]);
  if (b < 0) return;
  int v, lo, hi;
  chunk_range(t, st.hdr, b, v, lo, hi);
  if (lo >= hi || *row_flag) return;
  const int lane = threadIdx.x, TY = t.TY;
  for (int y = lane; y < TY; y += 64)
    cur[y] = row_rg[(size_t)v * TY + y].x + counts[(size_t)b * TY + y];
  __builtin_amdgcn_wave_barrier();
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
      const int y0 = rx >> 16, y1 = ry >> 16;
      const uint32_t xs = (rx & 0xFFFF) | (ry << 16);
      // A pair appears at most once per row, so the lanes' rows are
      // distinct; LDS operations of one wave complete in issue order, so the
      // next pair sees these cursor updates.
      for (int y = y0 + lane; y < y1; y += 64) {
        const uint32_t pos = cur[y];
        if (pos < row_cap) rows[pos] = make_uint2(pj, xs);
        cur[y] = pos + 1;
      }
    }
  }
}

// Per (view, row): tile counts of the row from its list.
__global__ __launch_bounds__(256) void k_tile_count(BinTab t, const uint2* row_rg,
                                                    const uint2* rows, uint32_t* tile_cnt,
                                                    const unsigned int* row_flag) {
  __shared__ int dif[MAX_COLS + 1];
  const int r = xcd_remap(blockIdx.x, t.nv * t.TY);
  if (r < 0) return;
  const int TX = t.TX;
  for (int i = threadIdx.x; i <= TX; i += 256) dif[i] = 0;
  __syncthreads();
  const uint2 rg = *row_flag ? make_uint2(0u, 0u) : row_rg[r];
  for (uint32_t i = rg.x + threadIdx.x; i < rg.y; i += 256) {
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
      if (x < TX) tile_cnt[(size_t)r * TX + x] = (uint32_t)inc;
      carry = __shfl(inc, 63, 64);
    }
  }
}

// Per (view, row), 4 waves; wave q owns the row's tiles [c0, c1).  Each
// batch of 64 row entries (lane order = list order) is ranked per tile with
// a ballot, and each lane writes its pair at cursor + rank for every tile
// of its span that the wave owns.
constexpr int TS_WAVES = 4;
__global__ __launch_bounds__(64 * TS_WAVES) void k_tile_scatter(BinTab t, StateDev st,
                                                               const uint2* row_rg,
                                                               const uint2* rows) {
  __shared__ uint32_t cur[TS_WAVES][MAX_COLS];
  __shared__ unsigned long long msk[TS_WAVES][MAX_COLS];
  const int r = xcd_remap(blockIdx.x, t.nv * t.TY);
  if (r < 0) return;
  if (st.hdr->overflow) return;
  const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int TX = t.TX;
  const int per = (TX + TS_WAVES - 1) / TS_WAVES;
  const int c0 = min(TX, q * per), c1 = min(TX, c0 + per);
  if (c0 >= c1) return;
  const uint2* trg = st.ranges + (size_t)r * TX;
  uint32_t* cw = cur[q];
  unsigned long long* mw = msk[q];
  for (int x = c0 + lane; x < c1; x += 64) cw[x] = trg[x].x;
  const uint2 rg = row_rg[r];
  const unsigned long long lt = (1ull << lane) - 1ull;
  __builtin_amdgcn_wave_barrier();
  for (uint32_t base = rg.x; base < rg.y; base += 64) {
    const uint32_t i = base + lane;
    const bool valid = i < rg.y;
    const uint2 e = valid ? rows[i] : make_uint2(0u, 0u);
    const int x0 = max((int)(e.y & 0xFFFF), c0), x1 = min((int)(e.y >> 16), c1);
    const bool mine = valid && x0 < x1;
    if (__ballot(mine) == 0ull) continue;
    // columns this batch touches inside [c0, c1)
    int lo = mine ? x0 : c1, hi = mine ? x1 : c0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      lo = min(lo, __shfl_xor(lo, d, 64));
      hi = max(hi, __shfl_xor(hi, d, 64));
    }
    for (int x = lo; x < hi; ++x) {
      const unsigned long long m = __ballot(mine && x0 <= x && x < x1);
      if (lane == 0) mw[x] = m;
    }
    __builtin_amdgcn_wave_barrier();
    if (mine)
      for (int x = x0; x < x1; ++x) {
        const uint32_t pos = cw[x] + (uint32_t)__popcll(mw[x] & lt);
        if (pos < st.cap) st.inst[pos] = e.x;
      }
    __builtin_amdgcn_wave_barrier();
    for (int x = lo + lane; x < hi; x += 64) cw[x] += (uint32_t)__popcll(mw[x]);
    __builtin_amdgcn_wave_barrier();
  }
}

hipError_t launch_binning(const BinTab& t, StateDev st, const BinWork& w, hipStream_t s) {
  const int nc = t.cblk_off[t.nv];
  const int nrows = t.nv * t.TY;
  if (nc > 0)
    hipLaunchKernelGGL(k_row_count, dim3(xcd_grid(nc)), dim3(256), 0, s, t, st, w.counts);
  hipLaunchKernelGGL(k_colscan, dim3((nrows + CS_COLS - 1) / CS_COLS), dim3(CS_COLS * CS_SEGS),
                     0, s, t, st.hdr, t.TY, w.counts, w.row_tot);
  hipLaunchKernelGGL(k_range_scan, dim3(1), dim3(1024), 0, s, nrows, w.row_tot, w.row_rg,
                     w.row_cap, &st.hdr->row_total, w.row_flag, (const unsigned int*)nullptr,
                     (const unsigned long long*)nullptr);
  if (nc > 0)
    hipLaunchKernelGGL(k_row_scatter, dim3(xcd_grid(nc)), dim3(64), 0, s, t, st, w.counts,
                       w.row_rg, w.rows, w.row_cap, w.row_flag);
  hipLaunchKernelGGL(k_tile_count, dim3(xcd_grid(nrows)), dim3(256), 0, s, t, w.row_rg, w.rows,
                     w.tile_cnt, w.row_flag);
  hipLaunchKernelGGL(k_range_scan, dim3(1), dim3(1024), 0, s, t.nv * t.T, w.tile_cnt, st.ranges,
                     st.cap, &st.hdr->inst_total, &st.hdr->overflow, w.row_flag,
                     &st.hdr->row_total);
  hipLaunchKernelGGL(k_tile_scatter, dim3(xcd_grid(nrows)), dim3(64 * TS_WAVES), 0, s, t, st,
                     w.row_rg, w.rows);
  return hipGetLastError();
}

}  // namespace gsr
