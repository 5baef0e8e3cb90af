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
//   tile level : each row list (still in depth order) is cut into segments
//                of SEG entries; per segment the number of entries covering
//                each tile of the row, an exclusive scan down each tile's
//                segments, a scan over all tiles (the tile ranges), and a
//                scatter that groups a segment's instances by tile in LDS
//                and copies them out so that each tile's share is stored as
//                one contiguous run.
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
// Row entries are (pair id, x0 | x1 << 16).  Each step takes 64 consecutive
// pairs (lane order = depth order); for every row the step touches, a ballot
// gives the mask of lanes spanning it, so lane l's slot in that row is the
// row cursor plus the number of lower lanes in the mask.
__global__ __launch_bounds__(64) void k_row_scatter(BinTab t, StateDev st, const uint32_t* counts,
                                                    const uint2* row_rg, uint2* rows,
                                                    unsigned long long row_cap,
                                                    const unsigned int* row_flag) {
  __shared__ uint32_t cur[MAX_ROWS];
  __shared__ unsigned long long msk[MAX_ROWS];
  const int b = xcd_remap(blockIdx.x, t.cblk_off[t.nv]);
  if (b < 0) return;
  int v, lo, hi;
  chunk_range(t, st.hdr, b, v, lo, hi);
  if (lo >= hi || *row_flag) return;
  const int lane = threadIdx.x, TY = t.TY;
  for (int y = lane; y < TY; y += 64)
    cur[y] = row_rg[(size_t)v * TY + y].x + counts[(size_t)b * TY + y];
  const unsigned long long lt = (1ull << lane) - 1ull;
  __builtin_amdgcn_wave_barrier();
  for (int base = lo; base < hi; base += 64) {
    const int i = base + lane;
    const bool valid = i < hi;
    const uint32_t pair = valid ? st.order[i] : 0u;
    const uint2 r = valid ? st.rect[pair] : make_uint2(0u, 0u);
    const int y0 = valid ? (int)(r.x >> 16) : TY, y1 = valid ? (int)(r.y >> 16) : 0;
    const uint32_t xs = (r.x & 0xFFFF) | (r.y << 16);
    int ylo = y0, yhi = y1;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      ylo = min(ylo, __shfl_xor(ylo, d, 64));
      yhi = max(yhi, __shfl_xor(yhi, d, 64));
    }
    for (int y = ylo; y < yhi; ++y) {
      const unsigned long long m = __ballot(y0 <= y && y < y1);
      if (lane == 0) msk[y] = m;
    }
    // LDS operations of one wave complete in issue order
    __builtin_amdgcn_wave_barrier();
    for (int y = y0; y < y1; ++y) {
      const uint32_t pos = cur[y] + (uint32_t)__popcll(msk[y] & lt);
      if (pos < row_cap) rows[pos] = make_uint2(pair, xs);
    }
    __builtin_amdgcn_wave_barrier();
    for (int y = ylo + lane; y < yhi; y += 64) cur[y] += (uint32_t)__popcll(msk[y]);
    __builtin_amdgcn_wave_barrier();
  }
}

// Level 2 works on segments of SEG consecutive entries of a row list, so a
// long row is spread over many workgroups; segment s of row r covers
// entries [row_rg[r].x + (s - seg_off[r]) * SEG, ...) of that row.

// One workgroup: segment offsets of the row lists and the row of every
// segment (zero segments when the row level overflowed).
__global__ __launch_bounds__(1024) void k_seg_scan(int n, const uint2* row_rg, uint32_t* seg_off,
                                                  uint32_t* seg_row,
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
    if (r < n) {
      seg_off[r] = (uint32_t)pre;
      for (uint32_t k = 0; k < ns; ++k) seg_row[pre + k] = (uint32_t)r;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) seg_off[n] = (uint32_t)carry;
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

// Per segment (grid-stride): the segment is cut into batches of up to 256
// entries (one per thread) whose tile instances fit an LDS buffer.  A
// batch's instances are first placed in the buffer grouped by tile (each
// tile's part in list order, ranked with per-wave ballots), then copied out
// slot by slot, so consecutive lanes store to consecutive addresses of one
// tile's list: a tile's share of a batch is one contiguous run.
constexpr int TS_THREADS = 256, TS_WAVES = TS_THREADS / 64, TS_BUF = 4096;
static_assert(TS_BUF >= MAX_COLS, "one row entry must always fit a batch");
__global__ __launch_bounds__(TS_THREADS) void k_tile_scatter(BinTab t, StateDev st,
                                                             const uint32_t* seg_off,
                                                             const uint32_t* seg_row,
                                                             const uint32_t* seg_cnt,
                                                             const uint2* row_rg,
                                                             const uint2* rows) {
  __shared__ uint32_t buf[TS_BUF];                       // pair ids, grouped by tile
  __shared__ uint16_t bcol[TS_BUF];                      // tile column of each slot
  __shared__ unsigned long long wm[TS_WAVES][MAX_COLS];  // per-wave spanning masks
  __shared__ uint32_t woff[TS_WAVES][MAX_COLS];          // first slot per (wave, column)
  __shared__ uint32_t cur[MAX_COLS];                     // next list position per tile
  __shared__ uint32_t dst[MAX_COLS];                     // list position of slot 0's run
  __shared__ uint32_t wtot[TS_WAVES];
  __shared__ int wlo[TS_WAVES], whi[TS_WAVES], wfit[TS_WAVES];
  __shared__ uint32_t batch_tot;
  if (st.hdr->overflow) return;
  const int nrows = t.nv * t.TY;
  const uint32_t nseg = seg_off[nrows];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int TX = t.TX;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (uint32_t s = (uint32_t)xcd_remap(blockIdx.x, gridDim.x); s < nseg; s += gridDim.x) {
    int r;
    uint32_t lo, hi;
    seg_range(seg_off, seg_row, row_rg, s, r, lo, hi);
    const uint2* trg = st.ranges + (size_t)r * TX;
    // every thread has passed the previous segment's last read of cur
    __syncthreads();
    for (int x = tid; x < TX; x += TS_THREADS) cur[x] = trg[x].x + seg_cnt[(size_t)s * TX + x];
    uint2 e = lo + (uint32_t)tid < hi ? rows[lo + tid] : make_uint2(0u, 0u);
    for (uint32_t base = lo; base < hi;) {
      const bool valid = base + (uint32_t)tid < hi;
      const int x0 = (int)(e.y & 0xFFFF), x1 = (int)(e.y >> 16);
      const uint32_t wid = valid ? (uint32_t)(x1 - x0) : 0u;
      // inclusive prefix of the widths over the batch, in list order
      uint32_t incl = wave_incl_scan(wid);
      if (lane == 63) wtot[w] = incl;
      __syncthreads();
      for (int q = 0; q < w; ++q) incl += wtot[q];
      // the prefix is non-decreasing, so the entries that fit are a prefix
      // of the batch (at least one: a width is at most MAX_COLS)
      const bool fit = valid && incl <= (uint32_t)TS_BUF;
      int clo = fit ? x0 : TX, chi = fit ? x1 : 0;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        clo = min(clo, __shfl_xor(clo, d, 64));
        chi = max(chi, __shfl_xor(chi, d, 64));
      }
      for (int x = clo; x < chi; ++x) {
        const unsigned long long m = __ballot(fit && x0 <= x && x < x1);
        if (lane == 0) wm[w][x] = m;
      }
      const unsigned long long fm = __ballot(fit);
      if (lane == 0) {
        wlo[w] = clo;
        whi[w] = chi;
        wfit[w] = __popcll(fm);
      }
      __syncthreads();
      uint32_t nfit = 0;
#pragma unroll
      for (int q = 0; q < TS_WAVES; ++q) nfit += (uint32_t)wfit[q];
      // wave 0: per-column counts, slot bases and list destinations
      if (w == 0) {
        uint32_t carry = 0;
        for (int xb = 0; xb < TX; xb += 64) {
          const int x = xb + lane;
          uint32_t c[TS_WAVES], n = 0;
#pragma unroll
          for (int q = 0; q < TS_WAVES; ++q) {
            c[q] = (x < TX && x >= wlo[q] && x < whi[q]) ? (uint32_t)__popcll(wm[q][x]) : 0u;
            n += c[q];
          }
          const uint32_t inc = wave_incl_scan(n) + carry;
          if (x < TX) {
            uint32_t o = inc - n;
            const uint32_t c0 = cur[x];
            dst[x] = c0 - o;  // slot k of column x goes to list position dst[x] + k
            cur[x] = c0 + n;
#pragma unroll
            for (int q = 0; q < TS_WAVES; ++q) {
              woff[q][x] = o;
              o += c[q];
            }
          }
          carry = __shfl(inc, 63, 64);
        }
        if (lane == 0) batch_tot = carry;
      }
      __syncthreads();
      if (fit)
        for (int x = x0; x < x1; ++x) {
          const uint32_t slot = woff[w][x] + (uint32_t)__popcll(wm[w][x] & lt);
          buf[slot] = e.x;
          bcol[slot] = (uint16_t)x;
        }
      // next batch's entries are in flight while this one is copied out
      const uint32_t nb = base + nfit;
      e = nb + (uint32_t)tid < hi ? rows[nb + tid] : make_uint2(0u, 0u);
      __syncthreads();
      const uint32_t n = batch_tot;
      for (uint32_t k = (uint32_t)tid; k < n; k += TS_THREADS) {
        const uint32_t pos = dst[bcol[k]] + k;
        if (pos < st.cap) st.inst[pos] = buf[k];
      }
      base = nb;
    }
  }
}

hipError_t launch_binning(const BinTab& t, StateDev st, const BinWork& w, hipStream_t s) {
  const int nc = t.cblk_off[t.nv];
  const int nrows = t.nv * t.TY;
  // level 1: rows
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
  // level 2: tiles, per row segment
  hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, s, nrows, w.row_rg, w.seg_off,
                     w.seg_row, w.row_flag);
  hipLaunchKernelGGL(k_tile_count, dim3(w.seg_grid), dim3(256), 0, s, nrows, t.TX, w.seg_off,
                     w.seg_row, w.row_rg, w.rows, w.seg_cnt);
  hipLaunchKernelGGL(k_seg_colscan, dim3((nrows * t.TX + 255) / 256), dim3(256), 0, s, nrows,
                     t.TX, w.seg_off, w.seg_cnt, w.tile_cnt);
  hipLaunchKernelGGL(k_range_scan, dim3(1), dim3(1024), 0, s, t.nv * t.T, w.tile_cnt, st.ranges,
                     st.cap, &st.hdr->inst_total, &st.hdr->overflow, w.row_flag,
                     &st.hdr->row_total);
  hipLaunchKernelGGL(k_tile_scatter, dim3(w.seg_grid), dim3(TS_THREADS), 0, s, t, st, w.seg_off,
                     w.seg_row, w.seg_cnt, w.row_rg, w.rows);
  return hipGetLastError();
}

}  // namespace gsr
