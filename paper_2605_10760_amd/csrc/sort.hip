// Depth sort of the visible pairs: a stable LSD radix sort, 8-bit digits,
// segmented by view.
//
// The (tile, depth) key of a tile instance is sorted least-significant digit
// first.  Every instance of a pair shares the pair's depth, so the four
// depth digits are sorted on the visible pairs (before duplication, far
// fewer elements); the tile digit is the last pass and is done by the
// binning kernels.  Each view's visible pairs form a contiguous segment, so
// sorting segments independently equals sorting by (view, depth).
//
// A pass is three kernels: per-block digit histograms (LDS atomics, one per
// wave when the wave's keys share a digit, as the high depth digits mostly
// do, else one per digit present in the wave for the top digit), one
// workgroup per view turning the [block][digit] counts into
// scatter bases in (digit, block) order (a separate array: the scatter also
// reads its block's counts), and a scatter where each 256-key round is
// ranked stably inside the block by wave64 ballots over the digit bits, the
// block is reordered by digit in LDS and written out in runs.
#include "common.h"

namespace gsr {

__device__ __forceinline__ void sort_block_range(const SortTab& t, const StateHeader* hdr,
                                                 int b, int& v, int& lo, int& hi) {
  v = find_seg(t.sblk_off, t.nv, b);
  const int lb = b - t.sblk_off[v];
  const int seg_lo = (int)hdr->vis_off[v], seg_hi = (int)hdr->vis_off[v + 1];
  lo = seg_lo + lb * SORT_TILE;
  hi = min(seg_hi, lo + SORT_TILE);
}

template <int SH>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(SortTab t, const StateHeader* hdr,
                                                             const uint32_t* keys,
                                                             uint32_t* hist) {
  __shared__ uint32_t cnt[RADIX];
  const int b = xcd_remap(blockIdx.x, t.sblk_off[t.nv]);
  if (b < 0) return;
  int v, lo, hi;
  sort_block_range(t, hdr, b, v, lo, hi);
  cnt[threadIdx.x] = 0;
  __syncthreads();
  uint32_t d[SORT_ITEMS];
#pragma unroll
  for (int r = 0; r < SORT_ITEMS; ++r) {
    const int i = lo + r * SORT_THREADS + (int)threadIdx.x;
    d[r] = i < hi ? (keys[i] >> SH) & (RADIX - 1) : RADIX;
  }
#pragma unroll
  for (int r = 0; r < SORT_ITEMS; ++r) {
    const bool valid = d[r] < (uint32_t)RADIX;
    const unsigned long long act = __ballot(valid);
    if (act == 0ull) continue;  // uniform
    // the first valid lane's digit; a wave whose keys all share it adds them
    // with one atomic
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d[r], (int)__builtin_ctzll(act));
    if (__ballot(valid && d[r] == d0) == act) {
      if (lane_id() == (int)__builtin_ctzll(act)) atomicAdd(&cnt[d0], (uint32_t)__popcll(act));
    } else if (SH >= 24) {
      // the top digit takes few values: the lanes sharing a digit (found by
      // a ballot per digit bit) add their count with one atomic from the
      // lowest of them
      unsigned long long peers = act;
#pragma unroll
      for (int bit = 0; bit < RADIX_BITS; ++bit) {
        const bool on = (d[r] >> bit) & 1u;
        const unsigned long long bb = __ballot(on);
        peers &= on ? bb : ~bb;
      }
      const unsigned long long lt = (1ull << lane_id()) - 1ull;
      if (valid && (peers & lt) == 0ull) atomicAdd(&cnt[d[r]], (uint32_t)__popcll(peers));
    } else if (valid) {
      atomicAdd(&cnt[d[r]], 1u);
    }
  }
  __syncthreads();
  hist[(size_t)b * RADIX + threadIdx.x] = cnt[threadIdx.x];
}

// One workgroup per view; thread (q, d) owns digit d over the q-th quarter
// of the view's blocks (the walk down the blocks is 4x shorter).  Writes the
// scatter base of every (block, digit) into off; the counts stay in hist.
constexpr int SCAN_Q = 4;
__global__ __launch_bounds__(RADIX* SCAN_Q) void k_radix_scan(SortTab t, const StateHeader* hdr,
                                                             const uint32_t* hist,
                                                             uint32_t* off) {
  __shared__ unsigned long long sh[RADIX * SCAN_Q / 64 + 1];
  __shared__ uint32_t part[SCAN_Q][RADIX];
  __shared__ uint32_t dex[RADIX];
  const int v = blockIdx.x;
  const int d = (int)threadIdx.x & (RADIX - 1), q = (int)threadIdx.x / RADIX;
  const int n = (int)(hdr->vis_off[v + 1] - hdr->vis_off[v]);
  const int nb = (n + SORT_TILE - 1) / SORT_TILE;
  const int b0 = nb * q / SCAN_Q, b1 = nb * (q + 1) / SCAN_Q;
  const size_t base = (size_t)t.sblk_off[v] * RADIX + d;
  const uint32_t* h = hist + base;
  uint32_t* o = off + base;
  uint32_t tot = 0;
  int b = b0;
  for (; b + 8 <= b1; b += 8) {
    uint32_t x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = h[(size_t)(b + k) * RADIX];
#pragma unroll
    for (int k = 0; k < 8; ++k) tot += x[k];
  }
  for (; b < b1; ++b) tot += h[(size_t)b * RADIX];
  part[q][d] = tot;
  __syncthreads();
  uint32_t dtot = 0, before = 0;
#pragma unroll
  for (int k = 0; k < SCAN_Q; ++k) {
    const uint32_t x = part[k][d];
    dtot += x;
    before += k < q ? x : 0u;
  }
  // exclusive scan of the digit totals over the digits: the q = 0 threads
  // (the first RADIX of the workgroup) carry them, the others add zero
  unsigned long long all;
  const uint32_t ex = (uint32_t)wg_excl_scan<RADIX * SCAN_Q>(q == 0 ? dtot : 0u, sh, &all);
  if (q == 0) dex[d] = ex;
  __syncthreads();
  uint32_t run = hdr->vis_off[v] + dex[d] + before;
  b = b0;
  for (; b + 8 <= b1; b += 8) {
    uint32_t x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = h[(size_t)(b + k) * RADIX];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      o[(size_t)(b + k) * RADIX] = run;
      run += x[k];
    }
  }
  for (; b < b1; ++b) {
    o[(size_t)b * RADIX] = run;
    run += h[(size_t)b * RADIX];
  }
}

// Stable scatter.  Keys of round r are the 256 consecutive keys
// lo + r*256 + tid; within a round lower threads go first, earlier rounds go
// before later ones, so equal digits keep their input order.  The block's
// keys are first placed in LDS in digit order (each key's slot is its
// digit's offset within the block plus its stable rank), then written out
// slot by slot: a digit's run of the block (about 8 keys) is stored by
// consecutive lanes to consecutive addresses instead of one scattered store
// per key.
template <int SH, bool KEYS_OUT, bool VAL_INDEX = false>
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    SortTab t, const StateHeader* hdr, const uint32_t* hist, const uint32_t* off,
    const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout) {
  constexpr int NW = SORT_THREADS / 64;
  __shared__ uint32_t whist[NW][RADIX];
  __shared__ uint32_t cnt[RADIX];    // keys of each digit placed so far
  __shared__ uint32_t loff[RADIX];   // first slot of each digit in the block
  __shared__ uint32_t goff[RADIX];   // output position of the block's first key of each digit
  __shared__ uint32_t lk[SORT_TILE], lv[SORT_TILE];
  __shared__ unsigned long long sh[NW + 1];
  const int b = xcd_remap(blockIdx.x, t.sblk_off[t.nv]);
  if (b < 0) return;
  int v, lo, hi;
  sort_block_range(t, hdr, b, v, lo, hi);
  if (lo >= hi) return;
  const int tid = threadIdx.x, w = tid >> 6, lane = lane_id();
  const int n = hi - lo;
  // the block's digit counts (from the histogram pass) and global bases
#pragma unroll
  for (int i = 0; i < NW; ++i) whist[i][tid] = 0;
  uint32_t key[SORT_ITEMS], val[SORT_ITEMS];
#pragma unroll
  for (int r = 0; r < SORT_ITEMS; ++r) {
    const int i = r * SORT_THREADS + tid;
    key[r] = i < n ? kin[lo + i] : 0u;
    // the first pass's values are the keys' own positions
    val[r] = i < n ? (VAL_INDEX ? (uint32_t)(lo + i) : vin[lo + i]) : 0u;
  }
  {
    unsigned long long tot;
    const uint32_t c = hist[(size_t)b * RADIX + tid];
    const uint32_t o = (uint32_t)wg_excl_scan<SORT_THREADS>(c, sh, &tot);
    loff[tid] = o;
    goff[tid] = off[(size_t)b * RADIX + tid];
    cnt[tid] = 0;
  }
  __syncthreads();
  const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < SORT_ITEMS; ++r) {
    if (r * SORT_THREADS >= n) break;  // uniform
    const bool valid = r * SORT_THREADS + tid < n;
    const uint32_t d = (key[r] >> SH) & (RADIX - 1);
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < RADIX_BITS; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long bb = __ballot(on);
      peers &= on ? bb : ~bb;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) whist[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t slot = loff[d] + cnt[d] + (uint32_t)rank;
      for (int j = 0; j < w; ++j) slot += whist[j][d];
      lk[slot] = key[r];
      lv[slot] = val[r];
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      add += whist[j][tid];
      whist[j][tid] = 0;
    }
    cnt[tid] += add;
    __syncthreads();
  }
  // slot e holds a key of digit d: its output position is goff[d] + e - loff[d]
#pragma unroll
  for (int r = 0; r < SORT_ITEMS; ++r) {
    const int e = r * SORT_THREADS + tid;
    if (e < n) {
      const uint32_t k = lk[e];
      const uint32_t d = (k >> SH) & (RADIX - 1);
      const uint32_t pos = goff[d] + (uint32_t)e - loff[d];
      if (KEYS_OUT) kout[pos] = k;
      vout[pos] = lv[e];
    }
  }
}

hipError_t launch_depth_sort(const SortTab& t, StateDev st, uint32_t* ka, uint32_t* va,
                             uint32_t* kb, uint32_t* vb, uint32_t* hist, uint32_t* off,
                             hipStream_t s) {
  const int nb = t.sblk_off[t.nv];
  if (nb == 0) return hipSuccess;
  const dim3 g(xcd_grid(nb)), blk(SORT_THREADS), sg(t.nv), sb(RADIX * SCAN_Q);
  // pass 0: A -> B
  hipLaunchKernelGGL(k_radix_hist<0>, g, blk, 0, s, t, st.hdr, ka, hist);
  hipLaunchKernelGGL(k_radix_scan, sg, sb, 0, s, t, st.hdr, hist, off);
  hipLaunchKernelGGL((k_radix_scatter<0, true, true>), g, blk, 0, s, t, st.hdr, hist, off, ka,
                     (const uint32_t*)nullptr, kb, vb);
  // pass 1: B -> A
  hipLaunchKernelGGL(k_radix_hist<8>, g, blk, 0, s, t, st.hdr, kb, hist);
  hipLaunchKernelGGL(k_radix_scan, sg, sb, 0, s, t, st.hdr, hist, off);
  hipLaunchKernelGGL((k_radix_scatter<8, true>), g, blk, 0, s, t, st.hdr, hist, off, kb, vb, ka,
                     va);
  // pass 2: A -> B
  hipLaunchKernelGGL(k_radix_hist<16>, g, blk, 0, s, t, st.hdr, ka, hist);
  hipLaunchKernelGGL(k_radix_scan, sg, sb, 0, s, t, st.hdr, hist, off);
  hipLaunchKernelGGL((k_radix_scatter<16, true>), g, blk, 0, s, t, st.hdr, hist, off, ka, va, kb,
                     vb);
  // pass 3: B -> state order (values only)
  hipLaunchKernelGGL(k_radix_hist<24>, g, blk, 0, s, t, st.hdr, kb, hist);
  hipLaunchKernelGGL(k_radix_scan, sg, sb, 0, s, t, st.hdr, hist, off);
  hipLaunchKernelGGL((k_radix_scatter<24, false>), g, blk, 0, s, t, st.hdr, hist, off, kb, vb,
                     (uint32_t*)nullptr, st.order);
  return hipGetLastError();
}

}  // namespace gsr
