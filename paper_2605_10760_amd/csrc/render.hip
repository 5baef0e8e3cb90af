// Per-tile compositing, forward and backward.
//
// Forward: one wave per (view, tile), PPL = TW*TH/64 pixels per lane (one per
// 8x8 block of the tile), TPW tiles per workgroup with a private LDS slice
// each (no workgroup barrier).  The tile's list is walked in rounds of B
// entries: each lane gathers its entries' 48-byte records into
// the slice and tests which of the tile's 8x8 blocks each can reach; then
// the wave walks the round in list order, every lane reading the entry once
// (an LDS broadcast) for all of its pixels in the blocks the entry reaches.
// The tile stops once every pixel has terminated.
//
// Backward: one wave per (view, region), a region being one tile or two
// adjacent tiles of a tile row, PPL = region pixels / 64 per lane, TPW
// regions per workgroup with a private LDS slice each (no workgroup
// barrier).  Each tile's entries up to the largest last-contributor position
// are filtered from its row list back to front; every pixel recovers its
// transmittance by division (T_j = T_{j+1} / (1 - alpha_j)) instead of
// storing per-pixel lists, the ten splat gradients of an entry are summed
// over the wave by a transposing butterfly (DPP row operations and row
// swaps), and a dense pass per staging round turns the round's sums into
// screen-space gradients with one global atomic per (entry, value).
//
// A tile's list (its entries in depth order) is its row list filtered by
// column: both kernels scan the row list with a ballot per 64 entries and
// keep the covering entries' visible positions in a ring in LDS, so only the
// prefix of the row list a tile needs is ever read.
#include <algorithm>

#include "common.h"

namespace gsr {

constexpr float ALPHA_MAX = 0.99f;
constexpr float ALPHA_MIN = 1.0f / 255.0f;
constexpr float T_MIN = 1e-4f;

constexpr float LN2 = 0.6931471805599453f;

// Exponent of a splat at a pixel sample point, in base 2: the record holds
// the conic pre-scaled by -log2(e)/2 (A, C) and -log2(e) (B), so
// G = 2^p with p = A' dx^2 + B' dx dy + C' dy^2.  The operation sequence is
// spelled out (explicit fma, no other contraction) so the forward and the
// backward take identical skip decisions.
// The terms that depend on the pixel row only (B' dy and C' dy^2) are formed
// once per row of 8x8 blocks and shared by the blocks of that row; the
// result is the same sequence of roundings as the one-call form.
struct SplatRow {
  float bdy, cdy2;
};
__device__ __forceinline__ SplatRow splat_row(const float4& a, const float4& b, float fy) {
#pragma clang fp contract(off)
  const float dy = a.y - fy;
  return SplatRow{a.w * dy, (b.x * dy) * dy};
}
__device__ __forceinline__ float splat_power_row(const float4& a, const SplatRow& r, float fx) {
#pragma clang fp contract(off)
  const float dx = a.x - fx;
  // dx (A' dx + B' dy) + C' dy^2
  return fmaf(dx, fmaf(a.z, dx, r.bdy), r.cdy2);
}
__device__ __forceinline__ float splat_power(const float4& a, const float4& b, float fx, float fy) {
  return splat_power_row(a, splat_row(a, b, fy), fx);
}

__device__ __forceinline__ float exp2_fast(float p) { return __builtin_amdgcn_exp2f(p); }

// 1/x by the hardware reciprocal (about 1 ulp); the backward's transmittance
// recovery T_j = T_{j+1} / (1 - alpha_j) and its opacity gradient (a division
// by sigma > 1/255) use it instead of an IEEE division (x is far from
// denormal in both).
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// Whether the splat's alpha >= 1/255 region can reach a pixel centre of the
// box [x0, x1] x [y0, y1], in two parts: row_extent gives the region's x
// extent [xl, xr] within the pixel-centre rows y0..y1 (false: the rows miss
// it), cols_reached tests that extent against the columns.  The region is the ellipse
// a dx^2 + b dx dy + c dy^2 <= t (a = -A', b = -B', c = -C', dx = x - u,
// dy = y - v); taking t so that its y half-extent equals the record's
// conservative ey (which carries a margin) gives an ellipse containing the
// region.  Within the rows y0..y1 its x extent is reached at the clamped
// dy of the ellipse's leftmost / rightmost points (the right boundary
// x(dy) = u + (-b dy + sqrt(4ac - b^2) sqrt(ey^2 - dy^2)) / 2a is concave,
// the left one convex), and the comparison carries a further margin for
// the FP32 arithmetic.  Square roots and reciprocals are the hardware
// approximations (about 1 ulp, no correctly-rounded expansion): their error
// is orders of magnitude inside that margin.  NaN inputs give true.
__device__ __forceinline__ bool row_extent(const float4& r0, float Cs, float ey, float y0, float y1,
                                           float& xl, float& xr) {
  const float a = -r0.z, b = -r0.w, c = -Cs;
  const float lo = fmaxf(y0 - r0.y, -ey), hi = fminf(y1 - r0.y, ey);
  if (lo > hi) return false;
  const float sd = __builtin_amdgcn_sqrtf(fmaxf(4.f * a * c - b * b, 0.f));
  const float ys = 0.5f * b * ey * __builtin_amdgcn_rsqf(a * c);
  const float yr = fminf(fmaxf(-ys, lo), hi), yl = fminf(fmaxf(ys, lo), hi);
  const float wr = sd * __builtin_amdgcn_sqrtf(fmaxf((ey - yr) * (ey + yr), 0.f));
  const float wl = sd * __builtin_amdgcn_sqrtf(fmaxf((ey - yl) * (ey + yl), 0.f));
  const float h = 0.5f * __builtin_amdgcn_rcpf(a);
  xr = r0.x + (wr - b * yr) * h;
  xl = r0.x - (wl + b * yl) * h;
  return true;
}
__device__ __forceinline__ bool cols_reached(float xl, float xr, float ex, float x0, float x1) {
  const float m = 0.05f + 1e-3f * ex;
  return !(xr + m < x0 || xl - m > x1);
}
__device__ __forceinline__ bool reaches(const float4& r0, float Cs, float ex, float ey, float x0,
                                        float x1, float y0, float y1) {
  float xl, xr;
  return row_extent(r0, Cs, ey, y0, y1, xl, xr) && cols_reached(xl, xr, ex, x0, x1);
}

// Ring of visible positions filtered from a row list (slots mod RING), in
// the wave's LDS.  A round stages up to B entries; the ring is filled while
// it holds fewer than B, two scan steps (128 row entries) at a time, so it
// never holds more than B + 127.
template <int B>
struct RingSize {
  static constexpr int value = B <= 128 ? 256 : 512;
};

// Whether tile column tx lies in the row entry's column span [x0, x1).
__device__ __forceinline__ bool covers(uint32_t xs, uint32_t tx) {
  return tx - (xs & 0xFFFFu) < (xs >> 16) - (xs & 0xFFFFu);
}

// Front to back: append the visible positions of the row entries at
// [q, end) that cover column tx to the ring until it holds B or the list
// ends; q advances past what was scanned.
template <int B>
__device__ __forceinline__ void fill_front(const uint2* rows, uint32_t& q, uint32_t end,
                                           uint32_t tx, uint32_t* ring, uint32_t head,
                                           uint32_t& tail) {
  constexpr uint32_t RM = RingSize<B>::value - 1;
  const int lane = threadIdx.x & 63;
  while (tail - head < (uint32_t)B && q < end) {
    uint2 e[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const uint32_t i = q + (uint32_t)(64 * k + lane);
      e[k] = i < end ? rows[i] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const bool cov = covers(e[k].y, tx);
      const unsigned long long m = __ballot(cov);
      if (cov)
        ring[(tail + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))) &
             RM] = e[k].x;
      tail += (uint32_t)__popcll(m);
    }
    q += 128u;
  }
}

// Back to front: append the visible positions (and, for CP > 1, the column
// spans) of the row entries at [start, q) that cover one of the CP columns
// tx0 .. tx0 + CP - 1 to the ring, in decreasing position, until it holds B
// or the scan reaches start; q moves down past what was scanned.
template <int B, int CP>
__device__ __forceinline__ void fill_back(const uint2* rows, uint32_t& q, uint32_t start,
                                          uint32_t tx0, uint32_t* ring, uint32_t* ringx,
                                          uint32_t head, uint32_t& tail) {
  constexpr uint32_t RM = RingSize<B>::value - 1;
  const int lane = threadIdx.x & 63;
  const unsigned long long above = lane == 63 ? 0ull : (~0ull << (lane + 1));
  while (tail - head < (uint32_t)B && q > start) {
    uint2 e[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      // step k covers [q - 64 (k + 1), q - 64 k); lane l takes its entry l
      const uint32_t back = (uint32_t)(64 * (k + 1) - lane);
      e[k] = q - start >= back ? rows[q - back] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      bool cov = false;
#pragma unroll
      for (int c = 0; c < CP; ++c) cov = cov || covers(e[k].y, tx0 + (uint32_t)c);
      const unsigned long long m = __ballot(cov);
      // higher lanes (later entries) take the lower ring slots
      if (cov) {
        const uint32_t slot = (tail + (uint32_t)__popcll(m & above)) & RM;
        ring[slot] = e[k].x;
        if (CP > 1) ringx[slot] = e[k].y;
      }
      tail += (uint32_t)__popcll(m);
    }
    q = q - start > 128u ? q - 128u : start;
  }
}

// For CP columns tx0 + c with n[c] entries each to walk: the row position
// qb just after the last of the n[c]-th entries covering column tx0 + c
// (start when every n[c] is 0), and top[c], the number of entries of
// [start, qb) covering each column (n[c] for the column that ends last).
template <int CP>
__device__ __forceinline__ uint32_t cover_ends(const uint2* rows, uint32_t start, uint32_t end,
                                               uint32_t tx0, const uint32_t* n, uint32_t* top) {
  const int lane = threadIdx.x & 63;
  uint32_t cnt[CP], qe[CP];
  bool found[CP];
  bool all = true;
#pragma unroll
  for (int c = 0; c < CP; ++c) {
    cnt[c] = 0u;
    qe[c] = start;
    found[c] = n[c] == 0u;
    all = all && found[c];
    top[c] = 0u;
  }
  if (all) return start;
  for (uint32_t q = start; q < end; q += 64u) {
    const uint32_t i = q + (uint32_t)lane;
    const uint32_t xs = i < end ? rows[i].y : 0u;
    unsigned long long m[CP];
#pragma unroll
    for (int c = 0; c < CP; ++c) {
      const bool cov = covers(xs, tx0 + (uint32_t)c);
      m[c] = __ballot(cov);
      const uint32_t pc = (uint32_t)__popcll(m[c]);
      if (!found[c] && cnt[c] + pc >= n[c]) {
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m[c] >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m[c], 0u));
        const unsigned long long hit = __ballot(cov && rank == n[c] - cnt[c] - 1u);
        qe[c] = q + (uint32_t)__builtin_ctzll(hit) + 1u;
        found[c] = true;
      }
    }
    all = true;
#pragma unroll
    for (int c = 0; c < CP; ++c) all = all && found[c];
    if (all) {
      uint32_t qb = start;
#pragma unroll
      for (int c = 0; c < CP; ++c) qb = max(qb, qe[c]);
      // qb lies in this step: the covering entries before it
      const uint32_t in = qb - q;  // 1..64
      const unsigned long long low = in >= 64u ? ~0ull : ((1ull << in) - 1ull);
#pragma unroll
      for (int c = 0; c < CP; ++c) top[c] = cnt[c] + (uint32_t)__popcll(m[c] & low);
      return qb;
    }
#pragma unroll
    for (int c = 0; c < CP; ++c) cnt[c] += (uint32_t)__popcll(m[c]);
  }
  // fewer covering entries than asked (not reached for a consistent state)
#pragma unroll
  for (int c = 0; c < CP; ++c) top[c] = cnt[c];
  return end;
}

// The row position just after the n-th (1-based) entry of [q, end) that
// covers column tx; end when there are fewer.
__device__ __forceinline__ uint32_t nth_cover_end(const uint2* rows, uint32_t q, uint32_t end,
                                                  uint32_t tx, uint32_t n) {
  const int lane = threadIdx.x & 63;
  uint32_t cnt = 0u;
  while (q < end) {
    uint32_t xs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t i = q + (uint32_t)(64 * k + lane);
      xs[k] = i < end ? rows[i].y : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool cov = covers(xs[k], tx);
      const unsigned long long m = __ballot(cov);
      const uint32_t c = (uint32_t)__popcll(m);
      if (cnt + c >= n) {
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const unsigned long long hit = __ballot(cov && rank == n - cnt - 1u);
        return q + (uint32_t)(64 * k) + (uint32_t)__builtin_ctzll(hit) + 1u;
      }
      cnt += c;
    }
    q += 256u;
  }
  return end;
}

// One tile of the forward on one wave.  Lane l shades pixel (l % 8, l / 8)
// of each of the tile's PPL 8x8 blocks.  The tile's list is its row list
// filtered by column; B entries are staged per round in the wave's LDS
// slice, with a mask per entry of the blocks it can reach.
template <int TW, int TH, int B, bool NEVAL>
__device__ __forceinline__ void fwd_tile(int g, int W, int H, int TX, int TY, const CamDev& cam,
                                         const StateDev& st, float* color, float* depth,
                                         float* alpha, int32_t* n_eval, float4* s0, float4* s1,
                                         float4* s2, uint32_t* ring) {
  constexpr int PPL = TW * TH / 64, BX = TW / 8, BY = TH / 8, R = B / 64;
  static_assert(TW % 8 == 0 && TH % 8 == 0, "tiles are made of 8x8 blocks");
  static_assert(PPL <= 32, "one mask bit per block");
  const int T = TX * TY;
  const int v = g / T, tl = g - v * T;
  const int ty = tl / TX, tx = tl - ty * TX;
  const int lane = threadIdx.x & 63;
  uint2 rr = st.row_rg[(size_t)v * TY + ty];
  if (st.hdr->overflow) rr = make_uint2(0u, 0u);
  constexpr uint32_t RM = RingSize<B>::value - 1;
  uint32_t q = rr.x, head = 0u, tail = 0u;  // next row entry to scan; ring cursors
  uint32_t tbase = 0u;                      // tile entries staged before this round
  // pixel k of the lane: block (k % BX, k / BX); its centre is exact in FP32
  const float fx0 = (float)(tx * TW + (lane & 7)) + 0.5f;
  const float fy0 = (float)(ty * TH + (lane >> 3)) + 0.5f;
  // thr: the pixel's alpha threshold, 1/255 while it runs; once it has
  // stopped (and from the start for a pixel outside the image) a value no
  // alpha reaches (alpha <= 0.99, and the clamp maps a NaN product to 0.99),
  // so a stopped pixel needs no test of its own: 2, or, when the entry
  // counts are wanted, 2 + the 1-based position of the entry at which it
  // stopped (exact below 2^24 entries)
  float Tc[PPL], c0[PPL], c1[PPL], c2[PPL], dz[PPL], thr[PPL];
  uint32_t last[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int px = tx * TW + 8 * (k % BX) + (lane & 7);
    const int py = ty * TH + 8 * (k / BX) + (lane >> 3);
    thr[k] = (px < W && py < H) ? ALPHA_MIN : 2.f;
    Tc[k] = 1.f;
    c0[k] = c1[k] = c2[k] = dz[k] = 0.f;
    last[k] = 0u;
  }
  // pixel-centre corner of the tile
  const float x0c = (float)(tx * TW) + 0.5f;
  const float y0c = (float)(ty * TH) + 0.5f;
  bool live = true;
  for (;;) {
    fill_front<B>(st.rows, q, rr.y, (uint32_t)tx, ring, head, tail);
    const uint32_t n = min((uint32_t)B, tail - head);
    if (n == 0u) break;
    // bit k of mr[r]: the entry this lane staged in round r can reach alpha
    // >= 1/255 in block k (the extent within a block row is shared by the
    // blocks of that row)
    uint32_t mr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t idx = (uint32_t)(lane + 64 * r);
      mr[r] = 0u;
      if (idx < n) {
        const float4* rp = st.rec + 3 * (size_t)ring[(head + idx) & RM];
        const float4 r0 = rp[0], r1 = rp[1], r2 = rp[2];
        uint32_t m = 0u;
#pragma unroll
        for (int by = 0; by < BY; ++by) {
          float xl, xr;
          if (row_extent(r0, r1.x, r2.w, y0c + (float)(8 * by), y0c + (float)(8 * by + 7), xl, xr)) {
#pragma unroll
            for (int bx = 0; bx < BX; ++bx)
              m |= (uint32_t)cols_reached(xl, xr, r1.w, x0c + (float)(8 * bx),
                                          x0c + (float)(8 * bx + 7))
                   << (by * BX + bx);
          }
        }
        s0[lane + 64 * r] = r0;
        s1[lane + 64 * r] = r1;
        s2[lane + 64 * r] = r2;
        mr[r] = m;
      }
    }
    __builtin_amdgcn_wave_barrier();
    // In list order over the staged entries that reach a block of the tile
    // (set bits of a ballot per staging round).  Branch-free per pixel: a
    // finished or skipped pixel takes a zero weight (adding an exact zero
    // leaves the sums unchanged); a block the entry cannot reach is not
    // evaluated at all (a uniform branch on the entry's mask).
#pragma unroll
    for (int r = 0; r < R; ++r) {
      unsigned long long rel = __ballot(mr[r] != 0u);
      while (rel) {
        float run = thr[0];
#pragma unroll
        for (int k = 1; k < PPL; ++k) run = fminf(run, thr[k]);
        if (__ballot(run < 1.f) == 0ull) {
          live = false;
          break;
        }
        const int jj = (int)__builtin_ctzll(rel);
        rel &= rel - 1ull;
        const int j = 64 * r + jj;
        const uint32_t mj = (uint32_t)__builtin_amdgcn_readlane((int)mr[r], jj);
        // the entry's 1-based position, copied to a vector register once
        // for the per-pixel selects
        uint32_t pos1;
        asm volatile("v_mov_b32 %0, %1" : "=v"(pos1) : "s"(tbase + (uint32_t)j + 1u));
        const float stopv = NEVAL ? 2.f + (float)(tbase + (uint32_t)j + 1u) : 2.f;
        const float4 a = s0[j], b = s1[j], c = s2[j];
        auto blend = [&](int k, const SplatRow& rw) {
          const float p = splat_power_row(a, rw, fx0 + (float)(8 * (k % BX)));
          const float al = fminf(ALPHA_MAX, b.y * exp2_fast(p));
          const bool use = !(p > 0.f || al < thr[k]);
          // T (1 - alpha) with one rounding
          const float Tn = fmaf(-al, Tc[k], Tc[k]);
          const bool stop = use && Tn < T_MIN;
          const bool ok = use && !stop;
          thr[k] = stop ? stopv : thr[k];
          const float wgt = ok ? al * Tc[k] : 0.f;
          c0[k] += c.x * wgt;
          c1[k] += c.y * wgt;
          c2[k] += c.z * wgt;
          dz[k] += b.z * wgt;
          Tc[k] = ok ? Tn : Tc[k];
          last[k] = ok ? pos1 : last[k];
        };
#pragma unroll
        for (int by = 0; by < BY; ++by) {
          if (!((mj >> (by * BX)) & ((1u << BX) - 1u))) continue;
          const SplatRow rw = splat_row(a, b, fy0 + (float)(8 * by));
#pragma unroll
          for (int bx = 0; bx < BX; ++bx)
            if ((mj >> (by * BX + bx)) & 1u) blend(by * BX + bx, rw);
        }
      }
      if (!live) break;
    }
    if (!live) break;
    head += n;
    tbase += n;
    // the next round's staging overwrites the slice: every lane has read it
    __builtin_amdgcn_wave_barrier();
  }
  const size_t HW = (size_t)W * H;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int px = tx * TW + 8 * (k % BX) + (lane & 7);
    const int py = ty * TH + 8 * (k / BX) + (lane >> 3);
    if (px < W && py < H) {
      const size_t p = (size_t)py * W + px;
      color[(3 * (size_t)v + 0) * HW + p] = c0[k] + Tc[k] * cam.bg0;
      color[(3 * (size_t)v + 1) * HW + p] = c1[k] + Tc[k] * cam.bg1;
      color[(3 * (size_t)v + 2) * HW + p] = c2[k] + Tc[k] * cam.bg2;
      depth[v * HW + p] = dz[k];
      alpha[v * HW + p] = 1.f - Tc[k];
      st.tfinal[v * HW + p] = Tc[k];
      st.last[v * HW + p] = last[k];
      // entries examined: up to and including the stopping one, else the
      // list (every inside pixel has stopped when the walk ends early, so
      // tbase is the whole list whenever it is used)
      if (NEVAL)
        n_eval[v * HW + p] = (int)(thr[k] >= 2.f ? (uint32_t)(thr[k] - 2.f) : tbase);
    }
  }
}

// TPW waves per workgroup, each with a private LDS slice and no workgroup
// barrier.  Grid form: wave w of workgroup b takes tile b TPW + w (XCD-aware
// order).  Persistent form: a grid sized to the resident waves, each wave
// taking tiles from the length-ordered queue (longest lists first) until it
// is empty.
template <int TW, int TH, int FB, int TPW, bool PERSIST, bool NEVAL>
__global__ __launch_bounds__(64 * TPW) void k_render_fwd(int ntiles, int W, int H, int TX, int TY,
                                                         CamDev cam, StateDev st,
                                                         unsigned int* next, float* color,
                                                         float* depth, float* alpha,
                                                         int32_t* n_eval) {
  constexpr int B = 64 * FB;
  __shared__ float4 L0[TPW][B], L1[TPW][B], L2[TPW][B];
  __shared__ uint32_t LR[TPW][RingSize<B>::value];
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (!PERSIST) {
    const int blk = xcd_remap(blockIdx.x, (ntiles + TPW - 1) / TPW);
    if (blk < 0) return;
    const int g = blk * TPW + wv;
    if (g >= ntiles) return;
    fwd_tile<TW, TH, B, NEVAL>(g, W, H, TX, TY, cam, st, color, depth, alpha, n_eval, L0[wv], L1[wv],
                        L2[wv], LR[wv]);
    return;
  }
  for (;;) {
    uint32_t q = 0;
    if ((threadIdx.x & 63) == 0) q = atomicAdd(next, 1u);
    q = (uint32_t)__builtin_amdgcn_readfirstlane((int)q);
    if (q >= (uint32_t)ntiles) return;
    fwd_tile<TW, TH, B, NEVAL>((int)st.torder[q], W, H, TX, TY, cam, st, color, depth, alpha, n_eval,
                        L0[wv], L1[wv], L2[wv], LR[wv]);
    // the next tile's staging overwrites this wave's LDS slice
    __builtin_amdgcn_wave_barrier();
  }
}

// Wave sums of ten values at once, by a transposing butterfly: at each
// exchange a lane keeps half of its values and hands the other half to its
// partner, so the number of values per lane halves as the partial sums
// double (10 -> 5 -> 3 -> 2 -> 1 over lane bits 0..3, then bits 4 and 5 on
// the single value).  Lane l < 16 ends with the total of value sum10_index(l)
// (-1: no value); lanes 16..63 hold partial sums.  About 45 lane operations
// instead of 70 for ten separate reductions, none through LDS.
// z plus a second register after swapping z's odd 16-lane rows (R = 16) or
// its upper 32 lanes (R = 32) with that register's even rows / lower lanes:
// lane l of row 0 (and of row 2 for R = 16) gets z_l + z_{l+R}, whatever the
// second register held (its values reach only rows 1 and 3, or lanes 32..63,
// of the sum), so a value that is dead at this point serves and no register
// is cleared for it.  Both registers are written by the swap, so it is
// spelled out with both as in-out operands; the two wait states before it
// cover a vector write of its operands just ahead of it.
template <int R>
__device__ __forceinline__ float row_swap_sum(float z, float spare) {
  float o = spare;
  if (R == 16)
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(z), "+v"(o));
  else
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(z), "+v"(o));
  return z + o;
}

// A DPP lane move; a lane whose source lane lies outside its row reads 0
// (bound control set, so no zeroed register is needed for the old value).
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL,
                                                            0xF, 0xF, true));
}
__host__ __device__ constexpr int sum10_index(int l) {
  const int b0 = l & 1, b1 = (l >> 1) & 1, b2 = (l >> 2) & 1, b3 = (l >> 3) & 1;
  const int xi = b3 + 2 * b2, m = xi + 3 * b1;
  return (l < 16 && xi < 3 && m < 5) ? m + 5 * b0 : -1;
}
__device__ __forceinline__ float wave_sum10(const float (&v)[10], int lane) {
  const bool b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1, b3 = (lane >> 3) & 1;
  // lane bit 0 (quad_perm [1,0,3,2]): keep values 0..4 (b0 = 0) or 5..9
  float w[6];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const float keep = b0 ? v[i + 5] : v[i], send = b0 ? v[i] : v[i + 5];
    w[i] = keep + dpp_mov<0xB1>(send);
  }
  w[5] = 0.f;
  // lane bit 1 (quad_perm [2,3,0,1]): keep w 0..2 or 3..5
  float x[4];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float keep = b1 ? w[i + 3] : w[i], send = b1 ? w[i] : w[i + 3];
    x[i] = keep + dpp_mov<0x4E>(send);
  }
  x[3] = 0.f;
  // lane bit 2 (row_shl:4 from lane l+4, row_shr:4 from lane l-4)
  float y[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float keep = b2 ? x[i + 2] : x[i], send = b2 ? x[i] : x[i + 2];
    const float up = dpp_mov<0x104>(send), dn = dpp_mov<0x114>(send);
    y[i] = keep + (b2 ? dn : up);
  }
  // lane bit 3 (row_ror:8)
  float z = (b3 ? y[1] : y[0]) + dpp_mov<0x128>(b3 ? y[0] : y[1]);
  // lane bits 4 and 5: the same value index in both partners, by the row
  // swaps of the vector unit.  Swapping the odd 16-lane rows of z with the
  // even rows of a zero register leaves z's even rows in z and z's odd rows,
  // moved down one row, in the other register, so their sum holds the pair
  // totals in rows 0 and 2; the 32-lane swap adds row 2 to row 0 the same
  // way.
  // y is dead once z is formed: its registers take the swaps' second
  // operands (the first reaches rows 1 and 3 of the first sum and through
  // them lanes 16..31 of the result, the second lanes 32..63; lanes 0..15,
  // which hold the totals, depend on neither)
  return row_swap_sum<32>(row_swap_sum<16>(z, y[1]), y[0]);
}

// One tile, or CP adjacent tiles of a tile row, of the backward on one wave.
// Lane l shades pixel (l % 8, l / 8) of each of the region's PPL 8x8 blocks;
// a record staged in the wave's LDS slice (B entries) is read once per lane
// and used for its PPL pixels.  With CP = 2 the wave walks the entries that
// cover either tile (its row list filtered by two columns), and each entry
// carries its position in each tile's own list, which the pixels of that
// tile compare with their last contributor.
template <int TW, int TH, int B, int CP>
__device__ __forceinline__ void bwd_tile(int g, int W, int H, int TX, int TY,
                                         unsigned long long grad_mask, const CamDev& cam,
                                         const StateDev& st, const float* gcol, const float* gdep,
                                         const float* galp, float* grad2d, float4* s0, float4* s1,
                                         float4* s2, uint32_t* sp, uint32_t* ring, uint32_t* ringx,
                                         float* red) {
  constexpr int RW = CP * TW;           // region width
  constexpr int PPL = RW * TH / 64;
  constexpr int BX = RW / 8, HBX = TW / 8;  // blocks per region row, per tile row
  constexpr int R = B / 64;
  constexpr uint32_t RM = RingSize<B>::value - 1;
  static_assert(PPL <= 32, "one mask bit per block");
  const int TXR = (TX + CP - 1) / CP;   // regions per tile row
  const int T = TXR * TY;
  const int v = g / T, tl = g - v * T;
  if (!((grad_mask >> v) & 1ull)) return;
  if (st.hdr->overflow) return;
  const int ty = tl / TXR, tx0 = (tl - ty * TXR) * CP;
  const uint2 rr = st.row_rg[(size_t)v * TY + ty];
  if (rr.x == rr.y) return;
  const int lane = threadIdx.x & 63;
  const size_t HW = (size_t)W * H;
  // Per pixel: Q = sum over the entries behind the current one (and the
  // background) of the upstream-weighted colour and depth, minus T_final
  // times the upstream alpha gradient; then dL/dalpha_j = T_j cg_j - Q / (1 -
  // alpha_j) with cg_j = c_j . dL/dC + z_j dL/dD, and Q += w_j cg_j.
  float fxp[PPL], fyp[PPL], Tc[PPL], g0[PPL], g1[PPL], g2[PPL], gd[PPL], Q[PPL];
  uint32_t lastp[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int px = tx0 * TW + 8 * (k % BX) + (lane & 7);
    const int py = ty * TH + 8 * (k / BX) + (lane >> 3);
    fxp[k] = (float)px + 0.5f;
    fyp[k] = (float)py + 0.5f;
    Tc[k] = 1.f; lastp[k] = 0;
    g0[k] = g1[k] = g2[k] = gd[k] = 0.f;
    float ga = 0.f;
    if (px < W && py < H) {
      const size_t q = (size_t)py * W + px;
      Tc[k] = st.tfinal[v * HW + q];
      lastp[k] = st.last[v * HW + q];
      if (gcol) {
        g0[k] = gcol[(3 * (size_t)v + 0) * HW + q];
        g1[k] = gcol[(3 * (size_t)v + 1) * HW + q];
        g2[k] = gcol[(3 * (size_t)v + 2) * HW + q];
      }
      if (gdep) gd[k] = gdep[v * HW + q];
      if (galp) ga = galp[v * HW + q];
    }
    Q[k] = Tc[k] * (cam.bg0 * g0[k] + cam.bg1 * g1[k] + cam.bg2 * g2[k]) - Tc[k] * ga;
  }
  // the largest last-contributor position over each block's pixels: an
  // entry at or beyond it blends no pixel of the block
  uint32_t blast[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    uint32_t m = lastp[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
    blast[k] = (uint32_t)__builtin_amdgcn_readfirstlane((int)m);
  }
  // the lane's pixel offset within an 8x8 block
  const float lxf = (float)(lane & 7), lyf = (float)(lane >> 3);
  // the region's first pixel centre
  const float x0r = (float)(tx0 * TW) + 0.5f, y0r = (float)(ty * TH) + 0.5f;
  uint32_t nwalk[CP], top[CP];
  bool any = false;
#pragma unroll
  for (int c = 0; c < CP; ++c) nwalk[c] = 0u;
#pragma unroll
  for (int k = 0; k < PPL; ++k) nwalk[(k % BX) / HBX] = max(nwalk[(k % BX) / HBX], blast[k]);
#pragma unroll
  for (int c = 0; c < CP; ++c) any = any || nwalk[c] != 0u;
  if (!any) return;
  // The walk covers each tile's entries [0, nwalk[c]): the row entries before
  // the last of the nwalk[c]-th ones covering each column, back to front;
  // top[c] counts the entries of that range covering column tx0 + c.
  uint32_t qb;
  if (CP == 1) {
    qb = nth_cover_end(st.rows, rr.x, rr.y, (uint32_t)tx0, nwalk[0]);
    top[0] = nwalk[0];
  } else {
    qb = cover_ends<CP>(st.rows, rr.x, rr.y, (uint32_t)tx0, nwalk, top);
  }
  uint32_t head = 0u, tail = 0u;  // ring cursors
  for (;;) {
    fill_back<B, CP>(st.rows, qb, rr.x, (uint32_t)tx0, ring, ringx, head, tail);
    const uint32_t n = min((uint32_t)B, tail - head);
    if (n == 0u) break;
    uint32_t mr[R];        // blocks the entry this lane staged in round r can reach
    uint32_t posr[CP][R];  // its position in each tile's list
    uint32_t seen[CP];     // entries covering each column staged in earlier rounds
#pragma unroll
    for (int c = 0; c < CP; ++c) seen[c] = 0u;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t idx = (uint32_t)(lane + 64 * r);
      const bool valid = idx < n;
      const uint32_t slot = (head + idx) & RM;
      const uint32_t xs = (CP > 1 && valid) ? ringx[slot] : 0u;
      bool cov[CP];
#pragma unroll
      for (int c = 0; c < CP; ++c) {
        cov[c] = valid && (CP == 1 || covers(xs, (uint32_t)(tx0 + c)));
        const unsigned long long mc = __ballot(cov[c]);
        // staged entries run back to front: the first one covering column c
        // is its tile's entry top[c] - 1
        posr[c][r] = top[c] - 1u - seen[c] -
                     __builtin_amdgcn_mbcnt_hi((uint32_t)(mc >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)mc, 0u));
        seen[c] += (uint32_t)__popcll(mc);
      }
      mr[r] = 0u;
      if (valid) {
        const uint32_t pr = ring[slot];
        const float4* rp = st.rec + 3 * (size_t)pr;
        const float4 r0 = rp[0], r1 = rp[1], r2 = rp[2];
        // bit k: the entry can reach alpha >= 1/255 in the region's 8x8 block
        // k, within a tile whose list holds it, ahead of the block's last
        // contributor
        const float x0c = (float)(tx0 * TW) + 0.5f, y0c = (float)(ty * TH) + 0.5f;
        uint32_t m = 0u;
#pragma unroll
        for (int by = 0; by < TH / 8; ++by) {
          float xl, xr;
          if (row_extent(r0, r1.x, r2.w, y0c + (float)(8 * by), y0c + (float)(8 * by + 7), xl, xr)) {
#pragma unroll
            for (int bx = 0; bx < BX; ++bx)
              m |= (uint32_t)(cov[bx / HBX] && posr[bx / HBX][r] < blast[by * BX + bx] &&
                              cols_reached(xl, xr, r1.w, x0c + (float)(8 * bx),
                                           x0c + (float)(8 * bx + 7)))
                   << (by * BX + bx);
          }
        }
        s0[idx] = r0;
        s1[idx] = r1;
        s2[idx] = r2;
        // the entry's screen-space gradient row: its visible-list position
        sp[idx] = pr;
        mr[r] = m;
      }
    }
    // the round's wave sums start at zero (entries that reach no pixel keep it)
    for (uint32_t i = (uint32_t)lane; i < n * GRAD2D; i += 64u) red[i] = 0.f;
    __builtin_amdgcn_wave_barrier();
    // Walk the staged entries (back-to-front order) that can reach a block
    // of the region (set bits of a ballot per staging round).
#pragma unroll
    for (int r = 0; r < R; ++r) {
      unsigned long long rel = __ballot(mr[r] != 0u);
      while (rel) {
        const int jj = (int)__builtin_ctzll(rel);
        rel &= rel - 1ull;
        const int j = 64 * r + jj;
        int posc[CP];
#pragma unroll
        for (int c = 0; c < CP; ++c) posc[c] = __builtin_amdgcn_readlane((int)posr[c][r], jj);
        const uint32_t mj = (uint32_t)__builtin_amdgcn_readlane((int)mr[r], jj);
        const float4 a = s0[j], b = s1[j], c = s2[j];
        float acc[GRAD2D];
#pragma unroll
        for (int i = 0; i < GRAD2D; ++i) acc[i] = 0.f;
        // per-lane sums of gp weighted by the pixel's 8x8-block offsets
        // (ix, iy): Sx8 and Sxx64 carry the factors 8 ix and 64 ix^2, Sy and
        // Syy the factors iy and iy^2, Sxy64 the factor 64 ix iy (all
        // compile-time constants once unrolled)
        float S0 = 0.f, Sx8 = 0.f, Sy = 0.f, Sxx64 = 0.f, Sxy64 = 0.f, Syy = 0.f;
        bool act = false;
        // the exponent's row terms, once per row of blocks
        SplatRow rws[TH / 8];
#pragma unroll
        for (int by = 0; by < TH / 8; ++by) rws[by] = splat_row(a, b, fyp[by * BX]);
        // Branch-free per pixel: an entry a pixel does not blend gets a zero
        // alpha (selected, never multiplied, so an infinite exp2 of a skipped
        // entry cannot leak in), hence zero weight and gradients, and keeps
        // its transmittance; adding exact zeros leaves every sum unchanged.  A block the entry cannot reach is not
        // evaluated at all (a uniform branch on the entry's mask; none of its
        // pixels would blend it).
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
          if (!((mj >> k) & 1u)) continue;
          const float power = splat_power_row(a, rws[k / BX], fxp[k]);
          const float G = exp2_fast(power);
          const float raw = b.y * G;
          const float al = fminf(ALPHA_MAX, raw);
          const bool ok = posc[(k % BX) / HBX] < (int)lastp[k] && !(power > 0.f || al < ALPHA_MIN);
          act = act || ok;
          // the alpha the pixel blends: zero for an entry it does not blend,
          // whose transmittance factor is then the reciprocal of 1, exactly 1
          const float ab = ok ? al : 0.f;
          const float inv = rcp_fast(1.f - ab);
          const float Tb = Tc[k] * inv;
          const float wgt = ab * Tb;
          const float cg = c.x * g0[k] + c.y * g1[k] + c.z * g2[k] + b.z * gd[k];
          const float dA = Tb * cg - inv * Q[k];
          Q[k] += wgt * cg;
          acc[6] += wgt * g0[k];
          acc[7] += wgt * g1[k];
          acc[8] += wgt * g2[k];
          acc[9] += wgt * gd[k];
          // unclamped: alpha = sigma G, so dL/dsigma = G dA = gp / sigma
          const float gp = raw <= ALPHA_MAX ? ab * dA : 0.f;
          const int ix = k % BX, iy = k / BX;
          S0 += gp;
          if (ix != 0) {
            Sx8 = fmaf((float)(8 * ix), gp, Sx8);
            Sxx64 = fmaf((float)(64 * ix * ix), gp, Sxx64);
          }
          if (iy != 0) { Sy = fmaf((float)iy, gp, Sy); Syy = fmaf((float)(iy * iy), gp, Syy); }
          if (ix != 0 && iy != 0) Sxy64 = fmaf((float)(64 * ix * iy), gp, Sxy64);
          Tc[k] = Tb;
        }
        // moments of gp over the pixels' offsets (u, v) from the region's
        // first pixel centre: pixel k of the lane sits at u = lx + 8 ix, v =
        // ly + 8 iy.  Values 0..4 carry sum gp u, sum gp v, sum gp u^2, sum gp
        // u v, sum gp v^2 and value 5 sum gp; the output pass turns them into
        // moments over (dx, dy) = (DX - u, DY - v) with the entry's offset
        // (DX, DY) once per entry.
        {
          const float Sy8 = 8.f * Sy;
          acc[5] = S0;
          acc[0] = fmaf(lxf, S0, Sx8);
          acc[1] = fmaf(lyf, S0, Sy8);
          acc[2] = fmaf(lxf, acc[0] + Sx8, Sxx64);
          acc[3] = fmaf(lxf, acc[1], fmaf(lyf, Sx8, Sxy64));
          acc[4] = fmaf(lyf, acc[1] + Sy8, 64.f * Syy);
        }
        if (__ballot(act) != 0ull) {
          static_assert(GRAD2D == 10, "ten splat gradients");
          const float tot = wave_sum10(acc, lane);
          const int idx = sum10_index(lane);
          if (idx >= 0) red[GRAD2D * j + idx] = tot;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    // The round's wave sums to screen-space gradients, one (entry, value)
    // per lane, and one atomic each (zero results, as for entries no pixel
    // blended, are skipped).  With (DX, DY) the entry's offset from the
    // region's first pixel centre and T0, TU, TV, TUU, TUV, TVV the sums of
    // gp, gp u, gp v, gp u^2, gp u v, gp v^2: sum gp dx = DX T0 - TU, sum gp
    // dx^2 = DX (DX T0 - 2 TU) + TUU, sum gp dx dy = DX (DY T0 - TV) - DY TU +
    // TUV, and likewise for dy; d(power)/du = -(A dx + B dy) = ln2 (2A' dx +
    // B' dy), etc.; dL/dsigma = T0 / sigma, by the hardware reciprocal.
    for (uint32_t i0 = 0; i0 < n * GRAD2D; i0 += 64u) {
      const uint32_t i = i0 + (uint32_t)lane;
      if (i < n * GRAD2D) {
        const uint32_t j = i / GRAD2D, idx = i - j * GRAD2D;
        const float tot = red[i];
        float out = tot;
        if (idx <= 5u) {
          const float4 a = s0[j];
          const float T0 = red[GRAD2D * j + 5];
          if (idx == 5u) {
            out = tot * rcp_fast(s1[j].y);
          } else {
            const float TU = red[GRAD2D * j], TV = red[GRAD2D * j + 1];
            const float DX = a.x - x0r, DY = a.y - y0r;
            const float m0 = fmaf(DX, T0, -TU), m1 = fmaf(DY, T0, -TV);
            if (idx == 0u) {
              out = LN2 * (2.f * a.z * m0 + a.w * m1);
            } else if (idx == 1u) {
              out = LN2 * (a.w * m0 + 2.f * s1[j].x * m1);
            } else if (idx == 2u) {
              out = -0.5f * fmaf(DX, fmaf(DX, T0, -2.f * TU), tot);
            } else if (idx == 3u) {
              out = -fmaf(DX, m1, fmaf(-DY, TU, tot));
            } else {
              out = -0.5f * fmaf(DY, fmaf(DY, T0, -2.f * TV), tot);
            }
          }
        }
        if (out != 0.f) atomicAdd(grad2d + (size_t)GRAD2D * sp[j] + idx, out);
      }
    }
    head += n;
#pragma unroll
    for (int c = 0; c < CP; ++c) top[c] -= seen[c];
    // the next round's staging overwrites the slice: every lane has read it
    __builtin_amdgcn_wave_barrier();
  }
}

// TPW waves per workgroup, each with a private LDS slice and no workgroup
// barrier.  Grid form: wave w of workgroup b takes region b TPW + w
// (XCD-aware order; a region is CP adjacent tiles of a tile row).
// Persistent form (CP = 1): a grid sized to the resident waves, each wave
// taking tiles from the forward's length-ordered queue until it is empty.
// The two-tile form asks for 16 resident waves per CU: it fits in 128
// vector registers without spilling (four waves per SIMD instead of three
// at its natural 133).
template <int TW, int TH, int B, int TPW, bool PERSIST, int CP>
__global__ __launch_bounds__(64 * TPW, CP == 2 ? 16 / TPW : 1) void k_render_bwd_w(int ntiles, int W, int H, int TX, int TY,
                                                           unsigned long long grad_mask, CamDev cam,
                                                           StateDev st, unsigned int* next,
                                                           const float* gcol, const float* gdep,
                                                           const float* galp, float* grad2d) {
  static_assert(CP == 1 || !PERSIST, "the length-ordered queue holds single tiles");
  __shared__ float4 L0[TPW][B], L1[TPW][B], L2[TPW][B];
  __shared__ uint32_t LP[TPW][B];
  __shared__ uint32_t LR[TPW][RingSize<B>::value];
  __shared__ uint32_t LX[TPW][CP > 1 ? RingSize<B>::value : 1];
  __shared__ float LS[TPW][B * GRAD2D];
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (!PERSIST) {
    const int blk = xcd_remap(blockIdx.x, (ntiles + TPW - 1) / TPW);
    if (blk < 0) return;
    const int g = blk * TPW + wv;
    if (g >= ntiles) return;
    bwd_tile<TW, TH, B, CP>(g, W, H, TX, TY, grad_mask, cam, st, gcol, gdep, galp, grad2d,
                            L0[wv], L1[wv], L2[wv], LP[wv], LR[wv], LX[wv], LS[wv]);
    return;
  }
  for (;;) {
    uint32_t q = 0;
    if ((threadIdx.x & 63) == 0) q = atomicAdd(next, 1u);
    q = (uint32_t)__builtin_amdgcn_readfirstlane((int)q);
    if (q >= (uint32_t)ntiles) return;
    bwd_tile<TW, TH, B, CP>((int)st.torder[q], W, H, TX, TY, grad_mask, cam, st, gcol, gdep,
                            galp, grad2d, L0[wv], L1[wv], L2[wv], LP[wv], LR[wv], LX[wv],
                            LS[wv]);
    // the next tile's staging overwrites this wave's LDS slice: every lane
    // has finished reading it
    __builtin_amdgcn_wave_barrier();
  }
}

// Clears the pose gradients (the per-pair screen-space gradient rows are
// kept at zero between backward calls: the projection backward clears the
// rows it consumes).
__global__ __launch_bounds__(256) void k_zero_pose(float* d_pose, int nv, unsigned int* bwd_next) {
  for (int k = threadIdx.x; k < 6 * nv; k += 256) d_pose[k] = 0.f;
  // the persistent backward's tile cursor starts every call at 0
  if (threadIdx.x == 0 && bwd_next) *bwd_next = 0u;
}

// ------------------------------------------------------ tile scheduling
// The persistent forms take tiles in decreasing order of their row list's
// length (longest first, so that the last tiles to start are short ones; a
// tile's list is a share of its row's): a bucket sort by the position of the
// length's leading bit (bucket clz(len), empty rows last), per-workgroup
// bucket counts reserved with one global atomic per bucket and workgroup.
// Order within a bucket is arbitrary.
// sched: [0] forward tile cursor, [1] backward tile cursor,
// [2, 2 + NLB) bucket totals, [2 + NLB, 2 + 2 NLB) bucket fill cursors.
constexpr int NLB = 33;
__device__ __forceinline__ int len_bucket(const StateDev& st, int t, int TX, int TY) {
  const int T = TX * TY, v = t / T, ty = (t - v * T) / TX;
  const uint2 r = st.row_rg[(size_t)v * TY + ty];
  const uint32_t n = st.hdr->overflow ? 0u : r.y - r.x;
  return n ? __clz((int)n) : 32;
}

__global__ __launch_bounds__(64) void k_order_reset(unsigned int* sched) {
  for (int i = threadIdx.x; i < SCHED_WORDS; i += 64) sched[i] = 0u;
}

__global__ __launch_bounds__(1024) void k_len_hist(int ntiles, int TX, int TY, StateDev st,
                                                   unsigned int* sched) {
  __shared__ unsigned int h[NLB];
  if (threadIdx.x < NLB) h[threadIdx.x] = 0u;
  __syncthreads();
  const int t = blockIdx.x * 1024 + (int)threadIdx.x;
  if (t < ntiles) atomicAdd(&h[len_bucket(st, t, TX, TY)], 1u);
  __syncthreads();
  if (threadIdx.x < NLB && h[threadIdx.x]) atomicAdd(&sched[2 + threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(1024) void k_len_scatter(int ntiles, int TX, int TY, StateDev st,
                                                      unsigned int* sched) {
  __shared__ unsigned int h[NLB], off[NLB], fill[NLB];
  if (threadIdx.x < NLB) {
    h[threadIdx.x] = 0u;
    fill[threadIdx.x] = 0u;
  }
  __syncthreads();
  const int t = blockIdx.x * 1024 + (int)threadIdx.x;
  const int b = t < ntiles ? len_bucket(st, t, TX, TY) : 0;
  if (t < ntiles) atomicAdd(&h[b], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int run = 0;
    for (int k = 0; k < NLB; ++k) {
      off[k] = run;
      run += sched[2 + k];
    }
  }
  __syncthreads();
  if (threadIdx.x < NLB && h[threadIdx.x])
    off[threadIdx.x] += atomicAdd(&sched[2 + NLB + threadIdx.x], h[threadIdx.x]);
  __syncthreads();
  if (t < ntiles) st.torder[off[b] + atomicAdd(&fill[b], 1u)] = (uint32_t)t;
}

hipError_t launch_tile_order(int nv, int TX, int TY, StateDev st, unsigned int* sched,
                             hipStream_t s) {
  const int ntiles = nv * TX * TY;
  hipLaunchKernelGGL(k_order_reset, dim3(1), dim3(64), 0, s, sched);
  const int nb = (ntiles + 1023) / 1024;
  if (nb > 0) {
    hipLaunchKernelGGL(k_len_hist, dim3(nb), dim3(1024), 0, s, ntiles, TX, TY, st, sched);
    hipLaunchKernelGGL(k_len_scatter, dim3(nb), dim3(1024), 0, s, ntiles, TX, TY, st, sched);
  }
  return hipGetLastError();
}

// Workgroups of `kernel` (block threads) resident on the whole device at
// once: the persistent grid.
static int resident_blocks(const void* kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 1024;
  }
  return std::max(1, cus) * std::max(1, per);
}

// tiles (waves) per workgroup: one, so that a wave's LDS slice and registers
// are released as soon as its tile ends (a workgroup of four held them until
// its longest tile ended: 0.72 -> 0.70 ms forward, 1.46 -> 1.39 ms backward)
constexpr int FWD_TPW = 1;

template <int TW, int TH, int FB, bool NEVAL>
static void fwd_fbn(int nv, int W, int H, int TX, int TY, bool persist, const CamDev& cam,
                    StateDev st, unsigned int* sched, float* color, float* depth, float* alpha,
                    int32_t* n_eval, hipStream_t s) {
  const int ntiles = nv * TX * TY;
  const int need = (ntiles + FWD_TPW - 1) / FWD_TPW;
  if (persist) {
    const auto k = k_render_fwd<TW, TH, FB, FWD_TPW, true, NEVAL>;
    const int grid = std::min(need, resident_blocks((const void*)k, 64 * FWD_TPW));
    hipLaunchKernelGGL(k, dim3(std::max(1, grid)), dim3(64 * FWD_TPW), 0, s, ntiles, W, H, TX, TY,
                       cam, st, sched, color, depth, alpha, n_eval);
  } else {
    hipLaunchKernelGGL((k_render_fwd<TW, TH, FB, FWD_TPW, false, NEVAL>), dim3(xcd_grid(need)),
                       dim3(64 * FWD_TPW), 0, s, ntiles, W, H, TX, TY, cam, st, sched, color,
                       depth, alpha, n_eval);
  }
}

// the per-pixel entry counts (a debug output) only in their own instantiation
template <int TW, int TH, int FB>
static void fwd_fb(int nv, int W, int H, int TX, int TY, bool persist, const CamDev& cam,
                   StateDev st, unsigned int* sched, float* color, float* depth, float* alpha,
                   int32_t* n_eval, hipStream_t s) {
  if (n_eval)
    fwd_fbn<TW, TH, FB, true>(nv, W, H, TX, TY, persist, cam, st, sched, color, depth, alpha,
                              n_eval, s);
  else
    fwd_fbn<TW, TH, FB, false>(nv, W, H, TX, TY, persist, cam, st, sched, color, depth, alpha,
                               n_eval, s);
}

template <int TW, int TH>
static hipError_t fwd_t(int nv, int W, int H, int TX, int TY, const RenderCfg& rc,
                        const CamDev& cam, StateDev st, unsigned int* sched, float* color,
                        float* depth, float* alpha, int32_t* n_eval, hipStream_t s) {
  if (rc.fwd_batch == 2)
    fwd_fb<TW, TH, 2>(nv, W, H, TX, TY, rc.persistent, cam, st, sched, color, depth, alpha,
                      n_eval, s);
  else
    fwd_fb<TW, TH, 1>(nv, W, H, TX, TY, rc.persistent, cam, st, sched, color, depth, alpha,
                      n_eval, s);
  return hipGetLastError();
}

constexpr int BWD_TPW = 1;  // regions (waves) per workgroup, as for the forward

template <int TW, int TH, int B>
static void bwd_b(int nv, int W, int H, int TX, int TY, bool persist, int cols,
                  unsigned long long mask, const CamDev& cam, StateDev st, unsigned int* sched,
                  const float* gc, const float* gd, const float* ga, float* grad2d,
                  hipStream_t s) {
  if constexpr (TW <= 16 && 2 * TW * TH <= 512) {
    if (cols == 2) {
      // two tiles of a tile row per wave (grid form only)
      const int nreg = nv * TY * ((TX + 1) / 2);
      hipLaunchKernelGGL((k_render_bwd_w<TW, TH, B, BWD_TPW, false, 2>),
                         dim3(xcd_grid((nreg + BWD_TPW - 1) / BWD_TPW)), dim3(64 * BWD_TPW), 0,
                         s, nreg, W, H, TX, TY, mask, cam, st, sched + 1, gc, gd, ga, grad2d);
      return;
    }
  }
  const int ntiles = nv * TX * TY;
  if (persist) {
    const auto k = k_render_bwd_w<TW, TH, B, BWD_TPW, true, 1>;
    const int need = (ntiles + BWD_TPW - 1) / BWD_TPW;
    const int grid = std::min(need, resident_blocks((const void*)k, 64 * BWD_TPW));
    hipLaunchKernelGGL(k, dim3(std::max(1, grid)), dim3(64 * BWD_TPW), 0, s, ntiles, W, H, TX, TY,
                       mask, cam, st, sched + 1, gc, gd, ga, grad2d);
  } else {
    hipLaunchKernelGGL((k_render_bwd_w<TW, TH, B, BWD_TPW, false, 1>),
                       dim3(xcd_grid((ntiles + BWD_TPW - 1) / BWD_TPW)), dim3(64 * BWD_TPW), 0, s,
                       ntiles, W, H, TX, TY, mask, cam, st, sched + 1, gc, gd, ga, grad2d);
  }
}

template <int TW, int TH>
static hipError_t bwd_t(int nv, int W, int H, int TX, int TY, const RenderCfg& rc,
                        unsigned long long mask, const CamDev& cam, StateDev st,
                        unsigned int* sched, const float* gc, const float* gd, const float* ga,
                        float* grad2d, hipStream_t s) {
  if (rc.bwd_batch == 1)
    bwd_b<TW, TH, 64>(nv, W, H, TX, TY, rc.persistent, rc.bwd_cols, mask, cam, st, sched, gc, gd,
                      ga, grad2d, s);
  else if (rc.bwd_batch == 4)
    bwd_b<TW, TH, 256>(nv, W, H, TX, TY, rc.persistent, rc.bwd_cols, mask, cam, st, sched, gc, gd,
                       ga, grad2d, s);
  else
    bwd_b<TW, TH, 128>(nv, W, H, TX, TY, rc.persistent, rc.bwd_cols, mask, cam, st, sched, gc, gd,
                       ga, grad2d, s);
  return hipGetLastError();
}

#define GSR_TILE_SWITCH(F, ...)                                         \
  do {                                                                  \
    if (TW == 16 && TH == 16) return F<16, 16>(__VA_ARGS__);            \
    else if (TW == 8 && TH == 8) return F<8, 8>(__VA_ARGS__);           \
    else if (TW == 16 && TH == 8) return F<16, 8>(__VA_ARGS__);         \
    else if (TW == 8 && TH == 16) return F<8, 16>(__VA_ARGS__);         \
    else if (TW == 32 && TH == 8) return F<32, 8>(__VA_ARGS__);         \
    else if (TW == 32 && TH == 16) return F<32, 16>(__VA_ARGS__);       \
    else if (TW == 16 && TH == 32) return F<16, 32>(__VA_ARGS__);       \
    else return hipErrorInvalidValue;                                   \
  } while (0)

hipError_t launch_render_fwd(int nv, int W, int H, int TW, int TH, int TX, int TY,
                             const RenderCfg& rc, const CamDev& cam, StateDev st,
                             unsigned int* sched, float* color, float* depth, float* alpha,
                             int32_t* n_eval, hipStream_t s) {
  GSR_TILE_SWITCH(fwd_t, nv, W, H, TX, TY, rc, cam, st, sched, color, depth, alpha, n_eval, s);
}

hipError_t launch_render_bwd(int nv, int W, int H, int TW, int TH, int TX, int TY,
                             const RenderCfg& rc, unsigned long long grad_mask,
                             const CamDev& cam, StateDev st, unsigned int* sched,
                             const float* g_color, const float* g_depth, const float* g_alpha,
                             float* grad2d, hipStream_t s) {
  GSR_TILE_SWITCH(bwd_t, nv, W, H, TX, TY, rc, grad_mask, cam, st, sched, g_color, g_depth,
                  g_alpha, grad2d, s);
}

// ------------------------------------------------------ debug kernels
// The per-tile lists, filtered from the row lists (set-up and tests only):
// one wave per tile scans its row list; WRITE = false counts the entries
// covering the tile's column, WRITE = true writes their visible positions in
// order at the tile's offset.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_tile_lists(int ntiles, int TX, int TY, StateDev st,
                                                    uint32_t* tile_cnt, const uint2* ranges,
                                                    uint32_t* inst) {
  const int g = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (g >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const int T = TX * TY, v = g / T, tl = g - v * T, ty = tl / TX;
  const uint32_t tx = (uint32_t)(tl - ty * TX);
  uint2 rr = st.row_rg[(size_t)v * TY + ty];
  if (st.hdr->overflow) rr = make_uint2(0u, 0u);
  uint32_t c = WRITE ? ranges[g].x : 0u;
  for (uint32_t q = rr.x; q < rr.y; q += 64u) {
    const uint32_t i = q + (uint32_t)lane;
    const uint2 e = i < rr.y ? st.rows[i] : make_uint2(0u, 0u);
    const bool cov = covers(e.y, tx);
    const unsigned long long m = __ballot(cov);
    if (WRITE && cov)
      inst[c + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = e.x;
    c += (uint32_t)__popcll(m);
  }
  if (!WRITE && lane == 0) tile_cnt[g] = c;
}

hipError_t launch_tile_lists(int nv, int TX, int TY, StateDev st, uint32_t* tile_cnt,
                             const uint2* ranges, uint32_t* inst, hipStream_t s) {
  const int ntiles = nv * TX * TY;
  if (ntiles > 0) {
    if (inst)
      hipLaunchKernelGGL(k_tile_lists<true>, dim3((ntiles + 3) / 4), dim3(256), 0, s, ntiles, TX,
                         TY, st, tile_cnt, ranges, inst);
    else
      hipLaunchKernelGGL(k_tile_lists<false>, dim3((ntiles + 3) / 4), dim3(256), 0, s, ntiles,
                         TX, TY, st, tile_cnt, ranges, inst);
  }
  return hipGetLastError();
}

// Entries blended per pixel (alpha >= 1/255 and before the stop): the
// non-skipped entries before the pixel's last contributor, with the
// forward's own skip arithmetic.  One workgroup per tile, one thread per
// pixel, the tile's list from k_tile_lists (set-up and tests only).
__global__ __launch_bounds__(512) void k_count_blend(int ntiles, int W, int H, int TW, int TX,
                                                     int TY, StateDev st, const uint2* ranges,
                                                     const uint32_t* inst, int32_t* n_blend) {
  const int g = blockIdx.x;
  if (g >= ntiles) return;
  const int T = TX * TY, v = g / T, tl = g - v * T;
  const int ty = tl / TX, tx = tl - ty * TX;
  const int px = tx * TW + (int)threadIdx.x % TW, py = ty * (int)(blockDim.x / TW) +
                                                        (int)threadIdx.x / TW;
  if (px >= W || py >= H) return;
  const size_t HW = (size_t)W * H, q = v * HW + (size_t)py * W + px;
  const uint2 rg = ranges[g];
  const uint32_t last = st.hdr->overflow ? 0u : min(st.last[q], rg.y - rg.x);
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  int cnt = 0;
  for (uint32_t i = 0; i < last; ++i) {
    const float4* r = st.rec + 3 * (size_t)inst[rg.x + i];
    const float4 a = r[0], b = r[1];
    const float p = splat_power(a, b, fx, fy);
    const float al = fminf(ALPHA_MAX, b.y * exp2_fast(p));
    cnt += (p > 0.f || al < ALPHA_MIN) ? 0 : 1;
  }
  n_blend[q] = cnt;
}

hipError_t launch_count_blend(int nv, int W, int H, int TW, int TH, int TX, int TY, StateDev st,
                              const uint2* ranges, const uint32_t* inst, int32_t* n_blend,
                              hipStream_t s) {
  const int ntiles = nv * TX * TY;
  if (ntiles > 0)
    hipLaunchKernelGGL(k_count_blend, dim3(ntiles), dim3(TW * TH), 0, s, ntiles, W, H, TW, TX, TY,
                       st, ranges, inst, n_blend);
  return hipGetLastError();
}

hipError_t launch_zero_pose(float* d_pose, int nv, unsigned int* bwd_next, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_pose, dim3(1), dim3(256), 0, s, d_pose, nv, bwd_next);
  return hipGetLastError();
}

}  // namespace gsr
