// Internal declarations shared by the HIP translation units of libgsr.
// Host code builds small per-kernel tables of the call's structure (which
// view renders which Gaussian set, block offsets); they travel as kernel
// arguments so a launch needs no host-to-device copy and can be captured.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsr.h"

namespace gsr {

constexpr int MAXV = GSR_MAX_VIEWS;
constexpr int MAXS = GSR_MAX_SETS;

constexpr int PROJ_BLOCK = 256;   // pairs per projection / compaction block
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;  // keys per radix-sort block
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int GRAD2D = 10;        // u, v, A, B, C, sigma, r, g, b, z
constexpr uint32_t CULLED = 0xFFFFFFFFu;
constexpr int MAX_ROWS = 512;     // tile rows per view (binning LDS arrays)
constexpr int MAX_COLS = 512;     // tile columns per view
constexpr int MAX_CHUNK = 256;   // depth-sorted pairs per row-binning chunk
constexpr int RC_SUB = 4;        // row-binning chunks per counting workgroup
constexpr int SCHED_WORDS = 2 + 2 * 33;  // tile cursors + length-bucket counts (render.hip)
constexpr int GSR_MAX_DEVICES = 64;  // devices with a looked-up library-held buffer
constexpr long SEED_NOALLOC_MAX_POINTS = GSR_SEED_NOALLOC_MAX_POINTS;

// Pair p of view v is Gaussian (set_goff[view_set[v]] + p - pair_off[v]).
struct ProjTab {
  int nv;
  int P;                      // total pairs of the call
  int W, H, TW, TH, TX, TY;
  int pair_off[MAXV + 1];
  int blk_off[MAXV + 1];      // PROJ_BLOCK-pair blocks per view, prefix
  int g_off[MAXV];            // first global Gaussian of the view's set
  int ns;                     // sets
  int set_goff[MAXS + 1];     // Gaussian offsets of the sets
  int set_gblk[MAXS + 1];     // PROJ_BLOCK-Gaussian blocks of the rendered sets, prefix
  int set_voff[MAXS + 1];     // views of each set in vset
  int vset[MAXV];             // view ids grouped by set (every view)
};

struct SortTab {
  int nv;
  int sblk_off[MAXV + 1];     // SORT_TILE blocks per view, prefix (upper bound)
};

struct BinTab {
  int nv;
  int chunk;                  // pairs per chunk
  int TX, TY, T;              // tiles per view = T
  int cblk_off[MAXV + 1];     // chunks per view, prefix (upper bound)
};

struct SetTab {
  int ns;
  int set_goff[MAXS + 1];     // Gaussian offsets of the sets
  int set_blk[MAXS + 1];      // PROJ_BLOCK-Gaussian blocks per set, prefix
  int set_voff[MAXS + 1];     // views of each set in view_by_set
  int view_by_set[MAXV];      // view ids grouped by set (grad-needing only)
  int pair_off[MAXV + 1];
  int W, H;
};

struct SceneDev {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* opac;
  const float* colors;
  int sh_degree;
  int sh_stride;
};

struct CamDev {
  const float* viewmats;    // [V,12]
  const float* intrinsics;  // [V,4]
  float z_near;
  float bg0, bg1, bg2;
};

// Device header at the start of every saved-state buffer.
struct StateHeader {
  unsigned long long inst_total;  // (pair, tile) copies of the rects (reported only)
  unsigned int overflow;          // the row entries exceeded the capacity
  unsigned int vis_total;
  unsigned long long row_total;   // (pair, tile row) entries of the binning
  unsigned int vis_off[MAXV + 1]; // visible-pair offsets per view (compacted order)
};
constexpr size_t STATE_HEADER_BYTES = 512;
static_assert(sizeof(StateHeader) <= STATE_HEADER_BYTES, "header");

// Byte offsets of the arrays inside a saved-state buffer (all 256-aligned).
struct StateLayout {
  size_t hdr, zkey, vidx, rect, rec, order, row_rg, rows, torder, tfinal, last, total;
};

// Pointers into a saved-state buffer.
struct StateDev {
  StateHeader* hdr;
  uint32_t* zkey;     // [P]
  uint32_t* vidx;     // [P] position in the compacted visible list, CULLED if culled
  uint2* rect;        // [Pv] by visible position: packed (x0 | y0 << 16, x1 | y1 << 16)
  float4* rec;        // [Pv][3] by visible position: (u, v, A', B'), (C', sigma, z, ex),
                      //   (r, g, b, ey)
  uint32_t* order;    // [Pv] visible positions in (view, depth, id) order
  uint2* row_rg;      // [V*TY] range of each (view, tile row) list in rows
  uint2* rows;        // [cap] row lists: (visible position, x0 | x1 << 16) in
                      //   (depth, id) order
  uint32_t* torder;   // [V*T] tiles by decreasing row-list length (persistent render)
  float* tfinal;      // [V*H*W]
  uint32_t* last;     // [V*H*W]
  unsigned long long cap;
};

// Binning workspace (context-owned).
struct BinWork {
  uint32_t* counts;     // [chunks][TY] per-chunk row counts -> exclusive bases
  uint32_t* row_tot;    // [V*TY] entries per (view, row)
  uint32_t* area_part;  // [chunks / RC_SUB + 1] (pair, tile) copies per counting workgroup
};

// Sim(3) corrections: Gaussian set offsets, and the set of every view.
struct SimSetTab {
  int ns;
  long long off[MAXS + 1];
};
struct SimViewTab {
  int nv;
  int view_set[MAXV];
};

StateLayout state_layout(const gsr_plan_desc& p);
StateDev state_ptrs(void* base, const gsr_plan_desc& p);

// ------------------------------------------------------------------ launches
hipError_t launch_project_keys(const ProjTab& t, const SceneDev& sc, const CamDev& cam,
                               StateDev st, uint32_t* blk_cnt, hipStream_t s);
hipError_t launch_project_records(const ProjTab& t, const SceneDev& sc, const CamDev& cam,
                                  StateDev st, hipStream_t s);
hipError_t launch_compact(const ProjTab& t, StateDev st, const uint32_t* blk_cnt,
                          uint32_t* blk_scan, uint32_t* kout, hipStream_t s);
hipError_t launch_depth_sort(const SortTab& t, StateDev st, uint32_t* ka, uint32_t* va,
                             uint32_t* kb, uint32_t* vb, uint32_t* hist, uint32_t* off,
                             hipStream_t s);
hipError_t launch_binning(const BinTab& t, StateDev st, const BinWork& w, hipStream_t s);
// Compositing launch options (from the plan): list entries staged per lane
// in the forward (1 or 2) and in the backward (1, 2 or 4), tiles of a tile
// row per backward wave (1 or 2), and the persistent length-ordered tile
// queue instead of one wave per tile.
struct RenderCfg {
  int fwd_batch;
  int bwd_batch;
  int bwd_cols;
  bool persistent;
};
hipError_t launch_tile_order(int nv, int TX, int TY, StateDev st, unsigned int* sched,
                             hipStream_t s);
hipError_t launch_render_fwd(int nv, int W, int H, int TW, int TH, int TX, int TY,
                             const RenderCfg& rc, const CamDev& cam, StateDev st,
                             unsigned int* sched, float* color, float* depth, float* alpha,
                             int32_t* n_eval, hipStream_t s);
hipError_t launch_render_bwd(int nv, int W, int H, int TW, int TH, int TX, int TY,
                             const RenderCfg& rc, unsigned long long grad_mask,
                             const CamDev& cam, StateDev st, unsigned int* sched,
                             const float* g_color, const float* g_depth, const float* g_alpha,
                             float* grad2d, hipStream_t s);
// Debug only: the per-tile lists filtered from the row lists, first as
// counts per tile (tile_cnt [V*T]), then written at the tiles' offsets
// (ranges [V*T], from the counts' exclusive scan) into inst.
hipError_t launch_tile_lists(int nv, int TX, int TY, StateDev st, uint32_t* tile_cnt,
                             const uint2* ranges, uint32_t* inst, hipStream_t s);
hipError_t launch_count_blend(int nv, int W, int H, int TW, int TH, int TX, int TY, StateDev st,
                              const uint2* ranges, const uint32_t* inst, int32_t* n_blend,
                              hipStream_t s);
hipError_t launch_zero_pose(float* d_pose, int nv, unsigned int* bwd_next, hipStream_t s);
hipError_t launch_project_bwd(const SetTab& t, const SceneDev& sc, const CamDev& cam,
                              StateDev st, float* grad2d, const gsr_grads& g,
                              int n_total, hipStream_t s);
hipError_t launch_pose_delta(const float* vin, const float* delta, float* vout, int nv,
                             hipStream_t s);
hipError_t launch_sim3_gaussians(const SimSetTab& tab, const float* m_in, const float* ls_in,
                                 const float* q_in, const float* sims, float* m_out,
                                 float* ls_out, float* q_out, hipStream_t s);
hipError_t launch_sim3_views(const SimViewTab& tab, const float* vin, const float* sims,
                             float* vout, hipStream_t s);
hipError_t launch_l1_grad(int nv, int HW, const float* color, const float* depth,
                          const float* tcol, const float* tdep, const float* expo, float w_col,
                          float w_dep, float* g_col, float* g_dep, float* g_expo, hipStream_t s);
size_t dedup_workspace_bytes(long long slots);
hipError_t launch_dedup(long long slots, void* ws, double v, double kenv, const float* tm,
                        const float* tls, long long n_tgt, const float* depth, const float* vms,
                        const float* intr, int nk, int W, int H, const float* sm, long long n_src,
                        uint8_t* keep, hipStream_t s, unsigned int** counters);
size_t ssim_workspace_bytes(int nv, int W, int H);
hipError_t launch_ssim(int nv, int W, int H, float weight, const float* color,
                       const float* target, const float* expo, void* ws, float* d_color,
                       float* d_expo, float* ssim_out, hipStream_t s);
hipError_t launch_prune(long n, const SceneDev& in, int color_stride, float thr,
                        const SimSetTab& sets, uint32_t* blk, long long* bounds, float* m,
                        float* ls, float* q, float* o, float* col, hipStream_t s);
// exclusive scan of nb block counts in place, total at blk[nb] (one workgroup)
hipError_t launch_block_scan(int nb, uint32_t* blk, hipStream_t s);
hipError_t launch_iso_grad(long n, const float* ls, float w, float* g, hipStream_t s);
hipError_t launch_normal_grad(int nv, int W, int H, const float* depth, const float* prior,
                              const float* intr, float w, float* g_dep, hipStream_t s);
hipError_t launch_seed(int W, int H, int stride, const float* depth, const float* color,
                       const float* vm, const float* intr, float opac_logit, long max_out,
                       uint32_t* blk, float* m, float* ls, float* q, float* o, float* c,
                       hipStream_t s);
hipError_t launch_adam(const gsr_adam_group* gr, int ng, double b1, double b2, double eps,
                       int32_t* step, hipStream_t s);
hipError_t seed_scratch(uint32_t** out);
hipError_t launch_seed_total(const uint32_t* blk, int nb, int64_t* n_out, hipStream_t s);

}  // namespace gsr
