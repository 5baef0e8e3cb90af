// The C ABI: context, planning, argument checking and the launch sequences
// of the forward and backward passes.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace gsr;

struct gsr_ctx {
  int device = 0;
  std::string err;
  bool planned = false;
  gsr_plan_desc plan{};
  int chunk = 0;
  int TX = 0, TY = 0, T = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t* blk_cnt = nullptr;   // visible pairs per projection block
  uint32_t* blk_scan = nullptr;  // their exclusive prefix
  uint32_t *ka = nullptr, *va = nullptr, *kb = nullptr, *vb = nullptr;
  uint32_t* hist = nullptr;
  uint32_t* hoff = nullptr;
  BinWork bw{};
  float* grad2d = nullptr;
  unsigned int* sched = nullptr;  // tile cursors of the persistent compositing
  RenderCfg rc{1, 2, false};
  size_t max_blocks = 0, max_sblocks = 0, max_chunks = 0;
  bool prof = false;
  hipEvent_t ev[GSR_NUM_STAGES][2] = {};
  bool ev_used[GSR_NUM_STAGES] = {};
};

namespace {

gsr_status fail(gsr_ctx* c, gsr_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

gsr_status hip_fail(gsr_ctx* c, hipError_t e, const char* what) {
  return fail(c, GSR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

bool pow2_tile(int x) { return x == 8 || x == 16 || x == 32; }

int auto_chunk(const gsr_plan_desc& p) {
  if (p.chunk > 0) return p.chunk;
  // 64..256 depth-sorted pairs per chunk: small batches (one view) need many
  // chunks to fill the GPU; large ones use longer per-tile runs per chunk.
  long c = 64;
  while (c < 256 && p.max_pairs / c > 65536) c *= 2;
  return (int)c;
}

// RAII guard that makes ctx->device current and restores the caller's.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

namespace gsr {

StateLayout state_layout(const gsr_plan_desc& p) {
  StateLayout L{};
  const int TX = (p.width + p.tile_w - 1) / p.tile_w, TY = (p.height + p.tile_h - 1) / p.tile_h;
  const size_t P = (size_t)p.max_pairs, V = (size_t)p.max_views;
  const size_t px = V * (size_t)p.width * (size_t)p.height;
  size_t o = 0;
  L.hdr = o; o = align256(o + STATE_HEADER_BYTES);
  L.zkey = o; o = align256(o + P * 4);
  L.vidx = o; o = align256(o + P * 4);
  L.rect = o; o = align256(o + P * 8);
  L.rec = o; o = align256(o + P * 48);
  L.order = o; o = align256(o + P * 4);
  L.row_rg = o; o = align256(o + V * (size_t)TY * 8);
  L.rows = o; o = align256(o + (size_t)p.max_instances * 8);
  L.torder = o; o = align256(o + V * (size_t)TX * TY * 4);
  L.tfinal = o; o = align256(o + px * 4);
  L.last = o; o = align256(o + px * 4);
  L.total = o;
  return L;
}

StateDev state_ptrs(void* base, const gsr_plan_desc& p) {
  const StateLayout L = state_layout(p);
  char* b = (char*)base;
  StateDev s;
  s.hdr = (StateHeader*)(b + L.hdr);
  s.zkey = (uint32_t*)(b + L.zkey);
  s.vidx = (uint32_t*)(b + L.vidx);
  s.rect = (uint2*)(b + L.rect);
  s.rec = (float4*)(b + L.rec);
  s.order = (uint32_t*)(b + L.order);
  s.row_rg = (uint2*)(b + L.row_rg);
  s.rows = (uint2*)(b + L.rows);
  s.torder = (uint32_t*)(b + L.torder);
  s.tfinal = (float*)(b + L.tfinal);
  s.last = (uint32_t*)(b + L.last);
  s.cap = (unsigned long long)p.max_instances;
  return s;
}

}  // namespace gsr

namespace {

gsr_status check_plan(gsr_ctx* c, const gsr_plan_desc* p) {
  if (!p) return fail(c, GSR_E_INVALID_ARG, "plan is NULL");
  if (p->max_pairs < 1 || p->max_pairs > 0x7FFFFFFFL)
    return fail(c, GSR_E_INVALID_ARG, "max_pairs must be in [1, 2^31-1]");
  if (p->max_instances < 1 || p->max_instances > 0xFFFFFFFEL)
    return fail(c, GSR_E_INVALID_ARG, "max_instances must be in [1, 2^32-2]");
  if (p->max_views < 1 || p->max_views > GSR_MAX_VIEWS)
    return fail(c, GSR_E_INVALID_ARG, "max_views must be in [1, %d]", GSR_MAX_VIEWS);
  if (p->width < 1 || p->height < 1 || p->width > 16384 || p->height > 16384)
    return fail(c, GSR_E_INVALID_ARG, "image size must be in [1, 16384]");
  if (!pow2_tile(p->tile_w) || !pow2_tile(p->tile_h) || p->tile_w * p->tile_h < 64 ||
      p->tile_w * p->tile_h > 512 || (p->tile_w == 32 && p->tile_h == 32) ||
      (p->tile_w == 8 && p->tile_h == 32))
    return fail(c, GSR_E_INVALID_ARG,
                "tile shape must be one of 8x8, 16x8, 8x16, 16x16, 32x8, 32x16, 16x32");
  const long TX = (p->width + p->tile_w - 1) / p->tile_w, TY = (p->height + p->tile_h - 1) / p->tile_h;
  if (TX > MAX_COLS || TY > MAX_ROWS)
    return fail(c, GSR_E_INVALID_ARG, "too many tiles per view (%ld x %ld, at most %d x %d)", TX,
                TY, MAX_COLS, MAX_ROWS);
  if (p->chunk < 0 || p->chunk > MAX_CHUNK)
    return fail(c, GSR_E_INVALID_ARG, "chunk must be in [0, %d]", MAX_CHUNK);
  if (p->fwd_batch < 0 || p->fwd_batch > 2)
    return fail(c, GSR_E_INVALID_ARG, "fwd_batch must be 0, 1 or 2");
  if (!(p->bwd_batch == 0 || p->bwd_batch == 1 || p->bwd_batch == 2 || p->bwd_batch == 4))
    return fail(c, GSR_E_INVALID_ARG, "bwd_batch must be 0, 1, 2 or 4");
  if (!(p->bwd_cols == 0 || p->bwd_cols == 1 || p->bwd_cols == 2))
    return fail(c, GSR_E_INVALID_ARG, "bwd_cols must be 0, 1 or 2");
  if (p->bwd_cols == 2 && (p->tile_w > 16 || 2 * p->tile_w * p->tile_h > 512))
    return fail(c, GSR_E_INVALID_ARG, "bwd_cols 2 needs tile_w <= 16 and 2 tile_w tile_h <= 512");
  if (p->persistent != 0 && p->persistent != 1)
    return fail(c, GSR_E_INVALID_ARG, "persistent must be 0 or 1");
  return GSR_OK;
}

struct CallTabs {
  ProjTab pt;
  SortTab stb;
  BinTab bt;
  SetTab set;
  int P = 0;
  unsigned long long grad_mask = 0;
};

gsr_status build_tabs(gsr_ctx* c, const gsr_scene* sc, const gsr_views* vw, CallTabs& t) {
  if (!sc || !vw) return fail(c, GSR_E_INVALID_ARG, "scene/views is NULL");
  if (!sc->means || !sc->log_scales || !sc->quats || !sc->opacity_logits || !sc->colors ||
      !sc->set_offsets)
    return fail(c, GSR_E_INVALID_ARG, "scene array is NULL");
  if (sc->n_sets < 1 || sc->n_sets > GSR_MAX_SETS)
    return fail(c, GSR_E_INVALID_ARG, "n_sets must be in [1, %d]", GSR_MAX_SETS);
  if (sc->sh_degree < 0 || sc->sh_degree > 3)
    return fail(c, GSR_E_INVALID_ARG, "sh_degree must be 0..3");
  if (sc->sh_degree > 0 && sc->sh_stride < (sc->sh_degree + 1) * (sc->sh_degree + 1))
    return fail(c, GSR_E_INVALID_ARG, "sh_stride too small for sh_degree");
  if (!vw->viewmats || !vw->intrinsics || !vw->view_set)
    return fail(c, GSR_E_INVALID_ARG, "views array is NULL");
  const gsr_plan_desc& p = c->plan;
  if (vw->n_views < 1 || vw->n_views > p.max_views)
    return fail(c, GSR_E_CAPACITY, "n_views %d outside [1, %d]", vw->n_views, p.max_views);
  if (vw->width != p.width || vw->height != p.height)
    return fail(c, GSR_E_INVALID_ARG, "image size %dx%d differs from the plan's %dx%d", vw->width,
                vw->height, p.width, p.height);
  if (sc->set_offsets[0] != 0) return fail(c, GSR_E_INVALID_ARG, "set_offsets[0] must be 0");
  for (int s = 0; s < sc->n_sets; ++s)
    if (sc->set_offsets[s + 1] < sc->set_offsets[s])
      return fail(c, GSR_E_INVALID_ARG, "set_offsets must be non-decreasing");
  if (sc->set_offsets[sc->n_sets] > 0x7FFFFFFFL)
    return fail(c, GSR_E_INVALID_ARG, "too many Gaussians");
  const int nv = vw->n_views;
  memset(&t.pt, 0, sizeof t.pt);
  memset(&t.stb, 0, sizeof t.stb);
  memset(&t.bt, 0, sizeof t.bt);
  memset(&t.set, 0, sizeof t.set);
  long P = 0;
  t.pt.nv = nv;
  t.pt.W = p.width; t.pt.H = p.height; t.pt.TW = p.tile_w; t.pt.TH = p.tile_h;
  t.pt.TX = c->TX; t.pt.TY = c->TY;
  t.stb.nv = nv;
  t.bt.nv = nv; t.bt.chunk = c->chunk; t.bt.TX = c->TX; t.bt.TY = c->TY; t.bt.T = c->T;
  int blk = 0, sblk = 0, cblk = 0;
  t.grad_mask = 0;
  for (int v = 0; v < nv; ++v) {
    const int s = vw->view_set[v];
    if (s < 0 || s >= sc->n_sets) return fail(c, GSR_E_INVALID_ARG, "view_set[%d] = %d out of range", v, s);
    const long n = sc->set_offsets[s + 1] - sc->set_offsets[s];
    t.pt.pair_off[v] = (int)P;
    t.pt.blk_off[v] = blk;
    t.pt.g_off[v] = (int)sc->set_offsets[s];
    t.stb.sblk_off[v] = sblk;
    t.bt.cblk_off[v] = cblk;
    P += n;
    if (P > p.max_pairs)
      return fail(c, GSR_E_CAPACITY, "pairs exceed plan max_pairs %lld", (long long)p.max_pairs);
    blk += ceil_div(n, PROJ_BLOCK);
    sblk += ceil_div(n, SORT_TILE);
    cblk += ceil_div(n, c->chunk);
    if (!vw->needs_grad || vw->needs_grad[v]) t.grad_mask |= 1ull << v;
  }
  t.pt.pair_off[nv] = (int)P;
  t.pt.blk_off[nv] = blk;
  t.stb.sblk_off[nv] = sblk;
  t.bt.cblk_off[nv] = cblk;
  t.pt.P = (int)P;
  t.P = (int)P;
  if ((size_t)blk > c->max_blocks || (size_t)sblk > c->max_sblocks || (size_t)cblk > c->max_chunks)
    return fail(c, GSR_E_CAPACITY, "block tables exceed the plan");
  // sets, for the projection: every view, blocks only for rendered sets
  {
    ProjTab& pt = t.pt;
    pt.ns = sc->n_sets;
    int gb = 0, nvs = 0;
    for (int s = 0; s < sc->n_sets; ++s) {
      pt.set_goff[s] = (int)sc->set_offsets[s];
      pt.set_gblk[s] = gb;
      pt.set_voff[s] = nvs;
      for (int v = 0; v < nv; ++v)
        if (vw->view_set[v] == s) pt.vset[nvs++] = v;
      if (nvs > pt.set_voff[s])
        gb += ceil_div(sc->set_offsets[s + 1] - sc->set_offsets[s], PROJ_BLOCK);
    }
    pt.set_goff[sc->n_sets] = (int)sc->set_offsets[sc->n_sets];
    pt.set_gblk[sc->n_sets] = gb;
    pt.set_voff[sc->n_sets] = nvs;
  }
  // sets, for the projection backward
  SetTab& st = t.set;
  st.ns = sc->n_sets;
  st.W = p.width; st.H = p.height;
  int sb = 0, nvs = 0;
  for (int s = 0; s < sc->n_sets; ++s) {
    st.set_goff[s] = (int)sc->set_offsets[s];
    st.set_blk[s] = sb;
    sb += ceil_div(sc->set_offsets[s + 1] - sc->set_offsets[s], PROJ_BLOCK);
    st.set_voff[s] = nvs;
    for (int v = 0; v < nv; ++v)
      if (vw->view_set[v] == s && ((t.grad_mask >> v) & 1ull)) st.view_by_set[nvs++] = v;
  }
  st.set_goff[sc->n_sets] = (int)sc->set_offsets[sc->n_sets];
  st.set_blk[sc->n_sets] = sb;
  st.set_voff[sc->n_sets] = nvs;
  for (int v = 0; v <= nv; ++v) st.pair_off[v] = t.pt.pair_off[v];
  return GSR_OK;
}

SceneDev scene_dev(const gsr_scene* sc) {
  SceneDev d;
  d.means = sc->means;
  d.log_scales = sc->log_scales;
  d.quats = sc->quats;
  d.opac = sc->opacity_logits;
  d.colors = sc->colors;
  d.sh_degree = sc->sh_degree;
  d.sh_stride = sc->sh_degree > 0 ? sc->sh_stride : 1;
  return d;
}

CamDev cam_dev(const gsr_views* vw, const gsr_settings* s) {
  CamDev c;
  c.viewmats = vw->viewmats;
  c.intrinsics = vw->intrinsics;
  c.z_near = s ? s->z_near : 0.2f;
  c.bg0 = s ? s->bg[0] : 0.f;
  c.bg1 = s ? s->bg[1] : 0.f;
  c.bg2 = s ? s->bg[2] : 0.f;
  return c;
}

// Records a stage's start/stop event when profiling is on and the stream is
// not being captured.
struct StageMark {
  gsr_ctx* c;
  int id;
  hipStream_t s;
  bool on;
  StageMark(gsr_ctx* c_, int id_, hipStream_t s_) : c(c_), id(id_), s(s_), on(false) {
    if (!c->prof) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    on = hipEventRecord(c->ev[id][0], s) == hipSuccess;
  }
  ~StageMark() {
    if (on && hipEventRecord(c->ev[id][1], s) == hipSuccess) c->ev_used[id] = true;
  }
};

void free_ws(gsr_ctx* c) {
  if (c->ws) (void)hipFree(c->ws);
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->planned = false;
}

}  // namespace

extern "C" {

const char* gsr_status_string(gsr_status s) {
  switch (s) {
    case GSR_OK: return "ok";
    case GSR_E_INVALID_ARG: return "invalid argument";
    case GSR_E_NOT_PLANNED: return "not planned";
    case GSR_E_CAPACITY: return "capacity exceeded";
    case GSR_E_OVERFLOW: return "instance overflow";
    case GSR_E_DEVICE: return "device error";
    case GSR_E_OOM: return "out of device memory";
    case GSR_E_UNIMPLEMENTED: return "unimplemented";
  }
  return "unknown status";
}

const char* gsr_last_error(const gsr_ctx* c) { return c ? c->err.c_str() : "no context"; }

gsr_status gsr_create(gsr_ctx** out, int device) {
  if (!out) return GSR_E_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return GSR_E_DEVICE;
  }
  if (device < 0 || device >= n) return GSR_E_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return GSR_E_DEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return GSR_E_DEVICE;
  gsr_ctx* c = new (std::nothrow) gsr_ctx();
  if (!c) return GSR_E_OOM;
  c->device = device;
  *out = c;
  return GSR_OK;
}

void gsr_destroy(gsr_ctx* c) {
  if (!c) return;
  {
    DeviceGuard g(c->device);
    free_ws(c);
    for (int i = 0; i < GSR_NUM_STAGES; ++i)
      for (int j = 0; j < 2; ++j)
        if (c->ev[i][j]) (void)hipEventDestroy(c->ev[i][j]);
  }
  delete c;
}

gsr_status gsr_state_bytes(const gsr_plan_desc* p, size_t* out) {
  if (!out) return GSR_E_INVALID_ARG;
  gsr_status s = check_plan(nullptr, p);
  if (s != GSR_OK) return s;
  *out = state_layout(*p).total;
  return GSR_OK;
}

gsr_status gsr_plan(gsr_ctx* c, const gsr_plan_desc* p) {
  if (!c) return GSR_E_INVALID_ARG;
  gsr_status s = check_plan(c, p);
  if (s != GSR_OK) return s;
  DeviceGuard g(c->device);
  free_ws(c);
  c->plan = *p;
  c->chunk = auto_chunk(*p);
  c->TX = (p->width + p->tile_w - 1) / p->tile_w;
  c->TY = (p->height + p->tile_h - 1) / p->tile_h;
  c->T = c->TX * c->TY;
  const size_t P = (size_t)p->max_pairs, V = (size_t)p->max_views;
  c->max_blocks = P / PROJ_BLOCK + V + 1;
  c->max_sblocks = P / SORT_TILE + V + 1;
  c->max_chunks = P / (size_t)c->chunk + V + 1;
  size_t o = 0;
  const size_t o_blk = o; o = align256(o + c->max_blocks * 4);
  const size_t o_bsc = o; o = align256(o + c->max_blocks * 4);
  const size_t o_ka = o; o = align256(o + P * 4);
  const size_t o_va = o; o = align256(o + P * 4);
  const size_t o_kb = o; o = align256(o + P * 4);
  const size_t o_vb = o; o = align256(o + P * 4);
  const size_t o_hist = o; o = align256(o + c->max_sblocks * RADIX * 4);
  const size_t o_hoff = o; o = align256(o + c->max_sblocks * RADIX * 4);
  const size_t o_cnt = o; o = align256(o + c->max_chunks * (size_t)c->TY * 4);
  const size_t o_rt = o; o = align256(o + V * (size_t)c->TY * 4);
  const size_t o_ap = o; o = align256(o + (c->max_chunks / RC_SUB + 1) * 4);
  const size_t o_g2 = o; o = align256(o + P * GRAD2D * 4);
  const size_t o_sch = o; o = align256(o + SCHED_WORDS * 4);
  void* ws = nullptr;
  hipError_t e = hipMalloc(&ws, o);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, GSR_E_OOM, "workspace of %zu bytes: %s", o, hipGetErrorString(e));
  }
  char* b = (char*)ws;
  c->ws = ws;
  c->ws_bytes = o;
  c->blk_cnt = (uint32_t*)(b + o_blk);
  c->blk_scan = (uint32_t*)(b + o_bsc);
  c->ka = (uint32_t*)(b + o_ka);
  c->va = (uint32_t*)(b + o_va);
  c->kb = (uint32_t*)(b + o_kb);
  c->vb = (uint32_t*)(b + o_vb);
  c->hist = (uint32_t*)(b + o_hist);
  c->hoff = (uint32_t*)(b + o_hoff);
  c->bw.counts = (uint32_t*)(b + o_cnt);
  c->bw.row_tot = (uint32_t*)(b + o_rt);
  c->bw.area_part = (uint32_t*)(b + o_ap);
  c->grad2d = (float*)(b + o_g2);
  c->sched = (unsigned int*)(b + o_sch);
  c->rc.fwd_batch = p->fwd_batch == 2 ? 2 : 1;
  c->rc.bwd_batch = p->bwd_batch == 0 ? 1 : p->bwd_batch;
  c->rc.persistent = p->persistent == 1;
  c->rc.bwd_cols = p->bwd_cols == 2 ? 2 : 1;
  // The per-pair screen-space gradient rows start at zero and every
  // backward leaves them at zero (the projection backward clears what it
  // reads), so no clearing pass is needed per call.
  e = hipMemset(c->grad2d, 0, P * GRAD2D * 4);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_ws(c);
    return hip_fail(c, e, "workspace clear");
  }
  c->planned = true;
  return GSR_OK;
}

gsr_status gsr_forward(gsr_ctx* c, const gsr_scene* sc, const gsr_views* vw,
                       const gsr_settings* set, void* state, const gsr_images* out,
                       void* stream) {
  if (!c) return GSR_E_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_E_NOT_PLANNED, "gsr_plan first");
  if (!state || ((uintptr_t)state & 255)) return fail(c, GSR_E_INVALID_ARG, "state must be non-NULL and 256-byte aligned");
  if (!out || !out->color || !out->depth || !out->alpha)
    return fail(c, GSR_E_INVALID_ARG, "output image is NULL");
  CallTabs t;
  gsr_status s = build_tabs(c, sc, vw, t);
  if (s != GSR_OK) return s;
  DeviceGuard g(c->device);
  hipStream_t st = (hipStream_t)stream;
  StateDev sd = state_ptrs(state, c->plan);
  const SceneDev scd = scene_dev(sc);
  const CamDev cam = cam_dev(vw, set);
  hipError_t e;
  {
    StageMark m(c, GSR_STAGE_PROJECT, st);
    if ((e = launch_project_keys(t.pt, scd, cam, sd, c->blk_cnt, st)) != hipSuccess)
      return hip_fail(c, e, "project");
  }
  {
    StageMark m(c, GSR_STAGE_COMPACT, st);
    if ((e = launch_compact(t.pt, sd, c->blk_cnt, c->blk_scan, c->ka, st)) != hipSuccess) return hip_fail(c, e, "compact");
  }
  {
    StageMark m(c, GSR_STAGE_RECORD, st);
    if ((e = launch_project_records(t.pt, scd, cam, sd, st)) != hipSuccess)
      return hip_fail(c, e, "records");
  }
  {
    StageMark m(c, GSR_STAGE_DEPTH_SORT, st);
    if ((e = launch_depth_sort(t.stb, sd, c->ka, c->va, c->kb, c->vb, c->hist, c->hoff, st)) != hipSuccess)
      return hip_fail(c, e, "depth sort");
  }
  {
    StageMark m(c, GSR_STAGE_BINNING, st);
    if ((e = launch_binning(t.bt, sd, c->bw, st)) != hipSuccess) return hip_fail(c, e, "binning");
  }
  {
    StageMark m(c, GSR_STAGE_RENDER_FWD, st);
    if (c->rc.persistent &&
        (e = launch_tile_order(vw->n_views, c->TX, c->TY, sd, c->sched, st)) != hipSuccess)
      return hip_fail(c, e, "tile order");
    if ((e = launch_render_fwd(vw->n_views, c->plan.width, c->plan.height, c->plan.tile_w,
                               c->plan.tile_h, c->TX, c->TY, c->rc, cam, sd, c->sched,
                               out->color, out->depth, out->alpha, out->n_eval, st)) != hipSuccess)
      return hip_fail(c, e, "render forward");
  }
  return GSR_OK;
}

gsr_status gsr_backward(gsr_ctx* c, const gsr_scene* sc, const gsr_views* vw,
                        const gsr_settings* set, const void* state, const gsr_grad_images* gin,
                        const gsr_grads* out, void* stream) {
  if (!c) return GSR_E_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_E_NOT_PLANNED, "gsr_plan first");
  if (!state || ((uintptr_t)state & 255)) return fail(c, GSR_E_INVALID_ARG, "state must be non-NULL and 256-byte aligned");
  if (!out || !out->d_means || !out->d_log_scales || !out->d_quats || !out->d_opacity_logits ||
      !out->d_colors || !out->d_pose)
    return fail(c, GSR_E_INVALID_ARG, "gradient output is NULL");
  CallTabs t;
  gsr_status s = build_tabs(c, sc, vw, t);
  if (s != GSR_OK) return s;
  DeviceGuard g(c->device);
  hipStream_t st = (hipStream_t)stream;
  StateDev sd = state_ptrs(const_cast<void*>(state), c->plan);
  const SceneDev scd = scene_dev(sc);
  const CamDev cam = cam_dev(vw, set);
  const float* gc = gin ? gin->color : nullptr;
  const float* gd = gin ? gin->depth : nullptr;
  const float* ga = gin ? gin->alpha : nullptr;
  hipError_t e;
  {
    StageMark m(c, GSR_STAGE_ZERO, st);
    if ((e = launch_zero_pose(out->d_pose, vw->n_views, c->sched + 1, st)) != hipSuccess)
      return hip_fail(c, e, "zero");
  }
  {
    StageMark m(c, GSR_STAGE_RENDER_BWD, st);
    if ((e = launch_render_bwd(vw->n_views, c->plan.width, c->plan.height, c->plan.tile_w,
                               c->plan.tile_h, c->TX, c->TY, c->rc, t.grad_mask, cam, sd,
                               c->sched, gc, gd, ga, c->grad2d, st)) != hipSuccess)
      return hip_fail(c, e, "render backward");
  }
  {
    StageMark m(c, GSR_STAGE_PROJECT_BWD, st);
    if ((e = launch_project_bwd(t.set, scd, cam, sd, c->grad2d, *out, t.P, st)) != hipSuccess)
      return hip_fail(c, e, "projection backward");
  }
  return GSR_OK;
}

gsr_status gsr_poll(gsr_ctx* c, const void* state, gsr_counts* out, void* stream) {
  if (!c || !state || !out) return GSR_E_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_E_NOT_PLANNED, "gsr_plan first");
  DeviceGuard g(c->device);
  StateHeader h;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e == hipSuccess) e = hipMemcpy(&h, state, sizeof h, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "poll");
  out->visible_pairs = h.vis_total;
  out->instances = (int64_t)h.inst_total;
  out->row_entries = (int64_t)h.row_total;
  out->capacity = c->plan.max_instances;
  out->overflow = (int32_t)h.overflow;
  out->n_views = 0;
  if (h.overflow)
    return fail(c, GSR_E_OVERFLOW, "forward needed %llu (pair, tile row) entries, plan holds %lld",
                (unsigned long long)h.row_total, (long long)c->plan.max_instances);
  return GSR_OK;
}

gsr_status gsr_debug_export(gsr_ctx* c, const void* state, int32_t n_views, gsr_debug* d,
                            void* stream) {
  if (!c || !state || !d) return GSR_E_INVALID_ARG;
  if (!c->planned) return fail(c, GSR_E_NOT_PLANNED, "gsr_plan first");
  if (n_views < 1 || n_views > c->plan.max_views) return fail(c, GSR_E_INVALID_ARG, "n_views");
  DeviceGuard g(c->device);
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "debug sync");
  StateDev sd = state_ptrs(const_cast<void*>(state), c->plan);
  StateHeader h;
  if ((e = hipMemcpy(&h, sd.hdr, sizeof h, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(c, e, "debug hdr");
  const size_t np = (size_t)std::max<int64_t>(0, std::min<int64_t>(d->n_pairs, c->plan.max_pairs));
  const size_t px = (size_t)n_views * c->plan.width * c->plan.height;
  struct Cp { void* dst; const void* src; size_t bytes; };
  std::vector<Cp> cps;
  if (d->zkeys) cps.push_back({d->zkeys, sd.zkey, np * 4});
  if (d->order) cps.push_back({d->order, sd.order, std::min<size_t>(np, h.vis_total) * 4});
  // The tile lists are never stored by the forward: debug kernels filter
  // them from the row lists into temporary buffers (counts, host scan,
  // write), for the export and for the blend counter.
  size_t n_inst_out = 0;
  if (d->ranges || d->inst || d->n_blend) {
    const size_t nt = (size_t)n_views * c->T;
    hipStream_t hs = (hipStream_t)stream;
    uint32_t* tcnt = nullptr;
    uint2* trg = nullptr;
    uint32_t* tinst = nullptr;
    std::vector<uint32_t> cnt(nt);
    std::vector<uint2> rg(nt);
    size_t total = 0;
    auto release = [&]() {
      if (tcnt) (void)hipFree(tcnt);
      if (trg) (void)hipFree(trg);
      if (tinst) (void)hipFree(tinst);
    };
    e = hipMalloc(&tcnt, std::max<size_t>(nt, 1) * 4);
    if (e == hipSuccess) e = hipMalloc(&trg, std::max<size_t>(nt, 1) * 8);
    if (e == hipSuccess) e = launch_tile_lists(n_views, c->TX, c->TY, sd, tcnt, nullptr, nullptr, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e == hipSuccess) e = hipMemcpy(cnt.data(), tcnt, nt * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
      for (size_t t = 0; t < nt; ++t) {
        rg[t] = cnt[t] ? make_uint2((uint32_t)total, (uint32_t)(total + cnt[t])) : make_uint2(0u, 0u);
        total += cnt[t];
      }
      e = hipMemcpy(trg, rg.data(), nt * 8, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMalloc(&tinst, std::max<size_t>(total, 1) * 4);
    if (e == hipSuccess) e = launch_tile_lists(n_views, c->TX, c->TY, sd, tcnt, trg, tinst, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    if (e == hipSuccess && d->ranges)
      for (size_t t = 0; t < nt; ++t) {
        d->ranges[2 * t] = rg[t].x;
        d->ranges[2 * t + 1] = rg[t].y;
      }
    if (e == hipSuccess && d->inst) {
      n_inst_out = std::min<size_t>(total, (size_t)std::max<int64_t>(0, d->n_inst));
      if (n_inst_out) e = hipMemcpy(d->inst, tinst, n_inst_out * 4, hipMemcpyDeviceToHost);
    }
    if (e == hipSuccess && d->n_blend) {
      // blended entries per pixel, counted by a debug kernel into a temporary
      int32_t* tmp = nullptr;
      e = hipMalloc(&tmp, std::max<size_t>(px, 1) * 4);
      if (e == hipSuccess)
        e = launch_count_blend(n_views, c->plan.width, c->plan.height, c->plan.tile_w,
                               c->plan.tile_h, c->TX, c->TY, sd, trg, tinst, tmp, hs);
      if (e == hipSuccess) e = hipStreamSynchronize(hs);
      if (e == hipSuccess) e = hipMemcpy(d->n_blend, tmp, px * 4, hipMemcpyDeviceToHost);
      if (tmp) (void)hipFree(tmp);
    }
    release();
    if (e != hipSuccess) return hip_fail(c, e, "debug tile lists");
  }
  if (d->t_final) cps.push_back({d->t_final, sd.tfinal, px * 4});
  if (d->last) cps.push_back({d->last, sd.last, px * 4});
  for (auto& x : cps)
    if (x.bytes && (e = hipMemcpy(x.dst, x.src, x.bytes, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(c, e, "debug copy");
  // the sorted lists and the rects live at visible-list positions: report
  // pair ids (the pair of each position, from the position of each pair)
  // and per-pair rects
  const size_t nvis = std::min<size_t>((size_t)h.vis_total, (size_t)c->plan.max_pairs);
  std::vector<uint32_t> vpair(nvis, 0xFFFFFFFFu);
  std::vector<uint32_t> vi(np);
  if (np && (e = hipMemcpy(vi.data(), sd.vidx, np * 4, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(c, e, "debug vidx");
  for (size_t i = 0; i < np; ++i)
    if (vi[i] < nvis) vpair[vi[i]] = (uint32_t)i;
  auto to_pair = [&](uint32_t* a, size_t n) {
    for (size_t i = 0; i < n; ++i) a[i] = a[i] < nvis ? vpair[a[i]] : 0xFFFFFFFFu;
  };
  if (d->order) to_pair(d->order, std::min<size_t>(np, h.vis_total));
  if (d->inst) to_pair(d->inst, n_inst_out);
  if (d->rects && np) {
    std::vector<uint2> r(std::max<size_t>(nvis, 1));
    if (nvis && (e = hipMemcpy(r.data(), sd.rect, nvis * 8, hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(c, e, "debug rect");
    for (size_t i = 0; i < np; ++i) {
      const bool vis = vi[i] < nvis;
      const uint2 q = vis ? r[vi[i]] : make_uint2(0u, 0u);
      d->rects[4 * i + 0] = (uint16_t)(q.x & 0xFFFF);
      d->rects[4 * i + 1] = (uint16_t)(q.x >> 16);
      d->rects[4 * i + 2] = (uint16_t)(q.y & 0xFFFF);
      d->rects[4 * i + 3] = (uint16_t)(q.y >> 16);
    }
  }
  if (d->vis_off)
    for (int v = 0; v <= n_views; ++v) d->vis_off[v] = h.vis_off[v];
  return GSR_OK;
}

gsr_status gsr_profile_enable(gsr_ctx* c, int enable) {
  if (!c) return GSR_E_INVALID_ARG;
  DeviceGuard g(c->device);
  if (enable && !c->ev[0][0]) {
    for (int i = 0; i < GSR_NUM_STAGES; ++i)
      for (int j = 0; j < 2; ++j) {
        hipError_t e = hipEventCreate(&c->ev[i][j]);
        if (e != hipSuccess) return hip_fail(c, e, "event create");
      }
  }
  c->prof = enable != 0;
  for (int i = 0; i < GSR_NUM_STAGES; ++i) c->ev_used[i] = false;
  return GSR_OK;
}

gsr_status gsr_profile_read(gsr_ctx* c, float* ms, int32_t n) {
  if (!c || !ms || n < 0) return GSR_E_INVALID_ARG;
  DeviceGuard g(c->device);
  for (int i = 0; i < n; ++i) {
    ms[i] = 0.f;
    if (i >= GSR_NUM_STAGES || !c->ev_used[i]) continue;
    hipError_t e = hipEventSynchronize(c->ev[i][1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms[i], c->ev[i][0], c->ev[i][1]);
    if (e != hipSuccess) return hip_fail(c, e, "profile read");
  }
  return GSR_OK;
}

gsr_status gsr_apply_pose_delta(const float* vin, const float* delta, float* vout, int32_t nv,
                                void* stream) {
  if (!vin || !delta || !vout || nv < 1) return GSR_E_INVALID_ARG;
  hipError_t e = launch_pose_delta(vin, delta, vout, nv, (hipStream_t)stream);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_sim3_gaussians(const float* means_in, const float* log_scales_in,
                              const float* quats_in, const int64_t* set_offsets, int32_t n_sets,
                              const float* sims, float* means_out, float* log_scales_out,
                              float* quats_out, void* stream) {
  if (!means_in || !log_scales_in || !quats_in || !set_offsets || !sims || !means_out ||
      !log_scales_out || !quats_out || n_sets < 1 || n_sets > GSR_MAX_SETS)
    return GSR_E_INVALID_ARG;
  SimSetTab tab{};
  tab.ns = n_sets;
  if (set_offsets[0] != 0) return GSR_E_INVALID_ARG;
  for (int k = 0; k <= n_sets; ++k) {
    if (k > 0 && set_offsets[k] < set_offsets[k - 1]) return GSR_E_INVALID_ARG;
    tab.off[k] = set_offsets[k];
  }
  if (set_offsets[n_sets] > (int64_t)0x7FFFFFFF * 64) return GSR_E_INVALID_ARG;
  hipError_t e = launch_sim3_gaussians(tab, means_in, log_scales_in, quats_in, sims, means_out,
                                       log_scales_out, quats_out, (hipStream_t)stream);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_sim3_views(const float* viewmats_in, const float* sims, const int32_t* view_set,
                          int32_t n_views, int32_t n_sets, float* viewmats_out, void* stream) {
  if (!viewmats_in || !sims || !view_set || !viewmats_out || n_views < 1 ||
      n_views > GSR_MAX_VIEWS || n_sets < 1 || n_sets > GSR_MAX_SETS)
    return GSR_E_INVALID_ARG;
  SimViewTab tab{};
  tab.nv = n_views;
  for (int v = 0; v < n_views; ++v) {
    if (view_set[v] < 0 || view_set[v] >= n_sets) return GSR_E_INVALID_ARG;
    tab.view_set[v] = view_set[v];
  }
  hipError_t e = launch_sim3_views(tab, viewmats_in, sims, viewmats_out, (hipStream_t)stream);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_l1_loss_grad(const float* color, const float* depth, const float* target_color,
                            const float* target_depth, const float* exposure, int32_t n_views,
                            int32_t width, int32_t height, float w_color, float w_depth,
                            float* d_color, float* d_depth, float* d_exposure, void* stream) {
  if (!color || !target_color || !d_color || n_views < 1 || width < 1 || height < 1)
    return GSR_E_INVALID_ARG;
  if (d_depth && (!depth || !target_depth)) return GSR_E_INVALID_ARG;
  if ((long)width * height > 0x7FFFFFFFL / 3) return GSR_E_INVALID_ARG;
  const int HW = width * height;
  // the loss terms are means over every channel / pixel of the batch
  const float wc = (float)((double)w_color / (3.0 * n_views * (double)HW));
  const float wd = (float)((double)w_depth / ((double)n_views * HW));
  hipError_t e = launch_l1_grad(n_views, HW, color, depth, target_color, target_depth, exposure,
                                wc, wd, d_color, d_depth, d_exposure, (hipStream_t)stream);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_ssim_workspace_bytes(int32_t n_views, int32_t width, int32_t height,
                                    size_t* out_bytes) {
  if (!out_bytes || n_views < 1 || width < 1 || height < 1) return GSR_E_INVALID_ARG;
  if ((double)n_views * width * height * 3 > 2147483647.0) return GSR_E_INVALID_ARG;
  *out_bytes = ssim_workspace_bytes(n_views, width, height);
  return GSR_OK;
}

gsr_status gsr_ssim_grad(const float* color, const float* target_color, const float* exposure,
                         int32_t n_views, int32_t width, int32_t height, float weight,
                         void* workspace, float* d_color, float* d_exposure, float* ssim_out,
                         void* stream) {
  if (!color || !target_color || !workspace || !d_color || n_views < 1 || width < 1 ||
      height < 1)
    return GSR_E_INVALID_ARG;
  if (((uintptr_t)workspace & 255) != 0) return GSR_E_INVALID_ARG;
  if ((double)n_views * width * height * 3 > 2147483647.0) return GSR_E_INVALID_ARG;
  if (3L * n_views > 65535L) return GSR_E_INVALID_ARG;  // grid y
  hipError_t e = launch_ssim(n_views, width, height, weight, color, target_color, exposure,
                             workspace, d_color, d_exposure, ssim_out, (hipStream_t)stream);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_dedup_workspace_bytes(int64_t table_slots, size_t* out_bytes) {
  if (!out_bytes || table_slots < 2 || (table_slots & (table_slots - 1)) != 0)
    return GSR_E_INVALID_ARG;
  *out_bytes = dedup_workspace_bytes(table_slots);
  return GSR_OK;
}

gsr_status gsr_dedup(const gsr_dedup_params* p, const float* tgt_means,
                     const float* tgt_log_scales, int64_t n_tgt, const float* depth,
                     const float* viewmats, const float* intrinsics, int32_t n_keyframes,
                     int32_t width, int32_t height, const float* src_means, int64_t n_src,
                     uint8_t* keep, void* workspace, int64_t* n_voxels, void* stream) {
  if (!p || !workspace || n_tgt < 0 || n_src < 0 || n_keyframes < 0) return GSR_E_INVALID_ARG;
  if (!(p->voxel > 0.0) || !(p->k_env >= 0.0) || p->table_slots < 2 ||
      (p->table_slots & (p->table_slots - 1)) != 0)
    return GSR_E_INVALID_ARG;
  if ((n_tgt > 0 && (!tgt_means || !tgt_log_scales)) || (n_src > 0 && (!src_means || !keep)))
    return GSR_E_INVALID_ARG;
  if (n_keyframes > 0 && (!depth || !viewmats || !intrinsics || width < 1 || height < 1))
    return GSR_E_INVALID_ARG;
  if (((uintptr_t)workspace & 255) != 0) return GSR_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  unsigned int* dc = nullptr;
  hipError_t e = launch_dedup(p->table_slots, workspace, p->voxel, p->k_env, tgt_means,
                              tgt_log_scales, n_tgt, depth, viewmats, intrinsics, n_keyframes,
                              width, height, src_means, n_src, keep, st, &dc);
  unsigned int h[2] = {0u, 0u};
  if (e == hipSuccess) e = hipMemcpyAsync(h, dc, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return GSR_E_DEVICE;
  if (n_voxels) *n_voxels = (int64_t)h[1];
  if (h[0] & 2u) return GSR_E_INVALID_ARG;  // inputs outside the voxel key range
  return (h[0] & 1u) ? GSR_E_OVERFLOW : GSR_OK;
}

gsr_status gsr_prune(const gsr_scene* sc, float min_opacity, float* means_out,
                     float* log_scales_out, float* quats_out, float* opacity_out,
                     float* colors_out, int64_t* set_offsets_out, void* stream) {
  if (!sc || !sc->means || !sc->log_scales || !sc->quats || !sc->opacity_logits ||
      !sc->colors || !sc->set_offsets || !means_out || !log_scales_out || !quats_out ||
      !opacity_out || !colors_out || !set_offsets_out)
    return GSR_E_INVALID_ARG;
  if (sc->n_sets < 1 || sc->n_sets > GSR_MAX_SETS || !(min_opacity > 0.f && min_opacity < 1.f))
    return GSR_E_INVALID_ARG;
  if (sc->sh_degree < 0 || sc->sh_degree > 3) return GSR_E_INVALID_ARG;
  const int cstride = sc->sh_degree > 0 ? 3 * sc->sh_stride : 3;
  if (sc->sh_degree > 0 && sc->sh_stride < (sc->sh_degree + 1) * (sc->sh_degree + 1))
    return GSR_E_INVALID_ARG;
  SimSetTab tab{};
  tab.ns = sc->n_sets;
  if (sc->set_offsets[0] != 0) return GSR_E_INVALID_ARG;
  for (int k = 0; k <= sc->n_sets; ++k) {
    if (k > 0 && sc->set_offsets[k] < sc->set_offsets[k - 1]) return GSR_E_INVALID_ARG;
    tab.off[k] = sc->set_offsets[k];
  }
  const long n = (long)sc->set_offsets[sc->n_sets];
  if (n > 0xFFFFFFFFL) return GSR_E_INVALID_ARG;
  // sigmoid is increasing: keep o >= logit(min_opacity); the FP32 threshold
  // is the smallest float not below the exact logit, so the FP32 test on an
  // FP32 logit is exact
  const double lg = log((double)min_opacity / (1.0 - (double)min_opacity));
  float thr = (float)lg;
  if ((double)thr < lg) thr = nextafterf(thr, INFINITY);
  SceneDev in = scene_dev(sc);
  hipStream_t st = (hipStream_t)stream;
  const size_t nb = (size_t)((n + 255) / 256);
  void* tmp = nullptr;
  if (hipMalloc(&tmp, 4 * (nb + 1) + 8 * (GSR_MAX_SETS + 1) + 256) != hipSuccess) {
    (void)hipGetLastError();
    return GSR_E_OOM;
  }
  uint32_t* blk = (uint32_t*)tmp;
  long long* bounds = (long long*)((char*)tmp + ((4 * (nb + 1) + 255) / 256) * 256);
  hipError_t e = launch_prune(n, in, cstride, thr, tab, blk, bounds, means_out, log_scales_out,
                              quats_out, opacity_out, colors_out, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(set_offsets_out, bounds, 8 * (size_t)(sc->n_sets + 1),
                       hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_iso_grad(const float* log_scales, int64_t n, float weight, float* d_log_scales,
                        void* stream) {
  if (n < 0 || (n > 0 && (!log_scales || !d_log_scales))) return GSR_E_INVALID_ARG;
  if (n > 0x7FFFFFFFL * 64L) return GSR_E_INVALID_ARG;
  hipError_t e = launch_iso_grad((long)n, log_scales, weight, d_log_scales, (hipStream_t)stream);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_normal_loss_grad(const float* depth, const float* normal_prior,
                                const float* intrinsics, int32_t n_views, int32_t width,
                                int32_t height, float weight, float* d_depth, void* stream) {
  if (!depth || !normal_prior || !intrinsics || !d_depth || n_views < 1 || width < 1 ||
      height < 1)
    return GSR_E_INVALID_ARG;
  const double tiles = (double)n_views * ((width + 15) / 16) * ((height + 15) / 16);
  if (tiles > 2147483647.0 || (double)n_views * width * height * 3 > 9.0e15)
    return GSR_E_INVALID_ARG;
  if (width < 3 || height < 3) return GSR_OK;  // no interior pixel: the loss is empty
  // the loss is a mean over the interior pixels of the batch
  const float w =
      (float)((double)weight / ((double)n_views * (double)(height - 2) * (double)(width - 2)));
  hipError_t e = launch_normal_grad(n_views, width, height, depth, normal_prior, intrinsics, w,
                                    d_depth, (hipStream_t)stream);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_seed(const float* depth, const float* color, const float* viewmat,
                    const float* intrinsics, int32_t width, int32_t height, int32_t stride,
                    float opacity_logit, int64_t max_out, float* means_out,
                    float* log_scales_out, float* quats_out, float* opacity_out,
                    float* colors_out, int64_t* n_out, void* stream) {
  if (!depth || !color || !viewmat || !intrinsics || !n_out || width < 1 || height < 1 ||
      stride < 1 || max_out < 0)
    return GSR_E_INVALID_ARG;
  if (max_out > 0 && (!means_out || !log_scales_out || !quats_out || !opacity_out || !colors_out))
    return GSR_E_INVALID_ARG;
  const long gm = (long)((width + stride - 1) / stride) * ((height + stride - 1) / stride);
  if ((double)width * height * 3 > 2147483647.0 || gm > 0x7FFFFFFFL) return GSR_E_INVALID_ARG;
  const size_t nb = (size_t)((gm + 255) / 256);
  void* tmp = nullptr;
  if (hipMalloc(&tmp, 4 * (nb + 1)) != hipSuccess) {
    (void)hipGetLastError();
    return GSR_E_OOM;
  }
  hipStream_t st = (hipStream_t)stream;
  uint32_t* blk = (uint32_t*)tmp;
  uint32_t total = 0;
  hipError_t e = launch_seed(width, height, stride, depth, color, viewmat, intrinsics,
                             opacity_logit, (long)max_out, blk, means_out, log_scales_out,
                             quats_out, opacity_out, colors_out, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&total, blk + nb, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  if (e != hipSuccess) return GSR_E_DEVICE;
  *n_out = (int64_t)total;
  return (int64_t)total > max_out ? GSR_E_OVERFLOW : GSR_OK;
}

gsr_status gsr_adam(const gsr_adam_group* groups, int32_t n_groups, double beta1, double beta2,
                    double eps, int32_t* step, void* stream) {
  if (!groups || !step || n_groups < 1 || n_groups > GSR_ADAM_MAX_GROUPS) return GSR_E_INVALID_ARG;
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps >= 0.0))
    return GSR_E_INVALID_ARG;
  long long chunks = 0;
  for (int k = 0; k < n_groups; ++k) {
    const gsr_adam_group& g = groups[k];
    if (g.n < 0 || (g.n > 0 && (!g.param || !g.grad || !g.exp_avg || !g.exp_avg_sq)))
      return GSR_E_INVALID_ARG;
    chunks += (g.n + 1023) / 1024;
  }
  if (chunks > 0x7FFFFFF8LL) return GSR_E_INVALID_ARG;
  hipError_t e = launch_adam(groups, n_groups, beta1, beta2, eps, step, (hipStream_t)stream);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_seed_noalloc(const float* depth, const float* color, const float* viewmat,
                            const float* intrinsics, int32_t width, int32_t height,
                            int32_t stride, float opacity_logit, int64_t max_out,
                            float* means_out, float* log_scales_out, float* quats_out,
                            float* opacity_out, float* colors_out, int64_t* n_out_dev,
                            void* stream) {
  if (!depth || !color || !viewmat || !intrinsics || !n_out_dev || width < 1 || height < 1 ||
      stride < 1 || max_out < 0)
    return GSR_E_INVALID_ARG;
  if (max_out > 0 && (!means_out || !log_scales_out || !quats_out || !opacity_out || !colors_out))
    return GSR_E_INVALID_ARG;
  if ((double)width * height * 3 > 2147483647.0) return GSR_E_INVALID_ARG;
  const long gm = (long)((width + stride - 1) / stride) * ((height + stride - 1) / stride);
  if (gm > SEED_NOALLOC_MAX_POINTS) return GSR_E_CAPACITY;
  const int nb = (int)((gm + 255) / 256);
  uint32_t* blk = nullptr;
  hipError_t e = seed_scratch(&blk);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return GSR_E_DEVICE;
  }
  hipStream_t st = (hipStream_t)stream;
  e = launch_seed(width, height, stride, depth, color, viewmat, intrinsics, opacity_logit,
                  (long)max_out, blk, means_out, log_scales_out, quats_out, opacity_out,
                  colors_out, st);
  if (e == hipSuccess) e = launch_seed_total(blk, nb, n_out_dev, st);
  return e == hipSuccess ? GSR_OK : GSR_E_DEVICE;
}

gsr_status gsr_autotune(int device, const gsr_plan_desc* base, const gsr_scene* sc,
                        const gsr_views* vw, const gsr_settings* set, gsr_plan_desc* best,
                        float* best_ms, void* stream) {
  if (!base || !sc || !vw || !best || !best_ms) return GSR_E_INVALID_ARG;
  if (check_plan(nullptr, base) != GSR_OK) return GSR_E_INVALID_ARG;
  // Coordinate search: every tile shape with one and (where allowed) two
  // tiles per backward wave (other options at their defaults), then for the
  // best plan so far the binning chunk (depth-sorted pairs per wave of the
  // row binning), the forward's entries per lane, the backward's entries
  // per lane, and the persistent tile queue.
  static const int tiles[][3] = {{16, 16, 1}, {16, 16, 2}, {16, 8, 1}, {16, 8, 2}, {8, 16, 1},
                                 {8, 16, 2},  {8, 8, 1},   {8, 8, 2},  {32, 8, 1}, {32, 16, 1},
                                 {16, 32, 1}};
  static const int chunks[] = {64, 128, 256};
  static const int fbs[] = {1, 2};
  static const int bbs[] = {1, 2, 4};
  static const int pers[] = {0, 1};
  constexpr int NT_ = sizeof(tiles) / sizeof(tiles[0]), NC_ = sizeof(chunks) / sizeof(chunks[0]);
  constexpr int NF_ = 2, NB_ = 3, NP_ = 2;
  hipStream_t st = (hipStream_t)stream;
  DeviceGuard g(device);
  const int V = vw->n_views, W = vw->width, H = vw->height;
  const long N = sc->set_offsets[sc->n_sets];
  const long kcol = sc->sh_degree > 0 ? (long)sc->sh_stride * 3 : 3;
  const size_t px = (size_t)V * W * H;
  // outputs, a constant upstream gradient and gradient buffers (set-up only)
  const size_t n_img = 5 * px, n_grad = (size_t)N * (3 + 3 + 4 + 1 + kcol) + 6 * (size_t)V;
  float* buf = nullptr;
  if (hipMalloc(&buf, (n_img + 5 * px + n_grad) * sizeof(float)) != hipSuccess) return GSR_E_OOM;
  float* up = buf + n_img;
  float* gb = up + 5 * px;
  {
    std::vector<float> ones(5 * px, 1.0f / (float)px);
    if (hipMemcpy(up, ones.data(), ones.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(buf);
      return GSR_E_DEVICE;
    }
  }
  gsr_images img{buf, buf + 3 * px, buf + 4 * px, nullptr};
  gsr_grad_images gin{up, up + 3 * px, up + 4 * px};
  gsr_grads gr{gb, gb + 3 * N, gb + 6 * N, gb + 10 * N, gb + 11 * N, gb + 11 * N + kcol * N};
  float best_t = 1e30f;
  gsr_plan_desc best_p = *base;
  gsr_status result = GSR_E_INVALID_ARG;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  for (int ci = 0; ci < NT_ + NC_ + NF_ + NB_ + NP_; ++ci) {
    gsr_plan_desc p = *base;
    if (ci < NT_) {
      p.tile_w = tiles[ci][0];
      p.tile_h = tiles[ci][1];
      p.bwd_cols = tiles[ci][2];
      p.chunk = 0;
      p.fwd_batch = 1;
      p.bwd_batch = 1;
      p.persistent = 0;
    } else {
      if (result != GSR_OK) break;  // no tile shape ran
      p = best_p;
      int k = ci - NT_;
      if (k < NC_) {
        p.chunk = chunks[k];
      } else if ((k -= NC_) < NF_) {
        p.fwd_batch = fbs[k];
      } else if ((k -= NF_) < NB_) {
        p.bwd_batch = bbs[k];
      } else {
        p.persistent = pers[k - NB_];
      }
    }
    if (check_plan(nullptr, &p) != GSR_OK) continue;
    gsr_ctx* ctx = nullptr;
    if (gsr_create(&ctx, device) != GSR_OK) { result = GSR_E_DEVICE; break; }
    void* state = nullptr;
    size_t sb = 0;
    float t_ms = -1.f;
    for (int attempt = 0; attempt < 2 && t_ms < 0.f; ++attempt) {
      if (gsr_plan(ctx, &p) != GSR_OK) break;
      gsr_state_bytes(&p, &sb);
      if (state) (void)hipFree(state);
      state = nullptr;
      if (hipMalloc(&state, sb) != hipSuccess) { state = nullptr; break; }
      if (gsr_forward(ctx, sc, vw, set, state, &img, st) != GSR_OK) break;
      gsr_counts cnt;
      gsr_status ps = gsr_poll(ctx, state, &cnt, st);
      if (ps == GSR_E_OVERFLOW) {
        p.max_instances =
            std::min<int64_t>(0xFFFFFFFEL, cnt.row_entries + cnt.row_entries / 8 + 1024);
        continue;
      }
      if (ps != GSR_OK) break;
      if (gsr_backward(ctx, sc, vw, set, state, &gin, &gr, st) != GSR_OK) break;
      float tmin = 1e30f;
      for (int rep = 0; rep < 5; ++rep) {
        (void)hipEventRecord(e0, st);
        gsr_forward(ctx, sc, vw, set, state, &img, st);
        gsr_backward(ctx, sc, vw, set, state, &gin, &gr, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        tmin = std::min(tmin, ms);
      }
      t_ms = tmin;
    }
    if (state) (void)hipFree(state);
    gsr_destroy(ctx);
    if (t_ms >= 0.f) {
      result = GSR_OK;
      // a candidate replaces the best plan so far only if it is faster by
      // more than the run-to-run spread (3%): near-equal candidates keep the
      // earlier choice, so repeated tunings agree
      if (t_ms < 0.97f * best_t) {
        best_t = t_ms;
        best_p = p;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  if (result == GSR_OK) {
    *best = best_p;
    *best_ms = best_t;
  }
  return result;
}

}  // extern "C"
