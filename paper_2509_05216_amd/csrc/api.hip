// C ABI of the isogs library: contexts, device scratch, cameras and the
// orchestration of the forward/backward passes on a caller's HIP stream.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>

#include "internal.h"

namespace isogs {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

gs_status hip_fail(hipError_t e, const char* what) {
  set_error("%s failed: %s", what, hipGetErrorString(e));
  return (e == hipErrorOutOfMemory) ? GS_ERR_NOMEM : GS_ERR_HIP;
}

gs_status buf_ensure(Ctx* ctx, DevBuf& b, size_t bytes, hipStream_t s, hipEvent_t prior) {
  if (bytes <= b.cap) return GS_OK;
  if (ctx->capturing) {
    set_error("internal: a buffer would grow (%zu -> %zu bytes) during graph capture", b.cap,
              bytes);
    return GS_ERR_CAPACITY;
  }
  size_t want = bytes + bytes / 8;
  want = (want + 4095) & ~(size_t)4095;
  {
    std::lock_guard<std::mutex> lk(ctx->mem_mutex);
    const size_t after = ctx->in_use - b.cap + want;
    if (ctx->budget != 0 && after > ctx->budget) {
      set_error("device scratch budget exceeded: need %zu bytes, budget %zu", after,
                ctx->budget);
      return GS_ERR_NOMEM;
    }
  }
  if (b.p != nullptr) {
    // work queued on s, and before `prior`, may still use the old buffer
    GS_HIP(hipStreamSynchronize(s));
    if (prior != nullptr) GS_HIP(hipEventSynchronize(prior));
    GS_HIP(hipFree(b.p));
    {
      std::lock_guard<std::mutex> lk(ctx->mem_mutex);
      ctx->in_use -= b.cap;
    }
    b.p = nullptr;
    b.cap = 0;
  }
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    set_error("hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    return GS_ERR_NOMEM;
  }
  b.cap = want;
  std::lock_guard<std::mutex> lk(ctx->mem_mutex);
  ctx->in_use += want;
  if (ctx->in_use > ctx->peak) ctx->peak = ctx->in_use;
  return GS_OK;
}

void buf_free(Ctx* ctx, DevBuf& b) {
  if (b.p != nullptr) {
    (void)hipFree(b.p);
    std::lock_guard<std::mutex> lk(ctx->mem_mutex);
    ctx->in_use -= b.cap;
  }
  b.p = nullptr;
  b.cap = 0;
}

// ------------------------------------------------------------ stage timing
static hipEvent_t take_event(Ctx* c) {
  if (c->n_free > 0) return c->free_events[--c->n_free];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

static void give_event(Ctx* c, hipEvent_t e) {
  if (e == nullptr) return;
  if (c->n_free == c->cap_free) {
    const int nc = c->cap_free ? 2 * c->cap_free : 64;
    auto* p = new hipEvent_t[nc];
    for (int i = 0; i < c->n_free; ++i) p[i] = c->free_events[i];
    delete[] c->free_events;
    c->free_events = p;
    c->cap_free = nc;
  }
  c->free_events[c->n_free++] = e;
}

StageTimer::StageTimer(Ctx* c_, int st, hipStream_t s_) : c(c_), stage(st), s(s_) {
  if (c == nullptr || !c->timing || c->capturing) return;
  a = take_event(c);
  if (a != nullptr && hipEventRecord(a, s) != hipSuccess) {
    give_event(c, a);
    a = nullptr;
  }
}

StageTimer::~StageTimer() {
  if (a == nullptr) return;
  hipEvent_t b = take_event(c);
  if (b == nullptr || hipEventRecord(b, s) != hipSuccess) {
    give_event(c, a);
    give_event(c, b);
    return;
  }
  if (c->n_pending == c->cap_pending) {
    const int nc = c->cap_pending ? 2 * c->cap_pending : 64;
    auto* p = new PendingTiming[nc];
    for (int i = 0; i < c->n_pending; ++i) p[i] = c->pending[i];
    delete[] c->pending;
    c->pending = p;
    c->cap_pending = nc;
  }
  c->pending[c->n_pending++] = PendingTiming{stage, a, b};
}

gs_status timing_collect(Ctx* c) {
  for (int i = 0; i < c->n_pending; ++i) {
    PendingTiming& t = c->pending[i];
    GS_HIP(hipEventSynchronize(t.b));
    float ms = 0.f;
    GS_HIP(hipEventElapsedTime(&ms, t.a, t.b));
    c->stage_ms[t.stage] += ms;
    c->stage_count[t.stage] += 1;
    give_event(c, t.a);
    give_event(c, t.b);
  }
  c->n_pending = 0;
  return GS_OK;
}

static const char* kStageNames[ST_COUNT] = {
    "project", "depth_sort", "scan", "emit", "tile_sort", "ranges", "blend_fwd",
    "loss", "blend_bwd", "project_bwd", "adam", "init", "probe", "densify"};

size_t Frame::bytes() const {
  size_t s = splat.cap + rect.cap + dkey.cap + dkw[0].cap + dkw[1].cap + sidx[0].cap +
             sidx[1].cap + clampm.cap + offs.cap + tkey[0].cap + tkey[1].cap + tval[0].cap +
             tval[1].cap + ranges.cap + finalT.cap + ncon.cap + acc.cap + ss.hist.cap +
             ss.partial.cap + ss.total.cap + words.cap + okey[0].cap + okey[1].cap +
             oval[0].cap + oval[1].cap + radii.cap + gmu.cap;
  return s;
}

static void frame_free(Frame* f) {
  Ctx* c = f->ctx;
  DevBuf* all[] = {&f->splat,   &f->rect,    &f->dkey,    &f->dkw[0],     &f->dkw[1],
                   &f->sidx[0], &f->sidx[1], &f->clampm,  &f->offs,       &f->tkey[0],
                   &f->tkey[1], &f->tval[0], &f->tval[1], &f->ranges,     &f->finalT,
                   &f->ncon,    &f->acc,     &f->ss.hist, &f->ss.partial, &f->ss.total,
                   &f->words,   &f->okey[0], &f->okey[1], &f->oval[0],    &f->oval[1],
                   &f->radii,   &f->gmu};
  for (DevBuf* b : all) buf_free(c, *b);
  if (f->pinned != nullptr) (void)hipHostFree(f->pinned);
  f->pinned = nullptr;
  if (f->last_use != nullptr) (void)hipEventDestroy(f->last_use);
  f->last_use = nullptr;
  if (f->side != nullptr) (void)hipStreamDestroy(f->side);
  if (f->fork_ev != nullptr) (void)hipEventDestroy(f->fork_ev);
  if (f->join_ev != nullptr) (void)hipEventDestroy(f->join_ev);
  f->side = nullptr;
  f->fork_ev = f->join_ev = nullptr;
  f->ss.prior = nullptr;
}

static bool valid_params(const gs_params& p, const char* what) {
  if (p.means == nullptr || p.log_scales == nullptr || p.quats == nullptr ||
      p.opacity_logits == nullptr || p.sh == nullptr) {
    set_error("%s: null parameter pointer", what);
    return false;
  }
  if (p.n < 1 || p.n > 0x7fffffff) {
    set_error("%s: n = %lld out of range", what, (long long)p.n);
    return false;
  }
  if (p.sh_degree < 0 || p.sh_degree > 3) {
    set_error("%s: sh_degree %d not in 0..3", what, p.sh_degree);
    return false;
  }
  return true;
}

static bool valid_camera(const gs_camera& c, int v) {
  if (c.width < 1 || c.width > 16384 || c.height < 1 || c.height > 16384) {
    set_error("camera %d: size %dx%d outside [1, 16384]", v, c.width, c.height);
    return false;
  }
  if (!(c.fx > 0) || !(c.fy > 0) || !(c.z_near > 0)) {
    set_error("camera %d: focal lengths and z_near must be positive", v);
    return false;
  }
  return true;
}

GradsDev grads_dev(const gs_params& g, int flags) {
  GradsDev d;
  d.means = g.means;
  d.log_scales = g.log_scales;
  d.quats = g.quats;
  d.logits = g.opacity_logits;
  d.sh = g.sh;
  d.accumulate = (flags & GS_BWD_ACCUMULATE) != 0;
  d.keep_screen = (flags & GS_BWD_KEEP_SCREEN) != 0;
  return d;
}

ParamsDev params_dev(const gs_params& p) {
  ParamsDev d;
  d.means = p.means;
  d.log_scales = p.log_scales;
  d.quats = p.quats;
  d.logits = p.opacity_logits;
  d.sh = p.sh;
  d.n = (int)p.n;
  d.sh_degree = p.sh_degree;
  return d;
}

// Fill the view table of a frame from host cameras.
static gs_status build_views(Frame& f, const gs_camera* cams, int nv, float* const* images,
                             const float bg[3]) {
  ViewTable& vt = f.vt;
  std::memset(&vt, 0, sizeof(vt));
  vt.n = nv;
  vt.tile = f.tile;
  for (int k = 0; k < 3; ++k) vt.bg[k] = bg[k];
  long long tiles = 0, pix = 0;
  for (int v = 0; v < nv; ++v) {
    const gs_camera& c = cams[v];
    CamDev& d = vt.v[v];
    for (int k = 0; k < 9; ++k) d.R[k] = c.R[k];
    for (int k = 0; k < 3; ++k) d.t[k] = c.t[k];
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    d.znear = c.z_near;
    d.limx = kGuard * (0.5 * (double)c.width / (double)c.fx);
    d.limy = kGuard * (0.5 * (double)c.height / (double)c.fy);
    for (int k = 0; k < 3; ++k)  // camera centre -R^T t
      d.campos[k] = (float)(-((double)c.R[0 * 3 + k] * c.t[0] + (double)c.R[1 * 3 + k] * c.t[1] +
                              (double)c.R[2 * 3 + k] * c.t[2]));
    d.W = c.width;
    d.H = c.height;
    d.tiles_x = (c.width + f.tile - 1) / f.tile;
    d.tiles_y = (c.height + f.tile - 1) / f.tile;
    d.tile_offset = (int)tiles;
    d.entry_off = (uint32_t)((size_t)v * (size_t)f.n);  // multi-scene frames overwrite these
    d.pix_offset = pix;
    d.image = images != nullptr ? images[v] : nullptr;
    d.dimg = nullptr;
    tiles += (long long)d.tiles_x * d.tiles_y;
    pix += (long long)c.width * c.height;
  }
  if (tiles >= 0x7fffffffLL) {
    set_error("too many tiles (%lld)", tiles);
    return GS_ERR_INVALID;
  }
  vt.total_tiles = (int)tiles;
  f.total_pix = pix;
  int bits = 1;
  while ((1LL << bits) < tiles) ++bits;
  f.key_bits = bits;
  return GS_OK;
}

// Sizes the frame's buffers for its views; s: the stream of the calling pass.
static gs_status frame_buffers(Frame& f, hipStream_t s) {
  Ctx* c = f.ctx;
  const size_t vn = (size_t)f.entries;
  gs_status st;
  if (f.last_use == nullptr) {
    GS_HIP(hipEventCreateWithFlags(&f.last_use, hipEventDisableTiming));
    f.ss.prior = f.last_use;
  }
#define ENS(buf, bytes)                                       \
  do {                                                        \
    st = buf_ensure(c, (buf), (bytes), s, f.last_use);        \
    if (st != GS_OK) return st;                               \
  } while (0)
  ENS(f.splat, vn * 48);
  ENS(f.rect, vn * 8);
  ENS(f.dkey, vn * 4);
  ENS(f.dkw[0], vn * 4);
  ENS(f.dkw[1], vn * 4);
  ENS(f.sidx[0], vn * 4);
  ENS(f.sidx[1], vn * 4);
  ENS(f.clampm, vn);
  ENS(f.offs, vn * 4);
  ENS(f.ranges, (size_t)f.vt.total_tiles * 8);
  ENS(f.finalT, (size_t)f.total_pix * 4);
  ENS(f.ncon, (size_t)f.total_pix * 4);
  if (f.keep_radii) ENS(f.radii, vn * 4);
  if (!f.multi) {  // the projection backward's side stream and mean scratch
    ENS(f.gmu, (size_t)f.n * 12);
    if (f.side == nullptr) {
      GS_HIP(hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking));
      GS_HIP(hipEventCreateWithFlags(&f.fork_ev, hipEventDisableTiming));
      GS_HIP(hipEventCreateWithFlags(&f.join_ev, hipEventDisableTiming));
    }
  }
  const size_t acc_bytes = f.multi ? 0 : vn * kAccStride * 4;  // forward-only frames need none
  if (f.acc.cap < acc_bytes) {
    ENS(f.acc, acc_bytes);
    f.acc_zeroed = false;
  }
#undef ENS
  if (f.words.cap == 0) {
    st = buf_ensure(c, f.words, kWordCount * 4, s);
    if (st != GS_OK) return st;
    // cleared on the pass's own stream, ahead of the kernels that use the words
    st = launch_fill_u32(f.words.p, 0u, kWordCount, s);
    if (st != GS_OK) return st;
  }
  if (f.pinned == nullptr) GS_HIP(hipHostMalloc((void**)&f.pinned, 64, hipHostMallocDefault));
  return GS_OK;
}

static gs_status set_device(Ctx* ctx) {
  GS_HIP(hipSetDevice(ctx->device));
  return GS_OK;
}

}  // namespace isogs

using namespace isogs;

namespace isogs {

// Frees a context (its events, loss scratch and host state) once nothing holds it.
static void ctx_free(gs_ctx* ctx) {
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->loss_scratch != nullptr) {
    loss_scratch_free(ctx, *ctx->loss_scratch);
    delete ctx->loss_scratch;
    ctx->loss_scratch = nullptr;
  }
  buf_free(ctx, ctx->dens_blk);
  buf_free(ctx, ctx->init_xyz);
  if (ctx->dens_host != nullptr) (void)hipHostFree(ctx->dens_host);
  ctx->dens_host = nullptr;
  buf_free(ctx, ctx->iso_blk);
  if (ctx->iso_host != nullptr) (void)hipHostFree(ctx->iso_host);
  ctx->iso_host = nullptr;
  (void)timing_collect(ctx);
  for (int i = 0; i < ctx->n_free; ++i) (void)hipEventDestroy(ctx->free_events[i]);
  delete[] ctx->free_events;
  delete[] ctx->pending;
  delete ctx;
}

void ctx_retain(Ctx* ctx) {
  std::lock_guard<std::mutex> lk(ctx->life_mutex);
  ++ctx->dependents;
}

void ctx_release(Ctx* ctx) {
  bool now;
  {
    std::lock_guard<std::mutex> lk(ctx->life_mutex);
    now = --ctx->dependents == 0 && ctx->destroy_requested;
  }
  if (now) ctx_free(static_cast<gs_ctx*>(ctx));
}

// A frame's buffers, the frame and its hold on the context.
static void frame_delete(gs_frame* fr) {
  Ctx* ctx = fr->ctx;
  frame_free(fr);
  delete fr;
  ctx_release(ctx);
}

}  // namespace isogs

extern "C" {

const char* gs_last_error(void) { return g_err; }

const char* gs_version(void) { return "isogs 0.1 gfx950"; }

gs_status gs_ctx_create(int device, size_t mem_budget, gs_ctx** out) {
  if (out == nullptr) {
    set_error("gs_ctx_create: out is null");
    return GS_ERR_INVALID;
  }
  *out = nullptr;
  int count = 0;
  GS_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) {
    set_error("gs_ctx_create: device %d not in [0, %d)", device, count);
    return GS_ERR_INVALID;
  }
  gs_ctx* c = new (std::nothrow) gs_ctx();
  if (c == nullptr) {
    set_error("gs_ctx_create: out of host memory");
    return GS_ERR_NOMEM;
  }
  c->device = device;
  c->budget = mem_budget;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipGetDeviceProperties(&c->prop, device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDeviceProperties");
  }
  if (std::strncmp(c->prop.gcnArchName, "gfx950", 6) != 0) {
    set_error("device %d is %s; this library is built for gfx950 only", device,
              c->prop.gcnArchName);
    delete c;
    return GS_ERR_UNSUPPORTED;
  }
  c->cu_count = c->prop.multiProcessorCount;
  // address of this device's fixed loss workspace (gs_loss_grad_noalloc)
  const gs_status ws = loss_noalloc_setup(device);
  if (ws != GS_OK) {
    delete c;
    return ws;
  }
  *out = c;
  return GS_OK;
}

void gs_ctx_destroy(gs_ctx* ctx) {
  if (ctx == nullptr) return;
  bool now;
  {
    std::lock_guard<std::mutex> lk(ctx->life_mutex);
    ctx->destroy_requested = true;
    now = ctx->dependents == 0;
  }
  if (now) isogs::ctx_free(ctx);
}

gs_status gs_ctx_set_timing(gs_ctx* ctx, int32_t enable) {
  if (ctx == nullptr) {
    set_error("gs_ctx_set_timing: null context");
    return GS_ERR_INVALID;
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  st = timing_collect(ctx);
  if (st != GS_OK) return st;
  ctx->timing = enable != 0;
  for (int i = 0; i < ST_COUNT; ++i) {
    ctx->stage_ms[i] = 0.0;
    ctx->stage_count[i] = 0;
  }
  return GS_OK;
}

gs_status gs_ctx_stage_time(gs_ctx* ctx, int32_t stage, double* total_ms, int64_t* launches) {
  if (ctx == nullptr || stage < 0 || stage >= ST_COUNT) {
    set_error("gs_ctx_stage_time: bad context or stage %d", stage);
    return GS_ERR_INVALID;
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  st = timing_collect(ctx);
  if (st != GS_OK) return st;
  if (total_ms) *total_ms = ctx->stage_ms[stage];
  if (launches) *launches = ctx->stage_count[stage];
  return GS_OK;
}

const char* gs_stage_name(int32_t stage) {
  return (stage >= 0 && stage < ST_COUNT) ? kStageNames[stage] : nullptr;
}

gs_status gs_ctx_memory(gs_ctx* ctx, size_t* in_use, size_t* peak) {
  if (ctx == nullptr) {
    set_error("gs_ctx_memory: null context");
    return GS_ERR_INVALID;
  }
  if (in_use) *in_use = ctx->in_use;
  if (peak) *peak = ctx->peak;
  return GS_OK;
}

gs_status gs_orbit_cameras(int32_t n_views, float radius, float fov_y_deg, int32_t width,
                           int32_t height, gs_camera* out) {
  if (out == nullptr || n_views < 1 || !(radius > 0) || !(fov_y_deg > 0) || !(fov_y_deg < 180) ||
      width < 1 || width > 16384 || height < 1 || height > 16384) {
    set_error("gs_orbit_cameras: invalid arguments");
    return GS_ERR_INVALID;
  }
  const double pi = 3.14159265358979323846;
  const double f = height / (2.0 * std::tan(fov_y_deg * pi / 360.0));
  const double golden = pi * (3.0 - std::sqrt(5.0));
  for (int i = 0; i < n_views; ++i) {
    const double y = 1.0 - 2.0 * (i + 0.5) / n_views;
    const double rxz = std::sqrt(std::fmax(0.0, 1.0 - y * y));
    const double phi = i * golden;
    const double C[3] = {radius * rxz * std::cos(phi), radius * y, radius * rxz * std::sin(phi)};
    const double up[3] = {0.0, std::fabs(y) > 0.99 ? 0.0 : 1.0, std::fabs(y) > 0.99 ? 1.0 : 0.0};
    // forward = normalise(-C); right = normalise(forward x up); down = forward x right
    double fw[3] = {-C[0], -C[1], -C[2]};
    double ln = std::sqrt(fw[0] * fw[0] + fw[1] * fw[1] + fw[2] * fw[2]);
    for (double& x : fw) x /= ln;
    double rt[3] = {fw[1] * up[2] - fw[2] * up[1], fw[2] * up[0] - fw[0] * up[2],
                    fw[0] * up[1] - fw[1] * up[0]};
    ln = std::sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
    for (double& x : rt) x /= ln;
    const double dn[3] = {fw[1] * rt[2] - fw[2] * rt[1], fw[2] * rt[0] - fw[0] * rt[2],
                          fw[0] * rt[1] - fw[1] * rt[0]};
    gs_camera& c = out[i];
    std::memset(&c, 0, sizeof(c));
    const double* rows[3] = {rt, dn, fw};
    for (int r = 0; r < 3; ++r) {
      for (int k = 0; k < 3; ++k) c.R[r * 3 + k] = (float)rows[r][k];
      c.t[r] = (float)(-(rows[r][0] * C[0] + rows[r][1] * C[1] + rows[r][2] * C[2]));
    }
    c.fx = (float)f;
    c.fy = (float)f;
    c.cx = (float)(width / 2.0);
    c.cy = (float)(height / 2.0);
    c.z_near = 0.2f;
    c.width = width;
    c.height = height;
  }
  return GS_OK;
}

gs_status gs_init_from_points(gs_ctx* ctx, const float* xyz, int64_t n, const gs_init_opts* opts,
                              uint64_t seed, gs_params out, void* stream) {
  if (ctx == nullptr || xyz == nullptr || opts == nullptr) {
    set_error("gs_init_from_points: null argument");
    return GS_ERR_INVALID;
  }
  if (!valid_params(out, "gs_init_from_points") || out.n != n) {
    if (out.n != n) set_error("gs_init_from_points: out.n (%lld) != n (%lld)", (long long)out.n,
                              (long long)n);
    return GS_ERR_INVALID;
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  // the points may be host or device memory; host points are copied to a context
  // buffer first (a pageable pointer is unknown to HIP: clear that query's error)
  hipPointerAttribute_t attr{};
  const hipError_t pe = hipPointerGetAttributes(&attr, xyz);
  if (pe != hipSuccess) (void)hipGetLastError();
  const bool on_device =
      pe == hipSuccess && (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged);
  const float* src = xyz;
  if (!on_device && n > 0) {
    st = buf_ensure(ctx, ctx->init_xyz, (size_t)n * 3 * sizeof(float), s);
    if (st != GS_OK) return st;
    GS_HIP(hipMemcpyAsync(ctx->init_xyz.p, xyz, (size_t)n * 3 * sizeof(float),
                          hipMemcpyHostToDevice, s));
    src = (const float*)ctx->init_xyz.p;
  }
  {
    StageTimer tm(ctx, ST_INIT, s);
    st = launch_init_points(src, n, *opts, seed, out, s);
  }
  if (st == GS_OK && src != xyz) GS_HIP(hipStreamSynchronize(s));
  return st;
}

gs_status gs_render_fwd(gs_ctx* ctx, gs_params params, const gs_camera* cams, int32_t n_views,
                        float* const* images, const gs_render_opts* opts, gs_frame** state,
                        void* stream) {
  if (ctx == nullptr || cams == nullptr || images == nullptr || state == nullptr) {
    set_error("gs_render_fwd: null argument");
    return GS_ERR_INVALID;
  }
  if (!valid_params(params, "gs_render_fwd")) return GS_ERR_INVALID;
  if (n_views < 1 || n_views > kMaxViews) {
    set_error("gs_render_fwd: n_views %d not in [1, %d]", n_views, kMaxViews);
    return GS_ERR_INVALID;
  }
  for (int v = 0; v < n_views; ++v) {
    if (!valid_camera(cams[v], v)) return GS_ERR_INVALID;
    if (images[v] == nullptr) {
      set_error("gs_render_fwd: images[%d] is null", v);
      return GS_ERR_INVALID;
    }
  }
  if ((uint64_t)n_views * (uint64_t)params.n > kMaxRecords) {
    set_error("gs_render_fwd: n_views * n exceeds %llu", (unsigned long long)kMaxRecords);
    return GS_ERR_CAPACITY;
  }
  int tile = 16, depth = 256, flags = 0;
  float bg[3] = {0.f, 0.f, 0.f};
  if (opts != nullptr) {
    tile = opts->tile;
    depth = opts->lds_depth == 0 ? 256 : opts->lds_depth;
    flags = opts->flags;
    for (int k = 0; k < 3; ++k) bg[k] = opts->bg[k];
  }
  if ((flags & ~(GS_RENDER_PERSISTENT | GS_RENDER_LONGEST_FIRST | GS_RENDER_RADII)) != 0) {
    set_error("gs_render_fwd: unknown render flags 0x%x", flags);
    return GS_ERR_INVALID;
  }
  if (tile != 8 && tile != 16 && tile != 32) {
    set_error("gs_render_fwd: tile %d not in {8, 16, 32}", tile);
    return GS_ERR_INVALID;
  }
  if (depth != 32 && depth != 64 && depth != 128 && depth != 256) {
    set_error("gs_render_fwd: lds_depth %d not in {32, 64, 128, 256}", depth);
    return GS_ERR_INVALID;
  }
  if (tile == 8 && depth > 64) depth = 64;
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  hipStream_t s = (hipStream_t)stream;

  gs_frame* fr = *state;
  const bool fresh = (fr == nullptr);
  if (fresh) {
    fr = new (std::nothrow) gs_frame();
    if (fr == nullptr) {
      set_error("gs_render_fwd: out of host memory");
      return GS_ERR_NOMEM;
    }
    fr->ctx = ctx;
    ctx_retain(ctx);
  } else if (fr->ctx != ctx) {
    set_error("gs_render_fwd: frame belongs to another context");
    return GS_ERR_INVALID;
  }
  Frame& f = *fr;
  f.n = params.n;
  f.entries = (int64_t)n_views * params.n;
  f.multi = false;
  f.n_groups = 0;
  f.views = n_views;
  f.tile = tile;
  f.depth = depth;
  f.persistent = (flags & GS_RENDER_PERSISTENT) != 0;
  f.lpt = f.persistent && (flags & GS_RENDER_LONGEST_FIRST) != 0;
  f.tile_order = nullptr;
  f.sh_degree = params.sh_degree;
  f.K = 0;
  f.keep_radii = (flags & GS_RENDER_RADII) != 0;
  f.screen_kept = false;
  st = build_views(f, cams, n_views, images, bg);
  if (st == GS_OK) st = frame_buffers(f, s);
  if (st != GS_OK) {
    if (fresh) frame_delete(fr);
    return st;
  }
  if (!f.acc_zeroed && !f.multi) {
    st = launch_fill_u32(f.acc.p, 0u, (size_t)f.entries * kAccStride, s);
    if (st != GS_OK) {
      if (fresh) frame_delete(fr);
      return st;
    }
    f.acc_zeroed = true;
  }
  *state = fr;
  st = forward_stages(ctx, f, params_dev(params), s, 0);
  if (st != GS_OK) return st;
  GS_HIP(hipEventRecord(f.last_use, s));
  return GS_OK;
}

gs_status gs_render_fwd_multi(gs_ctx* ctx, const gs_params* params, const gs_camera* cams,
                              int32_t n_views, float* const* images, const gs_render_opts* opts,
                              gs_frame** state, void* stream) {
  if (ctx == nullptr || params == nullptr || cams == nullptr || images == nullptr ||
      state == nullptr) {
    set_error("gs_render_fwd_multi: null argument");
    return GS_ERR_INVALID;
  }
  if (n_views < 1 || n_views > kMaxViews) {
    set_error("gs_render_fwd_multi: n_views %d not in [1, %d]", n_views, kMaxViews);
    return GS_ERR_INVALID;
  }
  uint64_t total = 0;
  for (int v = 0; v < n_views; ++v) {
    if (!valid_params(params[v], "gs_render_fwd_multi")) return GS_ERR_INVALID;
    if (!valid_camera(cams[v], v)) return GS_ERR_INVALID;
    if (images[v] == nullptr) {
      set_error("gs_render_fwd_multi: images[%d] is null", v);
      return GS_ERR_INVALID;
    }
    total += (uint64_t)params[v].n;
  }
  if (total > kMaxRecords) {
    set_error("gs_render_fwd_multi: the views' Gaussian counts sum past %llu",
              (unsigned long long)kMaxRecords);
    return GS_ERR_CAPACITY;
  }
  int tile = 16, depth = 256, flags = 0;
  float bg[3] = {0.f, 0.f, 0.f};
  if (opts != nullptr) {
    tile = opts->tile;
    depth = opts->lds_depth == 0 ? 256 : opts->lds_depth;
    flags = opts->flags;
    for (int k = 0; k < 3; ++k) bg[k] = opts->bg[k];
  }
  if ((flags & ~(GS_RENDER_PERSISTENT | GS_RENDER_LONGEST_FIRST)) != 0) {
    set_error("gs_render_fwd_multi: render flags 0x%x not supported here", flags);
    return GS_ERR_INVALID;
  }
  if ((tile != 8 && tile != 16 && tile != 32) ||
      (depth != 32 && depth != 64 && depth != 128 && depth != 256)) {
    set_error("gs_render_fwd_multi: tile %d / lds_depth %d", tile, depth);
    return GS_ERR_INVALID;
  }
  if (tile == 8 && depth > 64) depth = 64;
  // views grouped by scene (scenes in order of first appearance, views in order)
  int order[kMaxViews], gid[kMaxViews], ng = 0;
  const gs_params* gp[kMaxViews];
  for (int v = 0; v < n_views; ++v) {
    int g = 0;
    while (g < ng && !(gp[g]->means == params[v].means && gp[g]->n == params[v].n &&
                       gp[g]->sh_degree == params[v].sh_degree && gp[g]->sh == params[v].sh))
      ++g;
    if (g == ng) gp[ng++] = &params[v];
    gid[v] = g;
  }
  gs_camera oc[kMaxViews];
  float* oi[kMaxViews];
  int m = 0;
  for (int g = 0; g < ng; ++g)
    for (int v = 0; v < n_views; ++v)
      if (gid[v] == g) {
        order[m] = v;
        oc[m] = cams[v];
        oi[m] = images[v];
        ++m;
      }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  gs_frame* fr = *state;
  const bool fresh = (fr == nullptr);
  if (fresh) {
    fr = new (std::nothrow) gs_frame();
    if (fr == nullptr) {
      set_error("gs_render_fwd_multi: out of host memory");
      return GS_ERR_NOMEM;
    }
    fr->ctx = ctx;
    ctx_retain(ctx);
  } else if (fr->ctx != ctx) {
    set_error("gs_render_fwd_multi: frame belongs to another context");
    return GS_ERR_INVALID;
  }
  Frame& f = *fr;
  f.n = 0;
  f.entries = (int64_t)total;
  f.multi = true;
  f.views = n_views;
  f.tile = tile;
  f.depth = depth;
  f.persistent = (flags & GS_RENDER_PERSISTENT) != 0;
  f.lpt = f.persistent && (flags & GS_RENDER_LONGEST_FIRST) != 0;
  f.tile_order = nullptr;
  f.sh_degree = -1;
  f.K = 0;
  f.keep_radii = false;
  f.screen_kept = false;
  st = build_views(f, oc, n_views, oi, bg);
  if (st == GS_OK) {
    uint32_t base = 0;
    int v = 0;
    f.n_groups = ng;
    for (int g = 0; g < ng; ++g) {
      SceneGroup& sg = f.groups[g];
      sg.pd = params_dev(*gp[g]);
      sg.v0 = v;
      sg.nv = 0;
      sg.base = base;
      while (v < n_views && gid[order[v]] == g) {
        f.vt.v[v].entry_off = base;
        base += (uint32_t)gp[g]->n;
        ++sg.nv;
        ++v;
      }
    }
    st = frame_buffers(f, s);
  }
  if (st != GS_OK) {
    if (fresh) frame_delete(fr);
    return st;
  }
  *state = fr;
  st = forward_stages(ctx, f, f.groups[0].pd, s, 0);
  if (st != GS_OK) return st;
  GS_HIP(hipEventRecord(f.last_use, s));
  return GS_OK;
}

}  // extern "C"

namespace isogs {

// The forward pipeline.  cap == 0: the record count K is read back to the host
// and the record buffers sized to it (one stream synchronisation).  cap > 0:
// no host synchronisation — K stays on the device (clamped to cap, with the
// overflow word set when the records do not fit), as a captured graph needs.
gs_status forward_stages(Ctx* ctx, Frame& f, const ParamsDev& pd, hipStream_t s, uint32_t cap) {
  gs_status st = GS_OK;
  const uint32_t vn = (uint32_t)f.entries;

  // 1. projection + SH (a multi-scene frame: one launch per scene, each on its
  // views' entry range)
  {
    StageTimer tm(ctx, ST_PROJECT, s);
    if (!f.multi) {
      st = launch_preprocess_fwd(pd, f.vt, f, s);
    } else {
      for (int g = 0; g < f.n_groups && st == GS_OK; ++g) {
        const SceneGroup& sg = f.groups[g];
        ViewTable vg = f.vt;
        vg.n = sg.nv;
        for (int k = 0; k < sg.nv; ++k) vg.v[k] = f.vt.v[sg.v0 + k];
        st = launch_preprocess_fwd(sg.pd, vg, f, s, sg.base);
      }
    }
  }
  if (st != GS_OK) return st;
  // 2. (view, Gaussian) entries in (depth bits, index) order
  int in_b = 0;
  {
    StageTimer tm(ctx, ST_DEPTH_SORT, s);
    st = sort_pairs_u32(ctx, f.ss, (const uint32_t*)f.dkey.p, nullptr, (uint32_t*)f.dkw[0].p,
                        (uint32_t*)f.sidx[0].p, (uint32_t*)f.dkw[1].p, (uint32_t*)f.sidx[1].p,
                        vn, nullptr, 32, &in_b, s);
  }
  if (st != GS_OK) return st;
  uint32_t* words = (uint32_t*)f.words.p;
  st = launch_visible_count(f.ss, vn, words + kWordVisible, s);
  if (st != GS_OK) return st;
  f.sidx_sel = in_b;
  const uint32_t* sidx = (const uint32_t*)f.sidx[in_b].p;
  // 3. record offsets and the total K; the depth sort's key buffers are free now
  // and take the rectangles in depth order (x0|y0 words, x1|y1 words)
  uint64_t* d_total = (uint64_t*)(words + kWordTotal);
  uint32_t* srx = (uint32_t*)f.dkw[0].p;
  uint32_t* sry = (uint32_t*)f.dkw[1].p;
  {
    StageTimer tm(ctx, ST_SCAN, s);
    st = scan_tile_counts(ctx, f.ss, sidx, (const uint2*)f.rect.p, vn, (uint32_t*)f.offs.p, srx,
                          sry, d_total, s);
  }
  if (st != GS_OK) return st;
  uint32_t n_rec = 0;              // host bound on the record count (grid sizes)
  const uint32_t* d_K = nullptr;   // device record count (device-count pipelines)
  uint32_t* overflow = nullptr;
  if (cap == 0) {
    // words 8..11: the record total and the visible count, in one readback
    GS_HIP(hipMemcpyAsync(f.pinned, d_total, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    GS_HIP(hipStreamSynchronize(s));
    const uint64_t K = f.pinned[0];
    f.visible = (int64_t)(uint32_t)f.pinned[1];
    if (K > kMaxRecords) {
      set_error("gs_render_fwd: %llu (Gaussian, tile) records exceed the limit of %llu",
                (unsigned long long)K, (unsigned long long)kMaxRecords);
      return GS_ERR_CAPACITY;
    }
    f.K = (int64_t)K;
    n_rec = (uint32_t)K;
    for (int k = 0; k < 2; ++k) {
      st = buf_ensure(ctx, f.tkey[k], (size_t)(K + 1) * 4, s, f.last_use);
      if (st == GS_OK) st = buf_ensure(ctx, f.tval[k], (size_t)(K + 1) * 4, s, f.last_use);
      if (st != GS_OK) return st;
    }
  } else {
    f.K = cap;
    n_rec = cap;
    d_K = words + kWordK;
    overflow = words + kWordOverflow;
    st = launch_clamp_count(d_total, cap, words + kWordK, overflow, s);
    if (st != GS_OK) return st;
  }
  // 4. records in depth order, then the stable sort on the tile digits
  {
    StageTimer tm(ctx, ST_EMIT, s);
    st = launch_emit(f.vt, f, sidx, srx, sry, vn, overflow, s);
  }
  if (st != GS_OK) return st;
  {
    StageTimer tm(ctx, ST_TILE_SORT, s);
    st = sort_pairs_u32(ctx, f.ss, (const uint32_t*)f.tkey[0].p, (const uint32_t*)f.tval[0].p,
                        (uint32_t*)f.tkey[1].p, (uint32_t*)f.tval[1].p, (uint32_t*)f.tkey[0].p,
                        (uint32_t*)f.tval[0].p, n_rec, d_K, f.key_bits, &in_b, s);
  }
  if (st != GS_OK) return st;
  f.tkey_sel = (n_rec == 0) ? 0 : (in_b ? 0 : 1);
  // 5. per-tile ranges, 6. compositing
  {
    StageTimer tm(ctx, ST_RANGES, s);
    st = launch_ranges(f, n_rec, d_K, s);
    if (st == GS_OK && f.lpt) st = launch_tile_order(f, s);
    // persistent work queues start empty
    if (st == GS_OK && f.persistent) st = launch_fill_u32(f.words.p, 0u, 2, s);
  }
  if (st != GS_OK) return st;
  StageTimer tm(ctx, ST_BLEND_FWD, s);
  return launch_blend_fwd(f.vt, f, s);
}

// The backward pipeline: reverse traversal, then the chain rule to the parameters.
gs_status backward_stages(Ctx* ctx, Frame& f, const ParamsDev& pd, const GradsDev& g,
                          hipStream_t s) {
  gs_status st = GS_OK;
  if (f.K > 0) {
    if (f.persistent) {
      st = launch_fill_u32((uint32_t*)f.words.p + kWordBwdCounter, 0u, 1, s);
      if (st != GS_OK) return st;
    }
    StageTimer tm(ctx, ST_BLEND_BWD, s);
    st = launch_blend_bwd(f.vt, f, s);
  }
  if (st != GS_OK) return st;
  StageTimer tm(ctx, ST_PROJECT_BWD, s);
  return launch_preprocess_bwd(pd, f.vt, f, g, s);
}

// Arguments shared by gs_loss_grad and gs_loss_grad_noalloc: checks them and
// fills the view sizes.
static gs_status loss_args(const char* what, gs_ctx* ctx, const float* const* rendered,
                           const float* const* target, const gs_camera* cams, int32_t n_views,
                           float lambda_dssim, int* W, int* H) {
  if (ctx == nullptr || rendered == nullptr || target == nullptr || cams == nullptr) {
    set_error("%s: null argument", what);
    return GS_ERR_INVALID;
  }
  if (n_views < 1 || n_views > kMaxViews) {
    set_error("%s: n_views %d not in [1, %d]", what, n_views, kMaxViews);
    return GS_ERR_INVALID;
  }
  if (!(lambda_dssim >= 0.f && lambda_dssim <= 1.f)) {
    set_error("%s: lambda %g not in [0, 1]", what, (double)lambda_dssim);
    return GS_ERR_INVALID;
  }
  for (int v = 0; v < n_views; ++v) {
    if (!valid_camera(cams[v], v)) return GS_ERR_INVALID;
    if (rendered[v] == nullptr || target[v] == nullptr) {
      set_error("%s: image pointer of view %d is null", what, v);
      return GS_ERR_INVALID;
    }
    W[v] = cams[v].width;
    H[v] = cams[v].height;
  }
  return GS_OK;
}

}  // namespace isogs

extern "C" {

gs_status gs_loss_grad(gs_ctx* ctx, const float* const* rendered, const float* const* target,
                       const gs_camera* cams, int32_t n_views, float lambda_dssim,
                       float* loss_out, float* const* dl_dimg, void* stream) {
  int W[kMaxViews], H[kMaxViews];
  gs_status st = loss_args("gs_loss_grad", ctx, rendered, target, cams, n_views, lambda_dssim,
                           W, H);
  if (st != GS_OK) return st;
  st = set_device(ctx);
  if (st != GS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (ctx->loss_scratch == nullptr) {
    ctx->loss_scratch = new (std::nothrow) LossScratch();
    if (ctx->loss_scratch == nullptr) {
      set_error("gs_loss_grad: out of host memory");
      return GS_ERR_NOMEM;
    }
  }
  LossScratch& ls = *ctx->loss_scratch;
  st = loss_reserve(ctx, ls, W, H, n_views, s);
  if (st != GS_OK) return st;
  {
    StageTimer tm(ctx, ST_LOSS, s);
    st = launch_loss(ls, rendered, target, W, H, n_views, lambda_dssim, loss_out, dl_dimg, s);
  }
  if (st != GS_OK) return st;
  GS_HIP(hipEventRecord(ls.last_use, s));
  return GS_OK;
}

gs_status gs_image_metrics(gs_ctx* ctx, const float* const* rendered,
                           const float* const* reference, const gs_camera* cams,
                           int32_t n_views, float* out, void* stream) {
  int W[kMaxViews], H[kMaxViews];
  gs_status st = loss_args("gs_image_metrics", ctx, rendered, reference, cams, n_views, 0.5f,
                           W, H);
  if (st != GS_OK) return st;
  if (out == nullptr) {
    set_error("gs_image_metrics: out is null");
    return GS_ERR_INVALID;
  }
  st = set_device(ctx);
  if (st != GS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (ctx->loss_scratch == nullptr) {
    ctx->loss_scratch = new (std::nothrow) LossScratch();
    if (ctx->loss_scratch == nullptr) {
      set_error("gs_image_metrics: out of host memory");
      return GS_ERR_NOMEM;
    }
  }
  LossScratch& ls = *ctx->loss_scratch;
  st = loss_reserve(ctx, ls, W, H, n_views, s);
  if (st != GS_OK) return st;
  st = launch_metrics(ls, rendered, reference, W, H, n_views, out, s);
  if (st != GS_OK) return st;
  GS_HIP(hipEventRecord(ls.last_use, s));
  return GS_OK;
}

gs_status gs_loss_grad_noalloc(gs_ctx* ctx, const float* const* rendered,
                               const float* const* target, const gs_camera* cams,
                               int32_t n_views, float lambda_dssim, float* loss_out,
                               float* const* dl_dimg, void* stream) {
  int W[kMaxViews], H[kMaxViews];
  gs_status st = loss_args("gs_loss_grad_noalloc", ctx, rendered, target, cams, n_views,
                           lambda_dssim, W, H);
  if (st != GS_OK) return st;
  LossScratch ws;
  st = loss_noalloc_workspace(ctx->device, W, H, n_views, &ws);
  if (st != GS_OK) return st;
  st = set_device(ctx);
  if (st != GS_OK) return st;
  // the same kernels as gs_loss_grad; no stage timing (its events may be created here)
  return launch_loss(ws, rendered, target, W, H, n_views, lambda_dssim, loss_out, dl_dimg,
                     (hipStream_t)stream);
}

gs_status gs_render_bwd(gs_ctx* ctx, gs_frame* frame, gs_params params,
                        const float* const* dl_dimg, gs_params grads, int32_t flags,
                        void* stream) {
  if (ctx == nullptr || frame == nullptr || dl_dimg == nullptr) {
    set_error("gs_render_bwd: null argument");
    return GS_ERR_INVALID;
  }
  if (frame->ctx != ctx) {
    set_error("gs_render_bwd: frame belongs to another context");
    return GS_ERR_INVALID;
  }
  if (!valid_params(params, "gs_render_bwd (params)") ||
      !valid_params(grads, "gs_render_bwd (grads)"))
    return GS_ERR_INVALID;
  if (params.n != frame->n || grads.n != frame->n || params.sh_degree != frame->sh_degree ||
      grads.sh_degree != frame->sh_degree) {
    set_error("gs_render_bwd: parameter shapes differ from the frame's forward pass");
    return GS_ERR_INVALID;
  }
  if ((flags & ~(GS_BWD_ACCUMULATE | GS_BWD_KEEP_SCREEN)) != 0) {
    set_error("gs_render_bwd: unknown flags 0x%x", flags);
    return GS_ERR_INVALID;
  }
  Frame& f = *frame;
  if (f.multi) {
    set_error("gs_render_bwd: the frame holds views of several scenes (forward only)");
    return GS_ERR_UNSUPPORTED;
  }
  if (!f.acc_zeroed) {
    set_error("gs_render_bwd: the frame's screen-space sums were kept by the previous backward; "
              "run a forward first");
    return GS_ERR_INVALID;
  }
  for (int v = 0; v < f.views; ++v) {
    if (dl_dimg[v] == nullptr) {
      set_error("gs_render_bwd: dl_dimg[%d] is null", v);
      return GS_ERR_INVALID;
    }
    f.vt.v[v].dimg = dl_dimg[v];
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const GradsDev gd = grads_dev(grads, flags);
  st = backward_stages(ctx, f, params_dev(params), gd, s);
  if (st != GS_OK) return st;
  // kept sums are cleared by the next forward
  if (gd.keep_screen) {
    f.acc_zeroed = false;
    f.screen_kept = true;
  }
  GS_HIP(hipEventRecord(f.last_use, s));
  return GS_OK;
}

gs_status gs_density_accumulate(gs_ctx* ctx, gs_frame* frame, gs_density_stats stats,
                                float scale, void* stream) {
  if (ctx == nullptr || frame == nullptr) {
    set_error("gs_density_accumulate: null argument");
    return GS_ERR_INVALID;
  }
  if (frame->ctx != ctx) {
    set_error("gs_density_accumulate: frame belongs to another context");
    return GS_ERR_INVALID;
  }
  if (stats.grad == nullptr || stats.count == nullptr || stats.max_radius == nullptr) {
    set_error("gs_density_accumulate: null statistics array");
    return GS_ERR_INVALID;
  }
  Frame& f = *frame;
  if (f.multi) {
    set_error("gs_density_accumulate: the frame holds views of several scenes");
    return GS_ERR_UNSUPPORTED;
  }
  if (stats.n != f.n) {
    set_error("gs_density_accumulate: statistics hold %lld entries, the frame %lld",
              (long long)stats.n, (long long)f.n);
    return GS_ERR_INVALID;
  }
  if (!f.keep_radii || !f.screen_kept) {
    set_error("gs_density_accumulate: the frame needs a forward with GS_RENDER_RADII and a "
              "backward with GS_BWD_KEEP_SCREEN");
    return GS_ERR_INVALID;
  }
  if (!(scale >= 0.f)) {
    set_error("gs_density_accumulate: scale %g < 0", (double)scale);
    return GS_ERR_INVALID;
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  st = launch_density_accumulate(f, stats, scale, s);
  if (st != GS_OK) return st;
  GS_HIP(hipEventRecord(f.last_use, s));
  return GS_OK;
}

static bool same_shape(const gs_params& a, const gs_params& b) {
  return a.n == b.n && a.sh_degree == b.sh_degree;
}

static bool overlaps(const gs_params& a, const gs_params& b) {
  const int ra = 11 + (a.sh_degree + 1) * (a.sh_degree + 1) * 3;
  const int rb = 11 + (b.sh_degree + 1) * (b.sh_degree + 1) * 3;
  const float* pa[5] = {a.means, a.log_scales, a.quats, a.opacity_logits, a.sh};
  const float* pb[5] = {b.means, b.log_scales, b.quats, b.opacity_logits, b.sh};
  const int na[5] = {3, 3, 4, 1, ra - 11}, nb[5] = {3, 3, 4, 1, rb - 11};
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      const char* a0 = (const char*)pa[i];
      const char* a1 = a0 + sizeof(float) * (size_t)na[i] * (size_t)a.n;
      const char* b0 = (const char*)pb[j];
      const char* b1 = b0 + sizeof(float) * (size_t)nb[j] * (size_t)b.n;
      if (a0 < b1 && b0 < a1) return true;
    }
  return false;
}

gs_status gs_densify(gs_ctx* ctx, gs_params p, gs_params m, gs_params v, gs_density_stats stats,
                     const gs_density_opts* opts, gs_params p_out, gs_params m_out,
                     gs_params v_out, int32_t* src_index, gs_density_info* info, void* stream) {
  if (ctx == nullptr || opts == nullptr || info == nullptr) {
    set_error("gs_densify: null argument");
    return GS_ERR_INVALID;
  }
  if (!valid_params(p, "gs_densify (p)") || !valid_params(m, "gs_densify (m)") ||
      !valid_params(v, "gs_densify (v)"))
    return GS_ERR_INVALID;
  if (!same_shape(p, m) || !same_shape(p, v)) {
    set_error("gs_densify: p, m, v shapes differ");
    return GS_ERR_INVALID;
  }
  if (p.n > 0x7fffffffLL) {
    set_error("gs_densify: n %lld exceeds 2^31 - 1", (long long)p.n);
    return GS_ERR_CAPACITY;
  }
  if (stats.grad == nullptr || stats.count == nullptr || stats.max_radius == nullptr ||
      stats.n != p.n) {
    set_error("gs_densify: statistics must be three arrays of n = %lld entries",
              (long long)p.n);
    return GS_ERR_INVALID;
  }
  const gs_density_opts& o = *opts;
  if (o.n_split < 1 || o.n_split > 8 || !(o.split_div > 0.0) || !(o.extent > 0.0) ||
      !(o.grad_threshold >= 0.0) || !(o.percent_dense >= 0.0) || !(o.max_world >= 0.0) ||
      !(o.min_opacity >= 0.0) || o.max_screen != o.max_screen) {
    set_error("gs_densify: invalid options (n_split 1..8, split_div > 0, extent > 0, "
              "thresholds >= 0)");
    return GS_ERR_INVALID;
  }
  const bool write = p_out.means != nullptr;
  if (write) {
    if (!valid_params(p_out, "gs_densify (p_out)") || !valid_params(m_out, "gs_densify (m_out)") ||
        !valid_params(v_out, "gs_densify (v_out)"))
      return GS_ERR_INVALID;
    if (p_out.sh_degree != p.sh_degree || m_out.sh_degree != p.sh_degree ||
        v_out.sh_degree != p.sh_degree) {
      set_error("gs_densify: output SH degree differs from the input's");
      return GS_ERR_INVALID;
    }
    const gs_params ins[3] = {p, m, v}, outs[3] = {p_out, m_out, v_out};
    for (const gs_params& a : outs)
      for (const gs_params& b : ins)
        if (overlaps(a, b)) {
          set_error("gs_densify: an output array overlaps an input array");
          return GS_ERR_INVALID;
        }
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  StageTimer tm(ctx, ST_DENSIFY, (hipStream_t)stream);
  return densify_run(ctx, p, m, v, stats, o, write ? &p_out : nullptr, write ? &m_out : nullptr,
                     write ? &v_out : nullptr, src_index, info, (hipStream_t)stream);
}

static bool valid_volume(const gs_volume& v, const char* what) {
  if (v.values == nullptr) {
    set_error("%s: volume values are null", what);
    return false;
  }
  if (v.nx < 2 || v.ny < 2 || v.nz < 2 || v.nx > (1 << 20) || v.ny > (1 << 20) ||
      v.nz > (1 << 20) || (double)v.nx * v.ny * v.nz > 1.2e11) {
    set_error("%s: volume of %lld x %lld x %lld vertices (each side 2 .. 2^20)", what,
              (long long)v.nx, (long long)v.ny, (long long)v.nz);
    return false;
  }
  for (int a = 0; a < 3; ++a)
    if (!(v.hi[a] > v.lo[a])) {
      set_error("%s: empty volume box along axis %d", what, a);
      return false;
    }
  return true;
}

gs_status gs_iso_extract(gs_ctx* ctx, gs_volume vol, float iso, float keep_prob, uint64_t seed,
                         float* xyz, int64_t capacity, int64_t* n_points, void* stream) {
  if (ctx == nullptr || n_points == nullptr) {
    set_error("gs_iso_extract: null argument");
    return GS_ERR_INVALID;
  }
  if (!valid_volume(vol, "gs_iso_extract")) return GS_ERR_INVALID;
  if (!(keep_prob >= 0.f && keep_prob <= 1.f) || !(iso == iso)) {
    set_error("gs_iso_extract: keep_prob %g not in [0, 1] or iso is NaN", (double)keep_prob);
    return GS_ERR_INVALID;
  }
  if (xyz != nullptr && capacity < 1) {
    set_error("gs_iso_extract: capacity %lld < 1", (long long)capacity);
    return GS_ERR_INVALID;
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  return iso_extract_run(ctx, vol, iso, keep_prob, seed, xyz, capacity, n_points,
                         (hipStream_t)stream);
}

gs_status gs_raycast(gs_ctx* ctx, gs_volume vol, float iso, const gs_camera* cams,
                     int32_t n_views, float step, float* const* images, void* stream) {
  if (ctx == nullptr || cams == nullptr || images == nullptr) {
    set_error("gs_raycast: null argument");
    return GS_ERR_INVALID;
  }
  if (!valid_volume(vol, "gs_raycast")) return GS_ERR_INVALID;
  if (n_views < 1 || n_views > kMaxViews) {
    set_error("gs_raycast: n_views %d not in [1, %d]", n_views, kMaxViews);
    return GS_ERR_INVALID;
  }
  double diag = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double e = (double)vol.hi[a] - (double)vol.lo[a];
    diag += e * e;
  }
  diag = std::sqrt(diag);
  if (!(step > 0.f) || diag / (double)step > 1e5) {
    set_error("gs_raycast: step %g must be positive and at least 1e-5 of the box diagonal",
              (double)step);
    return GS_ERR_INVALID;
  }
  for (int v = 0; v < n_views; ++v) {
    if (!valid_camera(cams[v], v)) return GS_ERR_INVALID;
    if (images[v] == nullptr) {
      set_error("gs_raycast: images[%d] is null", v);
      return GS_ERR_INVALID;
    }
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  return launch_raycast(vol, iso, cams, n_views, images, (double)step, (hipStream_t)stream);
}

gs_status gs_opacity_reset(gs_ctx* ctx, gs_params p, gs_params m, gs_params v,
                           double max_opacity, void* stream) {
  if (ctx == nullptr) {
    set_error("gs_opacity_reset: null context");
    return GS_ERR_INVALID;
  }
  if (!valid_params(p, "gs_opacity_reset (p)") || !valid_params(m, "gs_opacity_reset (m)") ||
      !valid_params(v, "gs_opacity_reset (v)"))
    return GS_ERR_INVALID;
  if (!same_shape(p, m) || !same_shape(p, v)) {
    set_error("gs_opacity_reset: p, m, v shapes differ");
    return GS_ERR_INVALID;
  }
  if (!(max_opacity > 0.0 && max_opacity < 1.0)) {
    set_error("gs_opacity_reset: max_opacity %g not in (0, 1)", max_opacity);
    return GS_ERR_INVALID;
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  return launch_opacity_reset(p, m, v, max_opacity, (hipStream_t)stream);
}

gs_status gs_adam_step(gs_ctx* ctx, gs_params p, gs_params g, gs_params m, gs_params v,
                       const gs_adam_opts* opts, int64_t step, void* stream) {
  if (ctx == nullptr || opts == nullptr) {
    set_error("gs_adam_step: null argument");
    return GS_ERR_INVALID;
  }
  if (!valid_params(p, "gs_adam_step (p)") || !valid_params(g, "gs_adam_step (g)") ||
      !valid_params(m, "gs_adam_step (m)") || !valid_params(v, "gs_adam_step (v)"))
    return GS_ERR_INVALID;
  if (g.n != p.n || m.n != p.n || v.n != p.n || g.sh_degree != p.sh_degree ||
      m.sh_degree != p.sh_degree || v.sh_degree != p.sh_degree) {
    set_error("gs_adam_step: p, g, m, v shapes differ");
    return GS_ERR_INVALID;
  }
  if (step < 1) {
    set_error("gs_adam_step: step %lld < 1", (long long)step);
    return GS_ERR_INVALID;
  }
  if (!(opts->beta1 >= 0.f && opts->beta1 < 1.f && opts->beta2 >= 0.f && opts->beta2 < 1.f)) {
    set_error("gs_adam_step: betas must lie in [0, 1)");
    return GS_ERR_INVALID;
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  StageTimer tm(ctx, ST_ADAM, (hipStream_t)stream);
  return launch_adam(p, g, m, v, *opts, step, (hipStream_t)stream);
}

gs_status gs_bw_probe(gs_ctx* ctx, const void* src, void* dst, size_t bytes, void* stream) {
  if (ctx == nullptr || src == nullptr || dst == nullptr || bytes % 16 != 0 ||
      ((uintptr_t)src & 15u) != 0 || ((uintptr_t)dst & 15u) != 0) {
    set_error("gs_bw_probe: null pointer, or size / address not a multiple of 16");
    return GS_ERR_INVALID;
  }
  gs_status st = set_device(ctx);
  if (st != GS_OK) return st;
  StageTimer tm(ctx, ST_PROBE, (hipStream_t)stream);
  return launch_copy_probe(ctx, src, dst, bytes, (hipStream_t)stream);
}

gs_status gs_frame_stats_get(gs_frame* frame, gs_frame_stats* out) {
  if (frame == nullptr || out == nullptr) {
    set_error("gs_frame_stats_get: null argument");
    return GS_ERR_INVALID;
  }
  out->n_views = frame->views;
  out->tile = frame->tile;
  out->n_gaussians = frame->n;
  out->n_records = frame->K;
  out->n_visible = frame->visible;
  out->n_tiles = frame->vt.total_tiles;
  out->n_pixels = frame->total_pix;
  out->device_bytes = (int64_t)frame->bytes();
  return GS_OK;
}

gs_status gs_frame_export(gs_frame* frame, int32_t what, int32_t view, void* dst, size_t bytes,
                          void* stream) {
  if (frame == nullptr || dst == nullptr) {
    set_error("gs_frame_export: null argument");
    return GS_ERR_INVALID;
  }
  Frame& f = *frame;
  if (view < -1 || view >= f.views) {
    set_error("gs_frame_export: view %d out of range", view);
    return GS_ERR_INVALID;
  }
  if (f.multi && what != GS_EXPORT_KEYS && what != GS_EXPORT_VALUES && what != GS_EXPORT_RANGES &&
      what != GS_EXPORT_FINAL_T && what != GS_EXPORT_N_CONTRIB) {
    set_error("gs_frame_export: per-(view, Gaussian) arrays of a multi-scene frame are not "
              "exported");
    return GS_ERR_UNSUPPORTED;
  }
  gs_status st = set_device(f.ctx);
  if (st != GS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const size_t n = (size_t)f.n;
  size_t need = 0, off = 0;
  const void* src = nullptr;
  switch (what) {
    case GS_EXPORT_KEYS:
      need = (size_t)f.K * 8;
      if (view != -1) break;
      if (bytes < need) break;
      st = launch_export_keys(f, (uint64_t*)dst, s);
      if (st == GS_OK) GS_HIP(hipEventRecord(f.last_use, s));
      return st;
    case GS_EXPORT_VALUES:
      need = (size_t)f.K * 4;
      src = f.tval[f.tkey_sel].p;
      if (view != -1) need = 0;
      break;
    case GS_EXPORT_RANGES:
      need = (size_t)f.vt.total_tiles * 8;
      src = f.ranges.p;
      if (view >= 0) {
        const CamDev& c = f.vt.v[view];
        off = (size_t)c.tile_offset * 8;
        need = (size_t)c.tiles_x * c.tiles_y * 8;
      }
      break;
    case GS_EXPORT_FINAL_T:
    case GS_EXPORT_N_CONTRIB:
      src = (what == GS_EXPORT_FINAL_T) ? f.finalT.p : f.ncon.p;
      need = (size_t)f.total_pix * 4;
      if (view >= 0) {
        const CamDev& c = f.vt.v[view];
        off = (size_t)c.pix_offset * 4;
        need = (size_t)c.W * c.H * 4;
      }
      break;
    case GS_EXPORT_SCREEN_GRADS:
      // interleaved from the geometric and colour accumulators by a kernel
      need = (size_t)(view >= 0 ? 1 : f.views) * 12 * n * 4;
      if (bytes < need) break;
      if (((uintptr_t)dst & 15u) != 0) {
        set_error("gs_frame_export: screen gradients need a 16-byte aligned destination");
        return GS_ERR_INVALID;
      }
      st = launch_export_screen_grads(f, view, (float*)dst, s);
      if (st == GS_OK) GS_HIP(hipEventRecord(f.last_use, s));
      return st;
    case GS_EXPORT_SPLATS:
      src = f.splat.p;
      need = (size_t)f.views * n * 48;
      if (view >= 0) {
        off = (size_t)view * n * 48;
        need = n * 48;
      }
      break;
    case GS_EXPORT_RECTS:
      // stored packed as uint2; unpacked to 4 x u32 on the host side of the copy
      src = f.rect.p;
      need = (size_t)f.views * n * 8;
      if (view >= 0) {
        off = (size_t)view * n * 8;
        need = n * 8;
      }
      break;
    case GS_EXPORT_DEPTHS:
      src = f.dkey.p;
      need = (size_t)f.views * n * 4;
      if (view >= 0) {
        off = (size_t)view * n * 4;
        need = n * 4;
      }
      break;
    default:
      set_error("gs_frame_export: unknown export %d", what);
      return GS_ERR_INVALID;
  }
  if (src == nullptr || need == 0 || bytes < need) {
    set_error("gs_frame_export: export %d of view %d needs %zu bytes (have %zu)", what, view, need,
              bytes);
    return GS_ERR_INVALID;
  }
  GS_HIP(hipMemcpyAsync(dst, (const char*)src + off, need, hipMemcpyDeviceToDevice, s));
  GS_HIP(hipEventRecord(f.last_use, s));
  return GS_OK;
}

void gs_frame_release(gs_frame* frame) {
  if (frame == nullptr) return;
  (void)hipSetDevice(frame->ctx->device);
  // every call that enqueues work on the frame's buffers records last_use after it
  if (frame->last_use != nullptr)
    (void)hipEventSynchronize(frame->last_use);
  else
    (void)hipDeviceSynchronize();
  frame_delete(frame);
}

}  // extern "C"
