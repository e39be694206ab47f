// Batched training step captured in a hipGraph, and the render autotuner.
//
// The graph holds one whole step for a set of views: projection, depth sort,
// scan, emission, tile sort, ranges, (tile order), blending, loss gradient,
// reverse traversal, parameter chain rule and Adam.  Nothing in it waits on
// the host: the record count K stays on the device and is clamped to a
// preallocated capacity; if the records outgrow it, the emission sets an
// overflow word, Adam and the step counter skip that launch, and the host
// (after the replay) grows the capacity, recaptures and replays the step.
// Adam's bias corrections come from a device step counter advanced by the
// graph itself, so replays need no new kernel arguments.
#include <algorithm>
#include <cmath>
#include <new>

#include "internal.h"

using namespace isogs;

struct gs_graph {
  Ctx* ctx = nullptr;
  gs_frame* frame = nullptr;
  gs_step_desc desc;
  int nv = 0;
  gs_camera cams[kMaxViews];
  float* images[kMaxViews];
  const float* targets[kMaxViews];
  float* dl[kMaxViews];
  int W[kMaxViews], H[kMaxViews];
  uint32_t cap = 0;
  double slack = 1.25;
  hipStream_t cstream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t* pinned = nullptr;  // copy of the frame's device words after a replay
  int64_t records = 0;
  // the graph's own loss workspace: captured kernels hold its pointers, so it
  // is sized before capture and never shared with eager calls or other graphs
  LossScratch loss;
  hipEvent_t done = nullptr;   // recorded after every replay
};

namespace isogs {
namespace {

// Start of a step: clear the overflow word, bias corrections of the coming step.
__global__ void k_step_prep(uint32_t* words, float b1, float b2) {
  words[kWordOverflow] = 0u;
  const long long t = *reinterpret_cast<const long long*>(words + kWordStep);
  float* bc = reinterpret_cast<float*>(words + kWordBC);
  bc[0] = (float)(1.0 / (1.0 - pow((double)b1, (double)t)));
  bc[1] = (float)(1.0 / sqrt(1.0 - pow((double)b2, (double)t)));
}

// End of a step: advance the Adam step unless the records overflowed.
__global__ void k_step_commit(uint32_t* words) {
  if (words[kWordOverflow] == 0u) *reinterpret_cast<long long*>(words + kWordStep) += 1;
}

gs_status enqueue_step(gs_graph* g, hipStream_t s) {
  Ctx* ctx = g->ctx;
  Frame& f = *g->frame;
  const gs_step_desc& d = g->desc;
  uint32_t* words = (uint32_t*)f.words.p;
  hipLaunchKernelGGL(k_step_prep, dim3(1), dim3(1), 0, s, words, d.adam.beta1, d.adam.beta2);
  GS_LAUNCHED("step_prep");
  // the forward writes into the step's images
  for (int v = 0; v < g->nv; ++v) f.vt.v[v].image = g->images[v];
  gs_status st = forward_stages(ctx, f, params_dev(d.params), s, g->cap);
  if (st != GS_OK) return st;
  st = launch_loss(g->loss, g->images, g->targets, g->W, g->H, g->nv, d.lambda_dssim, d.loss,
                   g->dl, s);
  if (st != GS_OK) return st;
  for (int v = 0; v < g->nv; ++v) f.vt.v[v].dimg = g->dl[v];
  st = backward_stages(ctx, f, params_dev(d.params), grads_dev(d.grads, 0), s);
  if (st != GS_OK) return st;
  if (d.with_adam) {
    st = launch_adam(d.params, d.grads, d.adam_m, d.adam_v, d.adam, 1, s,
                     reinterpret_cast<const float*>(words + kWordBC), words + kWordOverflow);
    if (st != GS_OK) return st;
    hipLaunchKernelGGL(k_step_commit, dim3(1), dim3(1), 0, s, words);
    GS_LAUNCHED("step_commit");
  }
  return GS_OK;
}

void drop_graph(gs_graph* g) {
  if (g->exec != nullptr) (void)hipGraphExecDestroy(g->exec);
  if (g->graph != nullptr) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
}

// Size the record buffers and sort scratch for the capacity, then capture.
// Buffers are replaced only after the last replay (event `done`), the frame's
// last eager use and the capture stream have finished with them.
gs_status reserve_and_capture(gs_graph* g) {
  Ctx* ctx = g->ctx;
  Frame& f = *g->frame;
  GS_HIP(hipEventSynchronize(g->done));
  const hipStream_t cs = g->cstream;
  for (int k = 0; k < 2; ++k) {
    gs_status st = buf_ensure(ctx, f.tkey[k], ((size_t)g->cap + 1) * 4, cs, f.last_use);
    if (st == GS_OK) st = buf_ensure(ctx, f.tval[k], ((size_t)g->cap + 1) * 4, cs, f.last_use);
    if (st != GS_OK) return st;
  }
  const uint32_t vn = (uint32_t)f.entries;
  const uint32_t most = std::max(std::max(g->cap, vn), (uint32_t)f.vt.total_tiles);
  gs_status st = sort_reserve(ctx, f.ss, most, cs);
  if (st == GS_OK) st = loss_reserve(ctx, g->loss, g->W, g->H, g->nv, cs);
  if (st != GS_OK) return st;
  GS_HIP(hipStreamSynchronize(cs));
  drop_graph(g);
  ctx->capturing = true;
  hipError_t e = hipStreamBeginCapture(g->cstream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    ctx->capturing = false;
    return hip_fail(e, "hipStreamBeginCapture");
  }
  st = enqueue_step(g, g->cstream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(g->cstream, &graph);
  ctx->capturing = false;
  if (st != GS_OK) {
    if (graph != nullptr) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  g->graph = graph;
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  return GS_OK;
}

uint32_t capacity_for(uint64_t K, double slack) {
  const double c = std::max((double)K * slack, (double)K + 65536.0);
  return (uint32_t)std::min(c, (double)kMaxRecords);
}

}  // namespace
}  // namespace isogs

extern "C" {

gs_status gs_step_graph_create(gs_ctx* ctx, const gs_step_desc* desc, gs_graph** out,
                               void* stream) {
  if (ctx == nullptr || desc == nullptr || out == nullptr || desc->cams == nullptr ||
      desc->images == nullptr || desc->targets == nullptr || desc->dl_dimg == nullptr ||
      desc->loss == nullptr) {
    set_error("gs_step_graph_create: null argument");
    return GS_ERR_INVALID;
  }
  *out = nullptr;
  if (desc->n_views < 1 || desc->n_views > kMaxViews) {
    set_error("gs_step_graph_create: n_views %d not in [1, %d]", desc->n_views, kMaxViews);
    return GS_ERR_INVALID;
  }
  if (desc->with_adam && desc->first_step < 1) {
    set_error("gs_step_graph_create: first_step must be >= 1");
    return GS_ERR_INVALID;
  }
  gs_graph* g = new (std::nothrow) gs_graph();
  if (g == nullptr) {
    set_error("gs_step_graph_create: out of host memory");
    return GS_ERR_NOMEM;
  }
  g->ctx = ctx;
  ctx_retain(ctx);
  g->desc = *desc;
  g->nv = desc->n_views;
  g->slack = desc->capacity_slack >= 1.05 ? desc->capacity_slack : 1.25;
  for (int v = 0; v < g->nv; ++v) {
    g->cams[v] = desc->cams[v];
    g->images[v] = desc->images[v];
    g->targets[v] = desc->targets[v];
    g->dl[v] = desc->dl_dimg[v];
    g->W[v] = desc->cams[v].width;
    g->H[v] = desc->cams[v].height;
  }
  g->desc.cams = g->cams;
  hipStream_t s = (hipStream_t)stream;
  gs_status st = GS_OK;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->cstream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipHostMalloc((void**)&g->pinned, kWordCount * 4, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(g->done, g->cstream);
  if (e != hipSuccess) st = hip_fail(e, "gs_step_graph_create");
  // eager measuring pass: sizes every buffer and measures K
  if (st == GS_OK)
    st = gs_render_fwd(ctx, desc->params, g->cams, g->nv, g->images, &desc->render, &g->frame, s);
  if (st == GS_OK)
    st = gs_loss_grad(ctx, g->images, g->targets, g->cams, g->nv, desc->lambda_dssim, desc->loss,
                      g->dl, s);
  if (st == GS_OK) st = gs_render_bwd(ctx, g->frame, desc->params, g->dl, desc->grads, 0, s);
  if (st == GS_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
  }
  if (st == GS_OK) {
    g->records = g->frame->K;
    g->cap = capacity_for((uint64_t)g->frame->K, g->slack);
    // the graph's own Adam step counter starts at first_step
    const long long t0 = desc->with_adam ? desc->first_step : 1;
    e = hipMemcpy((uint32_t*)g->frame->words.p + kWordStep, &t0, sizeof(t0),
                  hipMemcpyHostToDevice);
    if (e != hipSuccess) st = hip_fail(e, "hipMemcpy(step)");
  }
  if (st == GS_OK) st = reserve_and_capture(g);
  if (st != GS_OK) {
    gs_step_graph_destroy(g);
    return st;
  }
  *out = g;
  return GS_OK;
}

gs_status gs_step_graph_capture(gs_ctx* ctx, const gs_step_desc* desc, gs_graph** out) {
  return gs_step_graph_create(ctx, desc, out, nullptr);
}

gs_status gs_step_graph_launch(gs_graph* g, void* stream) {
  if (g == nullptr || g->exec == nullptr) {
    set_error("gs_step_graph_launch: no captured graph");
    return GS_ERR_INVALID;
  }
  GS_HIP(hipSetDevice(g->ctx->device));
  hipStream_t s = (hipStream_t)stream;
  GS_HIP(hipGraphLaunch(g->exec, s));
  GS_HIP(hipMemcpyAsync(g->pinned, g->frame->words.p, kWordCount * 4, hipMemcpyDeviceToHost, s));
  GS_HIP(hipEventRecord(g->done, s));
  GS_HIP(hipEventRecord(g->frame->last_use, s));
  return GS_OK;
}

gs_status gs_step_graph_sync(gs_graph* g, int32_t* overflowed, int64_t* records, void* stream) {
  if (g == nullptr) {
    set_error("gs_step_graph_sync: null graph");
    return GS_ERR_INVALID;
  }
  GS_HIP(hipSetDevice(g->ctx->device));
  GS_HIP(hipStreamSynchronize((hipStream_t)stream));
  GS_HIP(hipEventSynchronize(g->done));
  const uint64_t total = *reinterpret_cast<const uint64_t*>(g->pinned + kWordTotal);
  g->frame->K = (int64_t)std::min<uint64_t>(total, g->cap);
  g->frame->visible = (int64_t)g->pinned[kWordVisible];
  const bool over = g->pinned[kWordOverflow] != 0u;
  g->records = (int64_t)total;
  if (records) *records = (int64_t)total;
  if (overflowed) *overflowed = over ? 1 : 0;
  if (over) {
    if (total > kMaxRecords) {
      set_error("gs_step_graph_sync: %llu records exceed the limit of %llu",
                (unsigned long long)total, (unsigned long long)kMaxRecords);
      return GS_ERR_CAPACITY;
    }
    g->cap = capacity_for(total, g->slack);
    return reserve_and_capture(g);
  }
  return GS_OK;
}

gs_status gs_step_graph_run(gs_graph* g, int64_t* records, void* stream) {
  for (int attempt = 0; attempt < 3; ++attempt) {
    gs_status st = gs_step_graph_launch(g, stream);
    if (st != GS_OK) return st;
    int32_t over = 0;
    st = gs_step_graph_sync(g, &over, records, stream);
    if (st != GS_OK) return st;
    if (!over) return GS_OK;
  }
  set_error("gs_step_graph_run: records kept outgrowing the capacity");
  return GS_ERR_CAPACITY;
}

gs_status gs_step_graph_info(gs_graph* g, int64_t* capacity, int64_t* records, gs_frame** frame) {
  if (g == nullptr) {
    set_error("gs_step_graph_info: null graph");
    return GS_ERR_INVALID;
  }
  if (capacity) *capacity = g->cap;
  if (records) *records = g->records;
  if (frame) *frame = g->frame;
  return GS_OK;
}

void gs_step_graph_destroy(gs_graph* g) {
  if (g == nullptr) return;
  (void)hipSetDevice(g->ctx->device);
  (void)hipDeviceSynchronize();
  drop_graph(g);
  if (g->frame != nullptr) gs_frame_release(g->frame);
  loss_scratch_free(g->ctx, g->loss);
  if (g->done != nullptr) (void)hipEventDestroy(g->done);
  if (g->cstream != nullptr) (void)hipStreamDestroy(g->cstream);
  if (g->pinned != nullptr) (void)hipHostFree(g->pinned);
  Ctx* ctx = g->ctx;
  delete g;
  ctx_release(ctx);
}

// ------------------------------------------------------------------ autotune

gs_status gs_autotune(gs_ctx* ctx, gs_params params, const gs_camera* cams, int32_t n_views,
                      int32_t reps, gs_render_opts* best, gs_tune_entry* table,
                      int32_t table_cap, int32_t* table_n, void* stream) {
  if (ctx == nullptr || cams == nullptr || best == nullptr || n_views < 1 ||
      n_views > kMaxViews || reps < 1) {
    set_error("gs_autotune: invalid arguments");
    return GS_ERR_INVALID;
  }
  hipStream_t s = (hipStream_t)stream;
  // scratch: images (also used as the upstream gradient) and parameter gradients
  DevBuf img, grd;
  size_t pix = 0;
  for (int v = 0; v < n_views; ++v) pix += (size_t)cams[v].width * cams[v].height;
  const size_t rows = 14 + (size_t)(params.sh_degree + 1) * (params.sh_degree + 1) * 3;
  gs_status st = buf_ensure(ctx, img, pix * 3 * 4, s);
  if (st == GS_OK) st = buf_ensure(ctx, grd, rows * (size_t)params.n * 4, s);
  if (st != GS_OK) {
    buf_free(ctx, img);
    buf_free(ctx, grd);
    return st;
  }
  float* images[kMaxViews];
  size_t off = 0;
  for (int v = 0; v < n_views; ++v) {
    images[v] = (float*)img.p + off;
    off += (size_t)cams[v].width * cams[v].height * 3;
  }
  const size_t n = (size_t)params.n;
  float* gb = (float*)grd.p;
  gs_params gr = params;
  gr.means = gb;
  gr.log_scales = gb + 3 * n;
  gr.quats = gb + 6 * n;
  gr.opacity_logits = gb + 10 * n;
  gr.sh = gb + 11 * n;
  struct Cfg { int tile, depth, flags; };
  const Cfg cfgs[] = {
      {8, 32, 0},   {8, 64, 0},   {16, 32, 0},  {16, 64, 0},  {16, 128, 0}, {16, 256, 0},
      {32, 32, 0},  {32, 64, 0},  {32, 128, 0}, {32, 256, 0}, {8, 64, 3},   {16, 64, 3},
      {16, 128, 3}, {16, 256, 3}, {32, 64, 3},  {32, 128, 3}, {32, 256, 3}};
  gs_frame* frame = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    st = hip_fail(hipErrorUnknown, "hipEventCreate");
  float best_ms = 1e30f;
  int count = 0;
  for (const Cfg& c : cfgs) {
    if (st != GS_OK) break;
    gs_render_opts o;
    std::memset(&o, 0, sizeof(o));
    o.tile = c.tile;
    o.lds_depth = c.depth;
    o.flags = c.flags;
    float ms = 0.f;
    for (int r = -1; r < reps && st == GS_OK; ++r) {  // r = -1: warm-up
      if (r == 0) (void)hipEventRecord(a, s);
      st = gs_render_fwd(ctx, params, cams, n_views, images, &o, &frame, s);
      if (st == GS_OK) st = gs_render_bwd(ctx, frame, params, images, gr, 0, s);
    }
    if (st != GS_OK) break;
    (void)hipEventRecord(b, s);
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
      st = hip_fail(hipErrorUnknown, "autotune timing");
      break;
    }
    ms /= (float)reps;
    if (table != nullptr && count < table_cap) {
      table[count].tile = c.tile;
      table[count].lds_depth = c.depth;
      table[count].flags = c.flags;
      table[count].ms = ms;
    }
    ++count;
    if (ms < best_ms) {
      best_ms = ms;
      *best = o;
    }
  }
  if (table_n) *table_n = std::min(count, table_cap);
  if (frame != nullptr) gs_frame_release(frame);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  buf_free(ctx, img);
  buf_free(ctx, grd);
  return st;
}

}  // extern "C"
