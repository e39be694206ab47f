// Render server: resident scenes, continuous batching of novel-view requests,
// memory admission, latency statistics.
//
// Scenes stay on the device (caller-owned parameters).  Requests (scene,
// camera, output image) are queued as they arrive.  Each of n_slots worker
// threads owns a HIP stream and a frame; whenever it is free it takes the
// oldest pending requests, up to max_batch_views of them, of any scenes and
// resolutions, and renders them as one multi-scene forward (one projection
// launch per scene in the batch, one depth sort, one tile sort, one
// compositing launch over all their tiles).
// Before a batch starts, its device scratch is estimated and admitted against
// the server's memory budget together with the scratch the other slots hold;
// a batch that does not fit waits until a running batch completes.  Batches
// run concurrently on different streams, so requests
// arriving while others are on the device are admitted as soon as a slot and
// memory free up.  A request's latency runs from submission to the completion
// of its batch on the device.  The rendered image of a request does not
// depend on the batch it lands in.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

using namespace isogs;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket;
  int scene;
  gs_camera cam;
  float* out;
  Clock::time_point submitted;
};

struct Result {
  bool done = false;
  gs_status status = GS_OK;
  double latency_ms = 0.0;
};

struct Slot {
  hipStream_t stream = nullptr;
  gs_frame* frame = nullptr;
  size_t bytes = 0;     // scratch the slot's frame holds (ledger)
  size_t reserved = 0;  // admitted estimate while a batch runs
};

}  // namespace

struct gs_server {
  gs_ctx* ctx = nullptr;
  gs_server_opts opts;
  std::vector<gs_params> scenes;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> pending;
  std::unordered_map<uint64_t, Result> results;
  std::vector<Slot> slots;
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t next_ticket = 1;
  size_t ledger = 0;  // sum over slots of max(bytes, reserved)
  // statistics since the last reset
  std::vector<double> latencies;
  int64_t submitted = 0, completed = 0, batches = 0, batch_views = 0, deferred = 0;
  double pixels = 0.0;
  Clock::time_point first_submit, last_done;
  bool have_first = false;
  size_t peak_ledger = 0;
  int in_flight = 0;
};

namespace {

// Scratch a forward of these views is expected to need (vn: the sum over the
// views of their scenes' Gaussian counts).
size_t estimate_bytes(size_t vn, const std::vector<Request>& b) {
  size_t pix = 0;
  for (const Request& r : b) pix += (size_t)r.cam.width * r.cam.height;
  // per (view, Gaussian): splat 48, rect 8, keys/indices 20, clamp 1, scan 4;
  // records: about 4 per visible Gaussian, 16 bytes each; per pixel: T and count
  return vn * 81 + vn * 4 * 16 + pix * 8 + ((size_t)64 << 20);
}

void worker_main(gs_server* sv, int slot_id) {
  Slot& slot = sv->slots[slot_id];
  (void)hipSetDevice(sv->ctx->device);
  for (;;) {
    std::vector<Request> batch;
    gs_params view_params[kMaxViews];  // copied under the lock: add_scene may grow the vector
    size_t need = 0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      for (;;) {
        if (sv->stop) return;
        if (!sv->pending.empty()) {
          std::vector<Request> cand;
          size_t vn = 0;
          for (const Request& r : sv->pending) {
            cand.push_back(r);
            vn += (size_t)sv->scenes[r.scene].n;
            if ((int)cand.size() >= sv->opts.max_batch_views) break;
          }
          need = estimate_bytes(vn, cand);
          const size_t held = std::max(slot.bytes, slot.reserved);
          const size_t others = sv->ledger - held;
          const bool fits = sv->opts.mem_budget == 0 ||
                            others + std::max(need, slot.bytes) <= sv->opts.mem_budget ||
                            sv->in_flight == 0;  // an idle device always admits one batch
          if (fits) {
            for (const Request& r : cand) {
              auto it = std::find_if(sv->pending.begin(), sv->pending.end(),
                                     [&](const Request& q) { return q.ticket == r.ticket; });
              sv->pending.erase(it);
            }
            batch = std::move(cand);
            for (size_t i = 0; i < batch.size(); ++i) view_params[i] = sv->scenes[batch[i].scene];
            slot.reserved = std::max(need, slot.bytes);
            sv->ledger = sv->ledger - held + slot.reserved;
            sv->peak_ledger = std::max(sv->peak_ledger, sv->ledger);
            sv->in_flight += 1;
            break;
          }
          sv->deferred += 1;
          sv->cv_done.wait(lk);  // wait for a batch to finish and free memory
          continue;
        }
        sv->cv_work.wait(lk);
      }
    }
    // render the batch on this slot's stream
    gs_camera cams[kMaxViews];
    float* images[kMaxViews];
    for (size_t i = 0; i < batch.size(); ++i) {
      cams[i] = batch[i].cam;
      images[i] = batch[i].out;
    }
    gs_status st = gs_render_fwd_multi(sv->ctx, view_params, cams, (int32_t)batch.size(), images,
                                       &sv->opts.render, &slot.frame, slot.stream);
    if (st == GS_OK && hipStreamSynchronize(slot.stream) != hipSuccess)
      st = hip_fail(hipErrorUnknown, "server batch");
    const Clock::time_point done = Clock::now();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      const size_t held = std::max(slot.bytes, slot.reserved);
      slot.bytes = slot.frame != nullptr ? slot.frame->bytes() : 0;
      slot.reserved = 0;
      sv->ledger = sv->ledger - held + slot.bytes;
      sv->peak_ledger = std::max(sv->peak_ledger, sv->ledger);
      sv->in_flight -= 1;
      sv->batches += 1;
      sv->batch_views += (int64_t)batch.size();
      for (const Request& r : batch) {
        Result& res = sv->results[r.ticket];
        res.done = true;
        res.status = st;
        res.latency_ms = std::chrono::duration<double, std::milli>(done - r.submitted).count();
        if (st == GS_OK) {
          sv->latencies.push_back(res.latency_ms);
          sv->completed += 1;
          sv->pixels += (double)r.cam.width * r.cam.height;
        }
      }
      sv->last_done = done;
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

}  // namespace

extern "C" {

gs_status gs_server_create(gs_ctx* ctx, const gs_server_opts* opts, gs_server** out) {
  if (ctx == nullptr || opts == nullptr || out == nullptr) {
    set_error("gs_server_create: null argument");
    return GS_ERR_INVALID;
  }
  *out = nullptr;
  if (opts->n_slots < 1 || opts->n_slots > 8 || opts->max_batch_views < 1 ||
      opts->max_batch_views > kMaxViews || opts->max_queue < 1) {
    set_error("gs_server_create: n_slots in [1, 8], max_batch_views in [1, %d], max_queue >= 1",
              kMaxViews);
    return GS_ERR_INVALID;
  }
  gs_server* sv = new (std::nothrow) gs_server();
  if (sv == nullptr) {
    set_error("gs_server_create: out of host memory");
    return GS_ERR_NOMEM;
  }
  sv->ctx = ctx;
  ctx_retain(ctx);
  sv->opts = *opts;
  sv->slots.resize(opts->n_slots);
  (void)hipSetDevice(ctx->device);
  for (Slot& s : sv->slots) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) {
      set_error("gs_server_create: hipStreamCreate failed");
      gs_server_destroy(sv);
      return GS_ERR_HIP;
    }
  }
  for (int i = 0; i < opts->n_slots; ++i) sv->workers.emplace_back(worker_main, sv, i);
  *out = sv;
  return GS_OK;
}

gs_status gs_server_add_scene(gs_server* sv, gs_params scene, int32_t* scene_id) {
  if (sv == nullptr || scene_id == nullptr || scene.means == nullptr || scene.n < 1 ||
      scene.sh_degree < 0 || scene.sh_degree > 3) {
    set_error("gs_server_add_scene: invalid arguments");
    return GS_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->scenes.push_back(scene);
  *scene_id = (int32_t)sv->scenes.size() - 1;
  return GS_OK;
}

gs_status gs_server_submit(gs_server* sv, int32_t scene, const gs_camera* cam, float* out_image,
                           uint64_t* ticket) {
  if (sv == nullptr || cam == nullptr || out_image == nullptr || ticket == nullptr) {
    set_error("gs_server_submit: null argument");
    return GS_ERR_INVALID;
  }
  if (cam->width < 1 || cam->width > 16384 || cam->height < 1 || cam->height > 16384) {
    set_error("gs_server_submit: image size out of range");
    return GS_ERR_INVALID;
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (scene < 0 || scene >= (int32_t)sv->scenes.size()) {
      set_error("gs_server_submit: unknown scene %d", scene);
      return GS_ERR_INVALID;
    }
    if ((int32_t)sv->pending.size() >= sv->opts.max_queue) {
      set_error("gs_server_submit: queue full (%d pending)", (int)sv->pending.size());
      return GS_ERR_BUSY;
    }
    Request r;
    r.ticket = sv->next_ticket++;
    r.scene = scene;
    r.cam = *cam;
    r.out = out_image;
    r.submitted = Clock::now();
    if (!sv->have_first) {
      sv->first_submit = r.submitted;
      sv->have_first = true;
    }
    sv->pending.push_back(r);
    sv->results[r.ticket] = Result();
    sv->submitted += 1;
    *ticket = r.ticket;
  }
  sv->cv_work.notify_one();
  return GS_OK;
}

gs_status gs_server_poll(gs_server* sv, uint64_t ticket, int32_t* done, double* latency_ms) {
  if (sv == nullptr || done == nullptr) {
    set_error("gs_server_poll: null argument");
    return GS_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->results.find(ticket);
  if (it == sv->results.end()) {
    set_error("gs_server_poll: unknown ticket %llu", (unsigned long long)ticket);
    return GS_ERR_INVALID;
  }
  *done = it->second.done ? 1 : 0;
  if (latency_ms) *latency_ms = it->second.latency_ms;
  if (it->second.done) {
    const gs_status st = it->second.status;
    sv->results.erase(it);
    return st;
  }
  return GS_OK;
}

gs_status gs_server_wait(gs_server* sv, uint64_t ticket, double* latency_ms) {
  if (sv == nullptr) {
    set_error("gs_server_wait: null server");
    return GS_ERR_INVALID;
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->results.find(ticket);
  if (it == sv->results.end()) {
    set_error("gs_server_wait: unknown ticket %llu", (unsigned long long)ticket);
    return GS_ERR_INVALID;
  }
  sv->cv_done.wait(lk, [&] {
    auto f = sv->results.find(ticket);
    return f == sv->results.end() || f->second.done;
  });
  auto f = sv->results.find(ticket);
  if (f == sv->results.end()) {
    set_error("gs_server_wait: ticket %llu was collected by another caller",
              (unsigned long long)ticket);
    return GS_ERR_INVALID;
  }
  const Result r = f->second;
  sv->results.erase(f);
  if (latency_ms) *latency_ms = r.latency_ms;
  return r.status;
}

gs_status gs_server_drain(gs_server* sv) {
  if (sv == nullptr) {
    set_error("gs_server_drain: null server");
    return GS_ERR_INVALID;
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  sv->cv_done.wait(lk, [&] { return sv->pending.empty() && sv->in_flight == 0; });
  return GS_OK;
}

gs_status gs_server_stats(gs_server* sv, gs_serve_stats* out) {
  if (sv == nullptr || out == nullptr) {
    set_error("gs_server_stats: null argument");
    return GS_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = sv->submitted;
  out->completed = sv->completed;
  out->batches = sv->batches;
  out->deferred = sv->deferred;
  out->mean_batch_views = sv->batches ? (double)sv->batch_views / sv->batches : 0.0;
  out->p50_ms = percentile(sv->latencies, 0.50);
  out->p99_ms = percentile(sv->latencies, 0.99);
  double s = 0.0, mx = 0.0;
  for (double x : sv->latencies) {
    s += x;
    mx = std::max(mx, x);
  }
  out->mean_ms = sv->latencies.empty() ? 0.0 : s / (double)sv->latencies.size();
  out->max_ms = mx;
  if (sv->have_first && sv->completed > 0) {
    const double secs = std::chrono::duration<double>(sv->last_done - sv->first_submit).count();
    out->mpix_per_s = secs > 0 ? sv->pixels / secs / 1e6 : 0.0;
  }
  out->peak_bytes = (int64_t)sv->peak_ledger;
  return GS_OK;
}

gs_status gs_server_reset_stats(gs_server* sv) {
  if (sv == nullptr) {
    set_error("gs_server_reset_stats: null server");
    return GS_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->latencies.clear();
  sv->submitted = sv->completed = sv->batches = sv->batch_views = sv->deferred = 0;
  sv->pixels = 0.0;
  sv->have_first = false;
  sv->peak_ledger = sv->ledger;
  return GS_OK;
}

void gs_server_destroy(gs_server* sv) {
  if (sv == nullptr) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  sv->cv_done.notify_all();
  for (std::thread& t : sv->workers)
    if (t.joinable()) t.join();
  (void)hipSetDevice(sv->ctx->device);
  for (Slot& s : sv->slots) {
    if (s.stream != nullptr) (void)hipStreamSynchronize(s.stream);
    if (s.frame != nullptr) gs_frame_release(s.frame);
    if (s.stream != nullptr) (void)hipStreamDestroy(s.stream);
  }
  gs_ctx* ctx = sv->ctx;
  delete sv;
  ctx_release(ctx);
}

}  // extern "C"
