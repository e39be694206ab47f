// Internal declarations of the isogs HIP library (gfx950 only).
//
// Data layout in HBM (per frame of V views over N Gaussians):
//   splat   float4[V*N*3]  per (view, Gaussian): {A, B, C, opacity},
//                          {int(floor(mx)), int(floor(my)), 0.5-frac(mx), 0.5-frac(my)},
//                          {r, g, b, depth}
//   rect    uint2[V*N]     tile rectangle, x0 | y0 << 16 and x1 | y1 << 16
//   dkey    u32[V*N]       float32 depth bits, 0xffffffff when untouched
//   clampm  u8[V*N]        SH clamp mask (bit c set: channel c clamped at 0)
//   sidx    u32[V*N]       (view*N + gid) in (depth bits, index) order
//   offs    u32[V*N]       exclusive scan of tiles touched, in sidx order
//   tkey    u32[K]         global tile id of each record, tile-sorted
//   tval    u32[K]         view*N + gid of each record
//   ranges  uint2[tiles]   [start, end) per global tile
//   finalT  f32[P], ncon u32[P]   per pixel over all views
//   acc     f32[V][9][N]   screen-space gradient accumulators
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "isogs.h"

namespace isogs {

constexpr int kMaxViews = 16;
// Screen-gradient accumulators, one record per (view, Gaussian) in each of two
// arrays held in one allocation: the geometric sums dL/d(mx, my, A, B, C,
// opacity) + 2 pad floats, then (after all geometric records) the colour sums
// dL/d(r, g, b) + 1 pad float.  The projection backward's geometry and colour
// kernels each read (and clear) only their own array.
// Largest record count of a frame: the sort kernels index records with 32-bit
// integers and round grids up to 4096-record chunks, so the count stays 2^20
// below 2^32 (every index + chunk offset then fits).
constexpr uint64_t kMaxRecords = 0xFFF00000ull;

constexpr int kAccG = 8;
constexpr int kAccC = 4;
constexpr int kAccStride = kAccG + kAccC;  // floats per (view, Gaussian) in total

// Frame-owned device words (u32 slots; 64-bit values at even slots).
enum Word {
  kWordFwdCounter = 0,  // work counter of the persistent forward blend
  kWordBwdCounter = 1,  // work counter of the persistent backward blend
  kWordK = 2,           // record count clamped to the capacity (device-count pipelines)
  kWordOverflow = 3,    // set when the records exceed the capacity
  kWordBC = 4,          // two floats: Adam 1/(1 - b1^t), 1/sqrt(1 - b2^t)
  kWordStep = 6,        // int64: Adam step of the next graph launch
  kWordTotal = 8,       // u64: record count from the scan
  kWordVisible = 10,    // (view, Gaussian) entries touching at least one tile
  kWordCount = 16
};

// Guard band on t_x/t_z, t_y/t_z for the projection Jacobian: 1.3 times the
// half field of view.
constexpr double kGuard = 1.3;

struct CamDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy, znear;
  double limx, limy;  // guard-band limits kGuard (W / 2) / fx and kGuard (H / 2) / fy, float64
  float campos[3];
  int W, H, tiles_x, tiles_y;
  int tile_offset;  // first global tile id of the view
  uint32_t entry_off;  // first (view, Gaussian) entry of the view (view * n unless multi-scene)
  long long pix_offset;  // first pixel of the view in the frame-wide pixel arrays
  float* image;          // forward output [3][H][W]
  const float* dimg;     // upstream gradient [3][H][W]
};

struct ViewTable {
  int n;            // number of views
  int tile;         // tile side in pixels
  int total_tiles;  // tiles over all views
  int reserved;
  float bg[3];
  float reserved2;
  CamDev v[kMaxViews];
};

struct ParamsDev {
  const float* means;
  const float* log_scales;
  const float* quats;
  const float* logits;
  const float* sh;
  int n;
  int sh_degree;
};

struct GradsDev {
  float* means;
  float* log_scales;
  float* quats;
  float* logits;
  float* sh;
  int accumulate;
  int keep_screen;  // leave the screen-space accumulators for export (no clearing)
};

__host__ __device__ inline int view_of_entry(const ViewTable& vt, uint32_t e) {
  int v = 0;
  for (int i = 1; i < vt.n; ++i)
    if (e >= vt.v[i].entry_off) v = i;
  return v;
}

__host__ __device__ inline int view_of_tile(const ViewTable& vt, int gt) {
  int v = 0;
  for (int i = 1; i < vt.n; ++i)
    if (gt >= vt.v[i].tile_offset) v = i;
  return v;
}

// ----------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
gs_status hip_fail(hipError_t e, const char* what);

#define GS_HIP(call)                                    \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

#define GS_LAUNCHED(name)                                        \
  do {                                                           \
    hipError_t e_ = hipGetLastError();                           \
    if (e_ != hipSuccess) return hip_fail(e_, "launch " name);  \
  } while (0)

// ------------------------------------------------------------ device memory
struct Ctx;

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// Grows b to at least `bytes`.  A buffer that has to be replaced may still be
// read by work queued earlier: the work enqueued on stream s, and the work
// before event `prior` (optional, e.g. a frame's last use on another stream).
// Both are waited for before the old buffer is freed; nothing else on the
// device is (so the streams of other frames keep running).
gs_status buf_ensure(Ctx* ctx, DevBuf& b, size_t bytes, hipStream_t s, hipEvent_t prior = nullptr);
void buf_free(Ctx* ctx, DevBuf& b);

// Pipeline stages timed with HIP events when a context enables timing.
enum Stage {
  ST_PROJECT = 0, ST_DEPTH_SORT, ST_SCAN, ST_EMIT, ST_TILE_SORT, ST_RANGES, ST_BLEND_FWD,
  ST_LOSS, ST_BLEND_BWD, ST_PROJECT_BWD, ST_ADAM, ST_INIT, ST_PROBE, ST_DENSIFY, ST_COUNT
};

struct PendingTiming {
  int stage;
  hipEvent_t a, b;
};

struct Ctx {
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  size_t peak = 0;
  std::mutex mem_mutex;  // guards in_use / peak (render server workers share a context)
  int cu_count = 0;
  hipDeviceProp_t prop;
  struct LossScratch* loss_scratch = nullptr;  // workspace of eager gs_loss_grad calls
  DevBuf dens_blk;                 // gs_densify: block totals and offsets
  uint32_t* dens_host = nullptr;   // gs_densify: pinned read-back of the totals
  DevBuf iso_blk;                  // gs_iso_extract: block totals and offsets
  DevBuf init_xyz;                 // gs_init_from_points: device copy of host points
  unsigned long long* iso_host = nullptr;  // gs_iso_extract: pinned read-back of the count
  // set while a graph is being captured: no allocation, no stage events
  bool capturing = false;
  // stage timing
  bool timing = false;
  PendingTiming* pending = nullptr;
  int n_pending = 0, cap_pending = 0;
  hipEvent_t* free_events = nullptr;
  int n_free = 0, cap_free = 0;
  double stage_ms[ST_COUNT] = {0};
  long long stage_count[ST_COUNT] = {0};
  // lifetime: frames, step graphs and render servers hold the context; a
  // destroy request while any of them lives is carried out by the last release
  std::mutex life_mutex;
  int dependents = 0;
  bool destroy_requested = false;
};

void ctx_retain(Ctx* ctx);
void ctx_release(Ctx* ctx);

// Workspace of the loss kernels: per-pixel SSIM partial derivatives of one view
// (9 floats per pixel) and per-block loss partials.  The context holds one for
// eager calls; every step graph holds its own, sized before capture, so a later
// eager call that needs more room never frees memory a graph replays into.
struct LossScratch {
  DevBuf gmap, part;
  hipEvent_t last_use = nullptr;  // recorded after each eager use
};
// Bytes of the two workspace arrays for views of these sizes.
void loss_scratch_bytes(const int* W, const int* H, int nv, size_t* gmap_bytes,
                        size_t* part_bytes);
gs_status loss_reserve(Ctx* ctx, LossScratch& ls, const int* W, const int* H, int nv,
                       hipStream_t s);
void loss_scratch_free(Ctx* ctx, LossScratch& ls);

// Records HIP events around a stage on stream s when the context times stages.
struct StageTimer {
  Ctx* c;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr;
  StageTimer(Ctx* c_, int st, hipStream_t s_);
  ~StageTimer();
};
gs_status timing_collect(Ctx* c);

// Radix-sort / scan scratch.
struct SortScratch {
  DevBuf hist;      // u32[256 * blocks]
  DevBuf partial;   // u64[blocks]
  DevBuf total;     // u64[1]
  hipEvent_t prior = nullptr;  // last use of the owning frame (see buf_ensure)
};

// Views of one scene inside a multi-scene frame: views [v0, v0 + nv) of the
// frame's table, entries [base, base + nv * pd.n).
struct SceneGroup {
  ParamsDev pd;
  int v0 = 0, nv = 0;
  uint32_t base = 0;
};

struct Frame {
  Ctx* ctx = nullptr;
  int64_t n = 0;        // Gaussians per view (0 in a multi-scene frame)
  int64_t entries = 0;  // (view, Gaussian) entries: views * n, or the sum over the views
  bool multi = false;   // views of several scenes (forward only)
  SceneGroup groups[kMaxViews];
  int n_groups = 0;
  int views = 0;
  int tile = 16;
  int depth = 256;
  int sh_degree = 0;
  ViewTable vt;
  int64_t K = 0;
  int64_t visible = 0;
  int64_t total_pix = 0;
  int key_bits = 1;
  DevBuf splat, rect, dkey, dkw[2], sidx[2], clampm, offs, tkey[2], tval[2], ranges, finalT,
      ncon, acc;
  DevBuf radii;               // int32[views][n] pixel radii (GS_RENDER_RADII)
  DevBuf gmu;                 // float[3][n]: the colour kernel's mean-gradient term (several views)
  // the projection backward's geometry kernel runs on `side` beside the colour
  // kernel on the call's stream (fork / join by the two events)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool keep_radii = false;    // this forward writes radii
  bool screen_kept = false;   // the last backward kept its screen-space sums
  int tkey_sel = 0;  // which of tkey/tval holds the sorted records
  int sidx_sel = 0;  // which of sidx holds the depth-sorted (view, Gaussian) indices
  bool acc_zeroed = false;
  bool persistent = false;            // blend with persistent work-queue kernels
  bool lpt = false;                   // persistent queue in longest-list-first tile order
  const uint32_t* tile_order = nullptr;
  DevBuf words;                       // kWordCount device words
  DevBuf okey[2], oval[2];            // tile-order sort buffers
  SortScratch ss;
  uint64_t* pinned = nullptr;  // host-pinned readback words (K, visible count)
  // recorded on the call's stream after each call that enqueues work on the
  // frame's buffers; a later call that must replace a buffer waits for it
  hipEvent_t last_use = nullptr;
  size_t bytes() const;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
// 1, 2, 3", SC'11): ten rounds on counter c with key (k0, k1), in place.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
  }
}

// ------------------------------------------------------------- pipelines (api.hip)
ParamsDev params_dev(const gs_params& p);
GradsDev grads_dev(const gs_params& g, int flags);
gs_status forward_stages(Ctx* ctx, Frame& f, const ParamsDev& pd, hipStream_t s, uint32_t cap);
gs_status backward_stages(Ctx* ctx, Frame& f, const ParamsDev& pd, const GradsDev& g,
                          hipStream_t s);

// ----------------------------------------------------------- kernel hosts
// preprocess.hip
// Projection of views vt (entries laid out [v][p.n] from entry `base` of the frame's
// per-entry arrays).
gs_status launch_preprocess_fwd(const ParamsDev& p, const ViewTable& vt, Frame& f,
                                hipStream_t s, size_t base = 0);
gs_status launch_preprocess_bwd(const ParamsDev& p, const ViewTable& vt, Frame& f,
                                const GradsDev& g, hipStream_t s);
gs_status launch_init_points(const float* xyz, int64_t n, const gs_init_opts& o,
                             uint64_t seed, gs_params out, hipStream_t s);
// sort.hip
// Stable LSD sort of n (key, value) pairs on key bits [0, bits): the first pass
// reads kin/vin (vin == nullptr: values are the indices 0..n-1) and passes
// alternate between buffer pairs A and B; *result_in_b tells where the result is.
gs_status sort_pairs_u32(Ctx* ctx, SortScratch& ss, const uint32_t* kin, const uint32_t* vin,
                         uint32_t* kA, uint32_t* vA, uint32_t* kB, uint32_t* vB, uint32_t n,
                         const uint32_t* d_n, int bits, int* result_in_b, hipStream_t s);
// Tile counts of the depth-ordered entries, scanned into record offsets; the
// entries' rectangles are also written in that order (srx, sry: the two halves)
// so the emission reads them coalesced.
gs_status scan_tile_counts(Ctx* ctx, SortScratch& ss, const uint32_t* sidx, const uint2* rect,
                           uint32_t n, uint32_t* offs, uint32_t* srx, uint32_t* sry,
                           uint64_t* d_total, hipStream_t s);
// Scratch for sorts of up to n pairs (so that no allocation happens later, e.g. in capture).
gs_status sort_reserve(Ctx* ctx, SortScratch& ss, uint32_t n, hipStream_t s);
// K = min(*total, cap); *overflow |= (*total > cap).
gs_status launch_clamp_count(const uint64_t* total, uint32_t cap, uint32_t* K,
                             uint32_t* overflow, hipStream_t s);
// Records of count (view, Gaussian) entries; overflow (optional) is set, and the
// entry skipped, when its records would pass the record buffers' capacity.
gs_status launch_emit(const ViewTable& vt, Frame& f, const uint32_t* sidx, const uint32_t* srx,
                      const uint32_t* sry, uint32_t count, uint32_t* overflow, hipStream_t s);
// Per-tile ranges of n_rec records (d_K: device count bounding n_rec, optional).
gs_status launch_ranges(Frame& f, uint32_t n_rec, const uint32_t* d_K, hipStream_t s);
// Tiles in descending list length (ties by tile id) for the persistent queue.
gs_status launch_tile_order(Frame& f, hipStream_t s);
gs_status launch_fill_u32(void* p, uint32_t value, size_t count, hipStream_t s);
// After a depth sort of n keys (untouched entries keyed 0xffffffff): the count of
// touched entries, read from the last pass's scanned digit table, into *dst.
gs_status launch_visible_count(const SortScratch& ss, uint32_t n, uint32_t* dst, hipStream_t s);
gs_status launch_export_keys(Frame& f, uint64_t* dst, hipStream_t s);
// blend.hip
gs_status launch_blend_fwd(const ViewTable& vt, Frame& f, hipStream_t s);
gs_status launch_blend_bwd(const ViewTable& vt, Frame& f, hipStream_t s);
// Screen gradients of view `view` (all views: -1) in the exported layout,
// float[.][n][12]: the six geometric sums, the three colour sums, 3 zero pads.
gs_status launch_export_screen_grads(Frame& f, int view, float* dst, hipStream_t s);
// loss.hip
// The workspace must have been reserved for these sizes (loss_reserve).
// Fixed workspace of the allocation-free loss call: set up once per device (with
// that device current) when a context is created, then handed out as a
// LossScratch view (GS_ERR_CAPACITY when the views need more than it holds).
constexpr size_t kNoAllocMaxPixels = (size_t)1 << 20;  // per view
gs_status loss_noalloc_setup(int device);
gs_status loss_noalloc_workspace(int device, const int* W, const int* H, int nv,
                                 LossScratch* out);
gs_status launch_loss(const LossScratch& ls, const float* const* x, const float* const* y,
                      const int* W, const int* H, int nv, float lambda, float* loss_out,
                      float* const* dl, hipStream_t s);
// iso.hip
gs_status iso_extract_run(Ctx* ctx, const gs_volume& vol, float iso, float keep_prob,
                          uint64_t seed, float* xyz, int64_t cap, int64_t* n_kept,
                          hipStream_t s);
gs_status launch_raycast(const gs_volume& vol, float iso, const gs_camera* cams, int nv,
                         float* const* images, double step, hipStream_t s);
// density.hip
gs_status launch_density_accumulate(const Frame& f, const gs_density_stats& st, float scale,
                                    hipStream_t s);
gs_status densify_run(Ctx* ctx, const gs_params& p, const gs_params& m, const gs_params& v,
                      const gs_density_stats& st, const gs_density_opts& o, const gs_params* p_out,
                      const gs_params* m_out, const gs_params* v_out, int32_t* src_index,
                      gs_density_info* info, hipStream_t s);
gs_status launch_opacity_reset(const gs_params& p, const gs_params& m, const gs_params& v,
                               double max_opacity, hipStream_t s);
// Per-view MSE, PSNR, L1 and SSIM into out[nv][4] (workspace as for launch_loss).
gs_status launch_metrics(const LossScratch& ls, const float* const* x, const float* const* y,
                         const int* W, const int* H, int nv, float* out, hipStream_t s);
// probe.hip
gs_status launch_copy_probe(Ctx* ctx, const void* src, void* dst, size_t bytes, hipStream_t s);
// adam.hip
// dev_bc (optional): device {1/(1-b1^t), 1/sqrt(1-b2^t)} replacing the host values of
// `step`; skip (optional): device flag that suppresses the update while nonzero.
gs_status launch_adam(const gs_params& p, const gs_params& g, const gs_params& m,
                      const gs_params& v, const gs_adam_opts& o, int64_t step, hipStream_t s,
                      const float* dev_bc = nullptr, const uint32_t* skip = nullptr);

}  // namespace isogs

struct gs_ctx : isogs::Ctx {};
struct gs_frame : isogs::Frame {};
