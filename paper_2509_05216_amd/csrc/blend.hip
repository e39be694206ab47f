// Front-to-back alpha compositing of each tile's sorted list (forward) and its
// reverse traversal (backward).
//
// One workgroup per tile, one pixel per thread (TILE x TILE threads).  Each
// wave owns an 8 x 8 block of the tile.  The tile's records are staged
// through LDS in batches of DEPTH splats; every lane of a wave reads the same
// LDS address (broadcast).  When a splat is staged its loader also tests the
// axis-aligned box outside which alpha < 1/255 for certain (the ellipse power
// >= -ln(255 o), widened by a safety margin; computed once per splat by the
// projection) against the tile's 8 x 8 wave blocks; a ballot/popcount compaction then gives every wave
// the ordered list of staged splats that can touch its block, and the wave
// walks only that list.  Skipped pairs would be rejected by the alpha test
// anyway, so results are unchanged and most of the per-pair work disappears.
//
// The forward stops a batch loop once every pixel of the tile has terminated
// (block-wide vote).  The backward walks the list from the tile's last
// contributor down to its first, recomputing each pixel's transmittance as
// T * rcp(1 - alpha) from the final value (1 - alpha >= 0.01, so the 1-ulp
// hardware reciprocal is ample), so no per-pixel list is stored.  Each pair
// yields nine per-lane sums (dpow dx, dpow dy, dpow dx^2, dpow dx dy, dpow dy^2,
// dpow and the three colour weights; the conic is applied to the first two and
// the opacity divides the sixth once per (tile, Gaussian) when the sums are
// flushed).  They are
// reduce-scattered across the wave (eight by two gfx950 permlane swaps and DPP
// steps inside 16-lane rows, the ninth by DPP row sums: 21 VALU instructions
// for all nine), added
// across the workgroup's waves with LDS float atomics and to the per-Gaussian
// accumulators with one global atomic per component per (tile, Gaussian).
//
// Both walks are branch-free per pair (lanes that skip a pair select zeros),
// keep two slots' LDS operands in flight, and read the wave's list (slot byte
// offsets) four or two entries at a time straight into VGPRs that address the
// slot data.  The forward keeps its stopped lanes as a wave mask, so its
// per-pair use/stop decisions are scalar operations on comparison ballots; the
// backward's flush transforms each slot's sums in place before the global
// atomics.  A staged splat carries its conic pre-scaled by -log2(e)/2 (one
// fused quadratic and one v_exp per pair), log2 of its opacity in place of the
// opacity (one v_log per staged splat), so that pa = p2 + log2 o is log2 of
// o G: the alpha test o G >= 1/255 becomes pa >= -log2 255, taken before any
// v_exp (a backward pair the test rejects costs none; the log-domain test
// agrees with the linear one except within about 1e-6 of the threshold), and
// alpha = 2^pa.  Its mean is stored relative to the tile origin.  Both kernels evaluate the skip/stop decisions with the same
// inline code on the same staged values (the library is compiled with
// -ffp-contract=off, and the fused operations are explicit), so the backward
// reproduces the forward's decisions exactly.
#include "internal.h"

namespace isogs {
namespace {

constexpr float kAlphaMax = 0.99f;
constexpr float kLog2AlphaMin = -7.99435343685885793f;  // log2(1/255)
constexpr float kTMin = 1e-4f;

// Staged form of a splat: the conic scaled so that one fused quadratic gives
// log2 of the Gaussian factor,
//   p2 = log2(e) * power = a dx^2 + b dx dy + c dy^2,
//   (a, b, c) = -log2(e) (A / 2, B, C / 2),
// and the mean relative to the tile origin, so dx = (pixel x - tile x0) - mx'.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// p2 and the offsets (dx, dy) of a pixel (tile-relative integer coordinates
// rx, ry as floats) from a staged splat; exp2(p2) is the Gaussian factor.
__device__ inline float pair_eval(float4 q, float2 m, float rx, float ry, float& dx, float& dy) {
  dx = rx - m.x;
  dy = ry - m.y;
  return fmaf(fmaf(q.y, dy, q.x * dx), dx, (q.z * dy) * dy);
}

// Conservative box of the alpha >= 1/255 region, (mean_x, mean_y, half_w, half_h),
// from a splat record: the projection stored the half-widths (fp16, rounded
// up) in the fourth word of the colour quad; half_w < 0 when the splat can
// never pass the alpha test.
__device__ inline float half_lo(uint32_t u) {
  const uint16_t b = (uint16_t)(u & 0xffffu);
  _Float16 h;
  __builtin_memcpy(&h, &b, 2);
  return (float)h;
}

__device__ inline float4 splat_box(float4 q1, float4 q2) {
  const float mx = (float)__float_as_int(q1.x) + 0.5f - q1.z;
  const float my = (float)__float_as_int(q1.y) + 0.5f - q1.w;
  const uint32_t hb = __float_as_uint(q2.w);
  return make_float4(mx, my, half_lo(hb), half_lo(hb >> 16));
}

// True when the box misses the 8 x 8 block whose first pixel is (bx0, by0).
__device__ inline bool box_misses(float4 b, int bx0, int by0) {
  const float x0 = (float)bx0 + 0.5f, y0 = (float)by0 + 0.5f;
  return b.z < 0.f || b.x + b.z < x0 || b.x - b.z > x0 + 7.0f || b.y + b.w < y0 ||
         b.y - b.w > y0 + 7.0f;
}


// Stage records [base, base + cnt) of the tile list into LDS and build, for
// every wave, the ascending list of batch slots whose alpha box overlaps the
// wave's 8 x 8 block (ballot + popcount compaction; DEPTH <= threads).
template <int NT, int DEPTH>
struct Stage {
  static constexpr int NW = NT / 64;
  // 16 bytes per slot in every array, so one shifted index addresses all three.
  // The walks read 16 + 16 + 4 (forward) or 16 + 16 + 8 (backward) bytes per
  // slot: 12-byte LDS reads measured slower than 8- and 16-byte ones here
  // (layouts that read the colour or the mean quad as 12 bytes took 2-3% longer).
  float4 s0[DEPTH];  // scaled conic (a, b, c), log2 of the opacity
  float4 s1[DEPTH];  // mean relative to the tile origin (x, y), red, green
  float4 s2[DEPTH];  // blue, 4 x slot as bits (the slot's sum-table column), unused
  uint32_t sidx[DEPTH];
  // per wave: byte offsets (16 x slot) of the overlapping slots in ascending
  // order, then four zero entries, so that reads of up to four entries past the
  // end stay valid; 16-byte aligned for four-entry reads
  alignas(16) uint32_t list[NW][DEPTH + 4];
  uint32_t chunk[NW][DEPTH / 64 + 1];
  uint32_t count[NW];
};

template <int TILE, int DEPTH>
__device__ inline void stage_batch(Stage<TILE * TILE, DEPTH>& st, const uint32_t* __restrict__ tval,
                                   const float4* __restrict__ splat, uint32_t base, int cnt,
                                   int tile_x0, int tile_y0) {
  constexpr int NT = TILE * TILE;
  constexpr int NW = NT / 64;
  constexpr int BPR = TILE / 8;
  const int t = threadIdx.x;
  const int lane = __lane_id(), wave = t / 64;
  uint32_t mask = 0;
  if (t < cnt) {
    const uint32_t idx = tval[base + t];
    const float4 q0 = splat[(size_t)idx * 3 + 0], q1 = splat[(size_t)idx * 3 + 1];
    const float4 q2 = splat[(size_t)idx * 3 + 2];
    st.sidx[t] = idx;
    st.s0[t] = make_float4(q0.x * (-0.5f * kLog2e), q0.y * -kLog2e, q0.z * (-0.5f * kLog2e),
                           __builtin_amdgcn_logf(q0.w));  // log2 o (-inf for o = 0)
    st.s1[t] = make_float4((float)(__float_as_int(q1.x) - tile_x0) - q1.z,
                           (float)(__float_as_int(q1.y) - tile_y0) - q1.w,
                           q2.x, q2.y);
    st.s2[t] = make_float4(q2.z, __uint_as_float((uint32_t)t * 4u), 0.f, 0.f);
    const float4 b = splat_box(q1, q2);
#pragma unroll
    for (int w = 0; w < NW; ++w)
      if (!box_misses(b, tile_x0 + (w % BPR) * 8, tile_y0 + (w / BPR) * 8)) mask |= 1u << w;
  }
  const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  uint32_t rank[NW];
  if (t < DEPTH) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint64_t bal = __ballot((mask >> w) & 1u);
      rank[w] = (uint32_t)__popcll(bal & lt);
      if (lane == 0) st.chunk[w][wave] = (uint32_t)__popcll(bal);
    }
  }
  __syncthreads();
  if (t < DEPTH) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if ((mask >> w) & 1u) {
        uint32_t off = rank[w];
        for (int c = 0; c < wave; ++c) off += st.chunk[w][c];
        st.list[w][off] = (uint32_t)t * 16u;
      }
      if (t == 0) {
        uint32_t tot = 0;
        for (int c = 0; c < (DEPTH + 63) / 64; ++c) tot += st.chunk[w][c];
        st.count[w] = tot;
#pragma unroll
        for (int u = 0; u < 4; ++u) st.list[w][tot + u] = 0u;
      }
    }
  }
  __syncthreads();
}

template <int TILE>
struct Layout {
  static constexpr int NT = TILE * TILE;
  static constexpr int BPR = TILE / 8;  // 8x8 blocks per tile row
  __device__ static void pixel(int tile_x, int tile_y, int& px, int& py, int& bx0, int& by0) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    bx0 = tile_x * TILE + (wave % BPR) * 8;
    by0 = tile_y * TILE + (wave / BPR) * 8;
    px = bx0 + (lane & 7);
    py = by0 + (lane >> 3);
  }
};

// Operands of one staged splat, read from LDS (same address in every lane).
// The walks take slot byte offsets straight from the wave's list (LDS reads
// of several entries at once into VGPRs, used as addresses as they are).
struct Slot {
  uint32_t off;   // 16 x slot index
  uint32_t off4;  // 4 x slot index (byte offset of the slot's column in the sum table)
  float4 q0;      // scaled conic, log2 of the opacity
  float2 m;       // tile-relative mean
  float3 q2;      // rgb
};

template <int NT, int DEPTH>
__device__ inline Slot load_slot(const Stage<NT, DEPTH>& st, uint32_t off) {
  Slot s;
  s.off = off;
  s.q0 = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(st.s0) + off);
  const float4 m = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(st.s1) + off);
  s.m = make_float2(m.x, m.y);
  const float4 c = *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(st.s2) + off);
  s.off4 = __float_as_uint(c.y);
  s.q2 = make_float3(m.z, m.w, c.x);
  return s;
}

// Forward of one tile (global tile id gt) by the whole workgroup.
template <int TILE, int DEPTH>
__device__ inline void fwd_tile(Stage<TILE * TILE, DEPTH>& st, const ViewTable& vt, int gt,
                                const uint2* __restrict__ ranges,
                                const uint32_t* __restrict__ tval,
                                const float4* __restrict__ splat, float* __restrict__ finalT,
                                uint32_t* __restrict__ ncon) {
  constexpr int NT = TILE * TILE;
  const int v = view_of_tile(vt, gt);
  const CamDev& cam = vt.v[v];
  const int lt = gt - cam.tile_offset;
  const int tile_x = lt % cam.tiles_x, tile_y = lt / cam.tiles_x;
  int px, py, bx0, by0;
  Layout<TILE>::pixel(tile_x, tile_y, px, py, bx0, by0);
  const int wave = threadIdx.x / 64;
  const bool inside = px < cam.W && py < cam.H;
  const float rx = (float)(px - tile_x * TILE), ry = (float)(py - tile_y * TILE);
  const uint2 rg = ranges[gt];
  float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f;
  uint32_t last = 0;
  // lanes that have stopped (outside the image or terminated), as a wave mask:
  // the per-pair decisions are then scalar mask operations on comparison results
  uint64_t done_m = __builtin_amdgcn_ballot_w64(!inside);
  for (uint32_t base = rg.x; base < rg.y; base += DEPTH) {
    if (__syncthreads_count(__builtin_amdgcn_inverse_ballot_w64(done_m)) == NT) break;
    const int cnt = (int)min((uint32_t)DEPTH, rg.y - base);
    stage_batch<TILE, DEPTH>(st, tval, splat, base, cnt, tile_x * TILE, tile_y * TILE);
    const int nw = __builtin_amdgcn_readfirstlane((int)st.count[wave]);
    if (nw == 0 || done_m == ~0ull) continue;
    // Branch-free front-to-back step; a lane that has stopped keeps its state.
    // last_off: list offset of this batch's last record used by the lane
    uint32_t last_off = ~0u;
    auto step = [&](const Slot& s) {
      float dx, dy;
      const float p2 = pair_eval(s.q0, s.m, rx, ry, dx, dy);
      const float pa = p2 + s.q0.w;  // log2 (o G)
      // alpha ahead of the test (its v_exp overlaps the ballots)
      const float alpha = fminf(kAlphaMax, __builtin_amdgcn_exp2f(pa));
      uint64_t m_use = ~done_m & __builtin_amdgcn_ballot_w64(!(p2 > 0.f)) &
                       __builtin_amdgcn_ballot_w64(pa >= kLog2AlphaMin);
      if (m_use == 0) return;  // no lane takes this splat: nothing changes
      // weight alpha T and the transmittance after, T - alpha T = T (1 - alpha)
      const float wa = alpha * T;
      const float Tn = T - wa;
      const uint64_t m_stop = m_use & __builtin_amdgcn_ballot_w64(Tn < kTMin);
      done_m |= m_stop;
      m_use &= ~m_stop;
      const bool use = __builtin_amdgcn_inverse_ballot_w64(m_use);
      const float w = use ? wa : 0.f;
      cr = fmaf(s.q2.x, w, cr);
      cg = fmaf(s.q2.y, w, cg);
      cb = fmaf(s.q2.z, w, cb);
      T = use ? Tn : T;
      last_off = use ? s.off : last_off;
    };
    const uint32_t* row = st.list[wave];
    auto entries = [&](int k) { return *reinterpret_cast<const uint4*>(row + k); };
    // entries kk .. kk + 3 in one read; two slots in flight (the LDS reads of
    // one overlap the arithmetic of the other), eight per iteration
    uint4 e = entries(0);
    Slot a = load_slot(st, e.x);
    int kk = 0;
    bool all_done = false;
    for (; kk + 7 < nw; kk += 8) {
      const uint4 e1 = entries(kk + 4);
      Slot b = load_slot(st, e.y);
      step(a);
      a = load_slot(st, e.z);
      step(b);
      b = load_slot(st, e.w);
      step(a);
      a = load_slot(st, e1.x);
      step(b);
      const uint4 e2 = entries(kk + 8);  // <= nw + 3: padded
      b = load_slot(st, e1.y);
      step(a);
      a = load_slot(st, e1.z);
      step(b);
      b = load_slot(st, e1.w);
      step(a);
      a = load_slot(st, e2.x);
      step(b);
      e = e2;
      if (done_m == ~0ull) {
        all_done = true;
        break;
      }
    }
    if (!all_done) {
      if (kk + 3 < nw) {  // four more
        const uint4 e1 = entries(kk + 4);
        Slot b = load_slot(st, e.y);
        step(a);
        a = load_slot(st, e.z);
        step(b);
        b = load_slot(st, e.w);
        step(a);
        a = load_slot(st, e1.x);
        step(b);
        e = e1;
        kk += 4;
      }
      // up to three left: e holds entries kk .. kk + 3, a entry kk
      if (kk < nw) {
        const Slot b = load_slot(st, e.y);
        step(a);
        a = b;
      }
      if (kk + 1 < nw) {
        const Slot b = load_slot(st, e.z);
        step(a);
        a = b;
      }
      if (kk + 2 < nw) step(a);
    }
    if (last_off != ~0u) last = base - rg.x + 1u + (last_off >> 4);
  }
  if (inside) {
    const size_t pix = (size_t)py * cam.W + px;
    const size_t plane = (size_t)cam.W * cam.H;
    cam.image[pix] = cr + T * vt.bg[0];
    cam.image[plane + pix] = cg + T * vt.bg[1];
    cam.image[2 * plane + pix] = cb + T * vt.bg[2];
    finalT[cam.pix_offset + pix] = T;
    ncon[cam.pix_offset + pix] = last;
  }
}

// Waves of one tile wait at every batch for the slowest of them (the wave whose
// 8 x 8 block has the most steps in the batch walks about 1.75 times the mean,
// by a CPU count on one 2048 x 2048 view), so the forward is held to 64 VGPRs
// for tiles up to 16: eight resident waves per SIMD instead of seven fill more
// of those waits (1.37 against 1.44 ms for the 4M-Gaussian batched step).
template <int TILE>
constexpr int kFwdWaves = TILE <= 16 ? 8 : 1;

// One workgroup per tile.
template <int TILE, int DEPTH>
__global__ __launch_bounds__(TILE* TILE) __attribute__((amdgpu_waves_per_eu(kFwdWaves<TILE>))) void k_blend_fwd(ViewTable vt,
                                                          const uint2* __restrict__ ranges,
                                                          const uint32_t* __restrict__ tval,
                                                          const float4* __restrict__ splat,
                                                          float* __restrict__ finalT,
                                                          uint32_t* __restrict__ ncon) {
  __shared__ Stage<TILE * TILE, DEPTH> st;
  fwd_tile<TILE, DEPTH>(st, vt, blockIdx.x, ranges, tval, splat, finalT, ncon);
}

// Next work item of a persistent workgroup: a tile index from the shared
// counter, mapped through the tile order when one is given; -1 when drained.
__device__ inline int next_tile(uint32_t* counter, const uint32_t* order, int total,
                                uint32_t* slot) {
  __syncthreads();  // the previous item (and its LDS use) is finished
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1u);
  __syncthreads();
  const uint32_t it = *slot;
  if (it >= (uint32_t)total) return -1;
  return order != nullptr ? (int)order[it] : (int)it;
}

// Persistent form: a grid sized to the device's resident capacity drains the
// (view, tile) work queue of all views, in the given tile order.
template <int TILE, int DEPTH>
__global__ __launch_bounds__(TILE* TILE) __attribute__((amdgpu_waves_per_eu(kFwdWaves<TILE>))) void k_blend_fwd_persistent(
    ViewTable vt, const uint2* __restrict__ ranges, const uint32_t* __restrict__ tval,
    const float4* __restrict__ splat, float* __restrict__ finalT, uint32_t* __restrict__ ncon,
    const uint32_t* __restrict__ order, uint32_t* counter) {
  __shared__ Stage<TILE * TILE, DEPTH> st;
  __shared__ uint32_t slot;
  for (;;) {
    const int gt = next_tile(counter, order, vt.total_tiles, &slot);
    if (gt < 0) break;
    fwd_tile<TILE, DEPTH>(st, vt, gt, ranges, tval, splat, finalT, ncon);
  }
}

// ---------------------------------------------------------------- reduction
// (a + partner) where lanes 0-31 pair with 32-63: lower lanes get a's sum,
// upper lanes b's sum.
__device__ inline float swap32_sum(float a, float b) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Rows 0 and 2 get the xor-16 pair sum of a, rows 1 and 3 that of b.
__device__ inline float swap16_sum(float a, float b) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Reduce-scatter of nine per-lane values over the wave.  The first eight go
// through xor-32 pairs (g0..g3 kept by lanes 0-31, g4..g7 by 32-63) and xor-16
// pairs (row r then holds values (r & 1) + 4 (r >> 1) and that + 2); inside a
// 16-lane row the xor-8 step (row_ror:8) leaves one value per 8-lane half, and
// the mirror and two quad steps sum each half, so lane 0 of row r owns the
// first of the row's values and lane 8 the second.  The ninth is summed over
// each row by the same four DPP steps and added by the row's last lane (four
// LDS atomics).  lane_slot() names the value a lane ends up owning.
__device__ inline int lane_slot(int lane) {
  const int row = lane >> 4, p = lane & 15;
  const int base = (row & 1) + 4 * (row >> 1);
  if (p == 0) return base;
  if (p == 8) return base + 2;
  if (p == 15) return 8;
  return -1;
}

// Adds the wave sums of g[0..8] to the sum table (LDS atomics): the lane that
// owns sum k (slot = lane_slot(lane) = k) adds it at dst, its address for k.
__device__ inline void wave_reduce_add(const float* g, float* dst, int slot) {
  const float a0 = swap32_sum(g[0], g[4]);
  const float a1 = swap32_sum(g[1], g[5]);
  const float a2 = swap32_sum(g[2], g[6]);
  const float a3 = swap32_sum(g[3], g[7]);
  const float b0 = swap16_sum(a0, a1);
  const float b1 = swap16_sum(a2, a3);
  // xor 8 (row_ror:8): lanes 0-7 sum b0 with their partner's, lanes 8-15 b1 (two
  // adds, each writing two of a row's four 4-lane banks); then the half mirror and
  // two quad steps sum each 8-lane half.  The ninth value takes the same four steps
  // on its own register, and its last step writes the row total into d's lanes
  // 12-15, where lane 15 owns it.  A VALU write read by a DPP operand needs two
  // wait states, which the interleaving and the s_nops provide (the compiler does
  // not see inside the block, so the first s_nop covers the inputs' last writes).
  float d, e;
  asm("s_nop 1\n\t"
      "v_add_f32_dpp %0, %2, %2 row_ror:8 row_mask:0xf bank_mask:0xc\n\t"
      "v_add_f32_dpp %0, %3, %3 row_ror:8 row_mask:0xf bank_mask:0x3\n\t"
      "v_add_f32_dpp %1, %4, %4 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 0\n\t"
      "v_add_f32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
      "v_add_f32_dpp %1, %1, %1 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 0\n\t"
      "v_add_f32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
      "v_add_f32_dpp %1, %1, %1 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 0\n\t"
      "v_add_f32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
      "s_nop 0\n\t"
      "v_add_f32_dpp %0, %1, %1 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0x8"
      : "=&v"(d), "=&v"(e)
      : "v"(b1), "v"(b0), "v"(g[8]));
  (void)e;
  // an LDS add of a zero sum is harmless, so no test guards it
  if (slot >= 0) atomicAdd(dst, d);
}

template <int TILE, int DEPTH>
struct BwdSmem {
  static constexpr int kPart = DEPTH + 1;  // row of the sum table (odd: no bank conflicts)
  Stage<TILE * TILE, DEPTH> st;
  float part[9 * kPart];  // sum c of slot j at c * kPart + j
  uint32_t smax[TILE * TILE / 64];
};

// Backward of one tile (global tile id gt) by the whole workgroup.
template <int TILE, int DEPTH>
__device__ inline void bwd_tile(BwdSmem<TILE, DEPTH>& sm, const ViewTable& vt, int gt,
                                const uint2* __restrict__ ranges,
                                const uint32_t* __restrict__ tval,
                                const float4* __restrict__ splat,
                                const float* __restrict__ finalT,
                                const uint32_t* __restrict__ ncon, float* __restrict__ accG,
                                float* __restrict__ accC) {
  constexpr int NT = TILE * TILE;
  constexpr int NW = NT / 64;
  Stage<NT, DEPTH>& st = sm.st;
  float* part = sm.part;
  uint32_t* smax = sm.smax;
  const int v = view_of_tile(vt, gt);
  const CamDev& cam = vt.v[v];
  const int lt = gt - cam.tile_offset;
  const int tile_x = lt % cam.tiles_x, tile_y = lt / cam.tiles_x;
  int px, py, bx0, by0;
  Layout<TILE>::pixel(tile_x, tile_y, px, py, bx0, by0);
  const bool inside = px < cam.W && py < cam.H;
  const float rx = (float)(px - tile_x * TILE), ry = (float)(py - tile_y * TILE);
  const uint2 rg = ranges[gt];
  const int lane = __lane_id(), wave = threadIdx.x / 64;

  float T = 1.f, dr = 0.f, dg = 0.f, db = 0.f;
  uint32_t nc = 0;
  if (inside) {
    const size_t pix = (size_t)py * cam.W + px;
    const size_t plane = (size_t)cam.W * cam.H;
    T = finalT[cam.pix_offset + pix];
    nc = ncon[cam.pix_offset + pix];
    dr = cam.dimg[pix];
    dg = cam.dimg[plane + pix];
    db = cam.dimg[2 * plane + pix];
  }
  // D = dL/dout . S, with S the colour composited behind the current record
  // (it starts as T_final * bg); dL/dalpha needs S only through this product
  float D = T * (dr * vt.bg[0] + dg * vt.bg[1] + db * vt.bg[2]);
  const int slot = lane_slot(lane);
  constexpr int kPart = BwdSmem<TILE, DEPTH>::kPart;
  // this lane's sum row (slot >= 0); the slot's column is added per pair
  float* const part_lane = part + (slot >= 0 ? slot : 0) * kPart;
  // last contributor of the wave and of the tile
  uint32_t m = nc;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
  const int wave_n = __builtin_amdgcn_readfirstlane((int)m);
  if (lane == 0) smax[wave] = m;
  __syncthreads();
  uint32_t maxn = 0;
  for (int w = 0; w < NW; ++w) maxn = max(maxn, smax[w]);
  // the sum table starts cleared; each flush clears the entries it consumed
  for (int j = threadIdx.x; j < 9 * kPart; j += NT) part[j] = 0.f;

  for (int hi = (int)maxn; hi > 0; hi -= DEPTH) {
    const int lo = max(0, hi - DEPTH);
    const int cnt = hi - lo;
    __syncthreads();
    stage_batch<TILE, DEPTH>(st, tval, splat, rg.x + (uint32_t)lo, cnt, tile_x * TILE,
                             tile_y * TILE);
    // walk this wave's overlapping slots from the back, below its last contributor
    // entries of this wave's list below its last contributor: the list is
    // ascending, so they are a prefix, counted by ballots over its chunks
    const uint32_t* row = st.list[wave];
    const int cw = __builtin_amdgcn_readfirstlane((int)st.count[wave]);
    int nuse = 0;
    if (lo < wave_n) {
      for (int c0 = 0; c0 < cw; c0 += 64) {
        const int e = c0 + (int)__lane_id();
        const bool below = e < cw && lo + (int)(row[min(e, DEPTH - 1)] >> 4) < wave_n;
        nuse += (int)__popcll(__ballot(below));
      }
    }
    int k = nuse - 1;
    // lo + j < nc as a comparison of sum-table offsets: 4 j < 4 (nc - lo)
    const uint32_t ncb = nc > (uint32_t)lo ? min(nc - (uint32_t)lo, (uint32_t)DEPTH) * 4u : 0u;
    // One pair (this lane's pixel, slot s) of the reverse walk.
    auto pair = [&](const Slot& s) {
      const float3 q2 = s.q2;
      // the skip decisions are the forward's, from the same expressions
      float dx, dy;
      const float p2 = pair_eval(s.q0, s.m, rx, ry, dx, dy);
      const float pa = p2 + s.q0.w;  // log2 (o G)
      // nc = 0 outside the image, so the first test also covers the image bounds;
      // one ballot per comparison keeps the wave test on the comparison masks
      const bool c_pos = s.off4 < ncb;
      const bool c_pow = !(p2 > 0.f);
      const bool c_alpha = pa >= kLog2AlphaMin;
      if ((__builtin_amdgcn_ballot_w64(c_pos) & __builtin_amdgcn_ballot_w64(c_pow) &
           __builtin_amdgcn_ballot_w64(c_alpha)) == 0)
        return;
      const float a_raw = __builtin_amdgcn_exp2f(pa);  // o G
      const float alpha = fminf(kAlphaMax, a_raw);
      const bool contrib = c_pos && c_pow && c_alpha;
      // Gradient arithmetic, branch-free: a lane that does not contribute takes
      // alpha = 0, so 1 / (1 - 0) = 1 exactly, its T and D stay as they are and its
      // nine values are zeros.  1 - alpha >= 0.01, so the hardware reciprocal
      // (1 ulp) is safe here.
      const float ac = contrib ? alpha : 0.f;
      const float inv = __builtin_amdgcn_rcpf(1.f - ac);
      const float Tb = T * inv;  // transmittance before this record
      T = Tb;
      const float w = ac * Tb;
      // dL/dalpha = T_before (dL/dout . rgb) - D / (1 - alpha); clamped alpha has
      // zero derivative, so the alpha factor of dpow is zero there
      const float cdot = fmaf(db, q2.z, fmaf(dg, q2.y, dr * q2.x));
      const float ao = a_raw <= kAlphaMax ? ac : 0.f;
      const float dalpha = fmaf(Tb, cdot, -D * inv);
      D = fmaf(w, cdot, D);
      // Per-pair sums whose (tile, Gaussian) totals give the screen gradients:
      // dpow dx, dpow dy (mean, after the conic is applied at the flush),
      // dpow dx^2, dpow dx dy, dpow dy^2 (conic), dpow (opacity: dL/do is the sum
      // of dalpha G = dpow / o over unclamped pairs, and dpow is zero on the
      // others), w dL/dout (colour).
      const float dpow = dalpha * ao;
      const float ex = dpow * dx, ey = dpow * dy;
      float g[9];
      g[0] = ex;
      g[1] = ey;
      g[2] = ex * dx;
      g[3] = ex * dy;
      g[4] = ey * dy;
      g[5] = dpow;
      g[6] = w * dr;
      g[7] = w * dg;
      g[8] = w * db;
      wave_reduce_add(g, reinterpret_cast<float*>(reinterpret_cast<char*>(part_lane) + s.off4),
                      slot);
    };
    // two slots in flight: the LDS reads of one overlap the arithmetic of the
    // other; list entries two at a time (k - 1, k with k odd: 8-byte aligned)
    if (k >= 0) {
      if ((k & 1) == 0) {  // odd count: the top entry alone, then pairs (k, k - 1)
        pair(load_slot(st, row[k]));
        --k;
      }
      if (k >= 1) {
        uint2 e = *reinterpret_cast<const uint2*>(row + k - 1);  // entries k - 1, k
        Slot a = load_slot(st, e.y);
        for (;;) {
          const Slot b = load_slot(st, e.x);
          const uint2 en = *reinterpret_cast<const uint2*>(row + max(k - 3, 0));
          pair(a);
          k -= 2;
          if (k < 1) {
            pair(b);
            break;
          }
          a = load_slot(st, en.y);
          pair(b);
          e = en;
        }
      }
    }
    __syncthreads();
    // flush, first the per-slot transforms (one thread per slot, in place):
    // mean (A dx + B dy, B dx + C dy) dpow summed = the conic applied to the
    // first two sums; conic -dpow dx^2 / 2, -dpow dx dy, -dpow dy^2 / 2;
    // opacity: sum of dpow / o
    if ((int)threadIdx.x < cnt) {
      const int j = threadIdx.x;
      const float4 q = st.s0[j];
      const float A = q.x * (-2.f * kLn2), B = q.y * -kLn2, C = q.z * (-2.f * kLn2);
      const float e0 = part[j], e1 = part[kPart + j];
      part[j] = fmaf(A, e0, B * e1);
      part[kPart + j] = fmaf(B, e0, C * e1);
      part[2 * kPart + j] *= -0.5f;
      part[3 * kPart + j] *= -1.f;
      part[4 * kPart + j] *= -0.5f;
      // a nonzero sum comes from contributing pairs, whose opacity is >= about
      // 1/255 (the alpha test), so 1/o = 2^-log2(o) is finite; a zero sum stays
      // zero whatever the opacity (no 0 * inf at an opacity that underflowed to 0)
      const float e5 = part[5 * kPart + j];
      part[5 * kPart + j] = e5 != 0.f ? e5 * __builtin_amdgcn_exp2f(-q.w) : 0.f;
    }
    __syncthreads();
    // then the atomics, (slot, component) interleaved: the six geometric sums
    // of a (view, Gaussian) share one 32-byte record and its colour sums one
    // 16-byte record, so neighbouring lanes' atomics fall in few cache lines;
    // each consumed entry is cleared for the next batch
    for (int t = threadIdx.x; t < cnt * 9; t += NT) {
      const int j = t / 9, c = t - j * 9;
      const float s = part[c * kPart + j];
      part[c * kPart + j] = 0.f;
      if (s != 0.f) {
        const size_t o = st.sidx[j];
        float* const dst = c < 6 ? accG + o * kAccG + c : accC + o * kAccC + (c - 6);
        atomicAdd(dst, s);
      }
    }
  }
}

// The backward is held to 80 VGPRs (six waves per SIMD; the allocation
// granule is eight registers, so one register more would cost a wave).
template <int TILE, int DEPTH>
__global__ __launch_bounds__(TILE* TILE) __attribute__((amdgpu_waves_per_eu(6))) void k_blend_bwd(ViewTable vt,
                                                          const uint2* __restrict__ ranges,
                                                          const uint32_t* __restrict__ tval,
                                                          const float4* __restrict__ splat,
                                                          const float* __restrict__ finalT,
                                                          const uint32_t* __restrict__ ncon,
                                                          float* __restrict__ accG,
                                                          float* __restrict__ accC) {
  __shared__ BwdSmem<TILE, DEPTH> sm;
  bwd_tile<TILE, DEPTH>(sm, vt, blockIdx.x, ranges, tval, splat, finalT, ncon, accG, accC);
}

template <int TILE, int DEPTH>
__global__ __launch_bounds__(TILE* TILE) __attribute__((amdgpu_waves_per_eu(6))) void k_blend_bwd_persistent(
    ViewTable vt, const uint2* __restrict__ ranges, const uint32_t* __restrict__ tval,
    const float4* __restrict__ splat, const float* __restrict__ finalT,
    const uint32_t* __restrict__ ncon, float* __restrict__ accG, float* __restrict__ accC,
    const uint32_t* __restrict__ order, uint32_t* counter) {
  __shared__ BwdSmem<TILE, DEPTH> sm;
  __shared__ uint32_t slot;
  for (;;) {
    const int gt = next_tile(counter, order, vt.total_tiles, &slot);
    if (gt < 0) break;
    bwd_tile<TILE, DEPTH>(sm, vt, gt, ranges, tval, splat, finalT, ncon, accG, accC);
  }
}

// Workgroups of a persistent kernel that are resident at once on the device.
template <class K>
int resident_grid(K kernel, int threads, const Ctx* ctx) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * ctx->cu_count;
}

template <int TILE, int DEPTH>
gs_status fwd_t(const ViewTable& vt, Frame& f, hipStream_t s) {
  if (f.persistent) {
    auto kern = k_blend_fwd_persistent<TILE, DEPTH>;
    const int grid = std::min(resident_grid(kern, TILE * TILE, f.ctx), vt.total_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(TILE * TILE), 0, s, vt, (const uint2*)f.ranges.p,
                       (const uint32_t*)f.tval[f.tkey_sel].p, (const float4*)f.splat.p,
                       (float*)f.finalT.p, (uint32_t*)f.ncon.p, f.tile_order,
                       (uint32_t*)f.words.p + kWordFwdCounter);
    GS_LAUNCHED("blend_fwd_persistent");
    return GS_OK;
  }
  hipLaunchKernelGGL((k_blend_fwd<TILE, DEPTH>), dim3(vt.total_tiles), dim3(TILE * TILE), 0, s,
                     vt, (const uint2*)f.ranges.p, (const uint32_t*)f.tval[f.tkey_sel].p,
                     (const float4*)f.splat.p, (float*)f.finalT.p, (uint32_t*)f.ncon.p);
  GS_LAUNCHED("blend_fwd");
  return GS_OK;
}

template <int TILE, int DEPTH>
gs_status bwd_t(const ViewTable& vt, Frame& f, hipStream_t s) {
  float* accG = (float*)f.acc.p;
  float* accC = accG + (size_t)f.views * (size_t)f.n * kAccG;
  if (f.persistent) {
    auto kern = k_blend_bwd_persistent<TILE, DEPTH>;
    const int grid = std::min(resident_grid(kern, TILE * TILE, f.ctx), vt.total_tiles);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(TILE * TILE), 0, s, vt, (const uint2*)f.ranges.p,
                       (const uint32_t*)f.tval[f.tkey_sel].p, (const float4*)f.splat.p,
                       (const float*)f.finalT.p, (const uint32_t*)f.ncon.p, accG, accC,
                       f.tile_order, (uint32_t*)f.words.p + kWordBwdCounter);
    GS_LAUNCHED("blend_bwd_persistent");
    return GS_OK;
  }
  hipLaunchKernelGGL((k_blend_bwd<TILE, DEPTH>), dim3(vt.total_tiles), dim3(TILE * TILE), 0, s,
                     vt, (const uint2*)f.ranges.p, (const uint32_t*)f.tval[f.tkey_sel].p,
                     (const float4*)f.splat.p, (const float*)f.finalT.p,
                     (const uint32_t*)f.ncon.p, accG, accC);
  GS_LAUNCHED("blend_bwd");
  return GS_OK;
}

__global__ __launch_bounds__(256) void k_export_screen_grads(const float* __restrict__ accG,
                                                             const float* __restrict__ accC,
                                                             size_t count, float* __restrict__ dst) {
  const size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (r >= count) return;
  const float4 g0 = reinterpret_cast<const float4*>(accG)[2 * r];
  const float4 g1 = reinterpret_cast<const float4*>(accG)[2 * r + 1];
  const float4 c = reinterpret_cast<const float4*>(accC)[r];
  float4* o = reinterpret_cast<float4*>(dst) + 3 * r;
  o[0] = g0;
  o[1] = make_float4(g1.x, g1.y, c.x, c.y);
  o[2] = make_float4(c.z, 0.f, 0.f, 0.f);
}

#define GS_DISPATCH(FN, tile, depth, ...)                                   \
  switch (tile * 1000 + depth) {                                            \
    case 8032: return FN<8, 32>(__VA_ARGS__);                               \
    case 8064: return FN<8, 64>(__VA_ARGS__);                               \
    case 16032: return FN<16, 32>(__VA_ARGS__);                             \
    case 16064: return FN<16, 64>(__VA_ARGS__);                             \
    case 16128: return FN<16, 128>(__VA_ARGS__);                            \
    case 16256: return FN<16, 256>(__VA_ARGS__);                            \
    case 32032: return FN<32, 32>(__VA_ARGS__);                             \
    case 32064: return FN<32, 64>(__VA_ARGS__);                             \
    case 32128: return FN<32, 128>(__VA_ARGS__);                            \
    case 32256: return FN<32, 256>(__VA_ARGS__);                            \
    default:                                                                \
      set_error("unsupported tile %d / lds depth %d", tile, depth);         \
      return GS_ERR_UNSUPPORTED;                                            \
  }

}  // namespace

gs_status launch_blend_fwd(const ViewTable& vt, Frame& f, hipStream_t s) {
  GS_DISPATCH(fwd_t, f.tile, f.depth, vt, f, s)
}

gs_status launch_blend_bwd(const ViewTable& vt, Frame& f, hipStream_t s) {
  GS_DISPATCH(bwd_t, f.tile, f.depth, vt, f, s)
}

gs_status launch_export_screen_grads(Frame& f, int view, float* dst, hipStream_t s) {
  const size_t n = (size_t)f.n;
  const float* accG = (const float*)f.acc.p;
  const float* accC = accG + (size_t)f.views * n * kAccG;
  size_t first = 0, count = (size_t)f.views * n;
  if (view >= 0) {
    first = (size_t)view * n;
    count = n;
  }
  if (count == 0) return GS_OK;
  hipLaunchKernelGGL(k_export_screen_grads, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     s, accG + first * kAccG, accC + first * kAccC, count, dst);
  GS_LAUNCHED("export_screen_grads");
  return GS_OK;
}

}  // namespace isogs
