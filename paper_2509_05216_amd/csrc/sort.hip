// Tile binning: exclusive scan of per-Gaussian tile counts, record emission,
// a stable LSD radix sort of (u32 key, u32 value) pairs, and per-tile ranges.
//
// Order contract: records sorted by the 64-bit key (tile << 32) | depth bits,
// ties by (view * N + Gaussian index).  The LSD sort of that key is split in
// two: the 32 low (depth) digits are sorted once per (view, Gaussian) — every
// record of a Gaussian shares its depth — and records are then emitted in that
// order, so only the tile digits are sorted over the K records.  The result is
// the same permutation an LSD sort of the full 64-bit key over the emitted
// records gives, at a fraction of the traffic.
//
// Radix passes use 8-bit digits, 256 threads (4 waves of 64) and 16 keys per
// thread per block.  Stable ranking inside a block uses wave ballots: for each
// item slot the lanes holding the same digit are found with 8 ballots, the
// group's leader bumps a per-wave LDS counter, and lanes take their rank from
// the popcount of lower peer lanes.
#include "internal.h"

namespace isogs {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 16;
constexpr int kChunk = kThreads * kItems;  // 4096 elements per block
constexpr int kRadix = 256;

__device__ inline uint32_t load_n(uint32_t n_max, const uint32_t* d_n) {
  if (d_n == nullptr) return n_max;
  const uint32_t c = *d_n;
  return c < n_max ? c : n_max;
}

__device__ inline uint64_t lanemask_lt() {
  const int lane = __lane_id();
  return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

// ---------------------------------------------------------------- block scan
// Exclusive scan of one u64 value per thread over a 256-thread block.
__device__ inline uint64_t block_exclusive_scan(uint64_t x, uint64_t* sh_waves, uint64_t& total) {
  const int lane = __lane_id();
  const int wave = threadIdx.x / 64;
  uint64_t inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  if (lane == 63) sh_waves[wave] = inc;
  __syncthreads();
  uint64_t before = 0;
  total = 0;
  for (int w = 0; w < kWaves; ++w) {
    const uint64_t s = sh_waves[w];
    if (w < wave) before += s;
    total += s;
  }
  __syncthreads();
  return before + inc - x;
}


struct ArrayIn {
  const uint32_t* a;
  __device__ uint32_t operator()(uint32_t i) const { return a[i]; }
};

template <class F>
__global__ __launch_bounds__(kThreads) void k_scan_reduce(F f, uint32_t n, uint64_t* partial) {
  __shared__ uint64_t sw[kWaves];
  const uint32_t base = blockIdx.x * (uint32_t)kChunk;
  uint64_t s = 0;
#pragma unroll 4
  for (int j = 0; j < kItems; ++j) {
    const uint32_t i = base + j * kThreads + threadIdx.x;
    if (i < n) s += f(i);
  }
  uint64_t total;
  block_exclusive_scan(s, sw, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan, in place, of the nb block totals by one block (each thread a
// contiguous run); the grand total goes to d_total when given.  Used when there
// are too many blocks for the down-sweep to sum its predecessors itself.
__global__ __launch_bounds__(kThreads) void k_scan_partials(uint64_t* partial, uint32_t nb,
                                                            uint64_t* d_total) {
  __shared__ uint64_t sw[kWaves];
  const uint32_t per = (nb + kThreads - 1) / kThreads;
  const uint32_t lo = min(nb, threadIdx.x * per), hi = min(nb, lo + per);
  uint64_t s = 0;
  for (uint32_t j = lo; j < hi; ++j) s += partial[j];
  uint64_t total;
  uint64_t run = block_exclusive_scan(s, sw, total);
  for (uint32_t j = lo; j < hi; ++j) {
    const uint64_t v = partial[j];
    partial[j] = run;
    run += v;
  }
  if (d_total != nullptr && threadIdx.x == 0) *d_total = total;
}

// Down-sweep.  With few blocks each forms its carry-in by summing the totals of
// the blocks before it (read from L2), so no separate scan of the totals is
// launched, and the last block writes the grand total when d_total is given;
// with many (prescanned), k_scan_partials has already turned the totals into
// the carries and written the grand total.
template <class F>
__global__ __launch_bounds__(kThreads) void k_scan_down(F f, uint32_t n, const uint64_t* partial,
                                                        uint32_t* out, uint64_t* d_total,
                                                        int prescanned) {
  __shared__ uint64_t sw[kWaves];
  // striped (coalesced) loads and stores, transposed through LDS so that each
  // thread scans kItems consecutive elements; one pad word per 32 avoids bank conflicts
  __shared__ uint32_t buf[kChunk + kChunk / 32];
  const uint32_t base = blockIdx.x * (uint32_t)kChunk;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t p = j * kThreads + threadIdx.x;
    const uint32_t i = base + p;
    buf[p + (p >> 5)] = (i < n) ? f(i) : 0u;
  }
  __syncthreads();
  uint32_t v[kItems];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t p = threadIdx.x * kItems + j;
    v[j] = buf[p + (p >> 5)];
    s += v[j];
  }
  uint64_t ctot;
  if (prescanned) {
    ctot = partial[blockIdx.x];
  } else {
    uint64_t carry = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kThreads) carry += partial[b];
    block_exclusive_scan(carry, sw, ctot);  // ctot: the sum over all threads
  }
  uint64_t total;
  uint64_t run = block_exclusive_scan(s, sw, total) + ctot;
  if (!prescanned && d_total != nullptr && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    *d_total = ctot + total;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t p = threadIdx.x * kItems + j;
    buf[p + (p >> 5)] = (uint32_t)run;
    run += v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t p = j * kThreads + threadIdx.x;
    const uint32_t i = base + p;
    if (i < n) out[i] = buf[p + (p >> 5)];
  }
}

// The one random gather of the rectangles: the tile count of every (view,
// Gaussian) entry in depth order, and the rectangles themselves in that order
// for the emission.
__global__ __launch_bounds__(256) void k_counts(const uint32_t* __restrict__ sidx,
                                                const uint2* __restrict__ rect, uint32_t n,
                                                uint32_t* __restrict__ counts,
                                                uint32_t* __restrict__ srx,
                                                uint32_t* __restrict__ sry) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint2 r = rect[sidx[i]];
  srx[i] = r.x;
  sry[i] = r.y;
  const int x0 = (int)(r.x & 0xffffu), y0 = (int)(r.x >> 16);
  const int x1 = (int)(r.y & 0xffffu), y1 = (int)(r.y >> 16);
  counts[i] = (x1 < x0 || y1 < y0) ? 0u : (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
}

// ---------------------------------------------------------------- radix sort
// Chunk of this block (grid of nblocks blocks).  Workgroups go to the eight
// XCDs in turn, so consecutive block indices land in different L2s; this
// bijection gives each XCD a contiguous run of chunks instead (the last
// nblocks % 8 keep their place).
__device__ inline uint32_t xcd_chunk(uint32_t nblocks) {
  const uint32_t n8 = nblocks / 8;
  return blockIdx.x < 8 * n8 ? (blockIdx.x % 8) * n8 + blockIdx.x / 8 : blockIdx.x;
}

__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                         uint32_t n_max, const uint32_t* d_n,
                                                         int shift, uint32_t nblocks,
                                                         uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kWaves][kRadix];
  const int wave = threadIdx.x / 64, lane = __lane_id();
  for (int d = threadIdx.x; d < kWaves * kRadix; d += kThreads) (&h[0][0])[d] = 0;
  __syncthreads();
  const uint32_t n = load_n(n_max, d_n);
  // chunk of this block: XCD-contiguous as in k_radix_scatter, so that the
  // counts of neighbouring chunks, adjacent in every digit's row of the table,
  // are written through the same L2
  const uint32_t chunk = xcd_chunk(nblocks);
  // the wave's 1024 keys as four 16-byte reads per lane, all issued before the
  // counting (the order of counting does not matter)
  const uint32_t base = chunk * (uint32_t)kChunk + wave * 64 * kItems;
  uint4 q[kItems / 4];
#pragma unroll
  for (int j = 0; j < kItems / 4; ++j) {
    const uint32_t i = base + 4u * (j * 64 + lane);
    if (i + 4 <= n) {
      q[j] = *reinterpret_cast<const uint4*>(keys + i);
    } else {  // tail: absent keys marked ~0 and skipped below
      q[j].x = i < n ? keys[i] : ~0u;
      q[j].y = i + 1 < n ? keys[i + 1] : ~0u;
      q[j].z = i + 2 < n ? keys[i + 2] : ~0u;
      q[j].w = ~0u;
    }
  }
  // A digit shared by many lanes of the wave (the high bytes of depths, the
  // tile rows of neighbouring records) would serialise their LDS atomics on one
  // word: the lanes holding lane 0's digit, and those holding the digit of the
  // first lane left, are counted by one atomic each; the rest add one apiece.
#pragma unroll
  for (int j = 0; j < kItems / 4; ++j) {
    const uint32_t i = base + 4u * (j * 64 + lane);
    const uint32_t kk[4] = {q[j].x, q[j].y, q[j].z, q[j].w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool ok = i + u < n;
      const uint32_t d = (kk[u] >> shift) & 0xffu;
      const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
      const uint64_t m0 = __builtin_amdgcn_ballot_w64(ok && d == d0);
      const uint64_t r0 = __builtin_amdgcn_ballot_w64(ok && d != d0);
      uint32_t d1 = 0x100u;  // no digit
      uint64_t m1 = 0;
      if (r0 != 0) {
        d1 = (uint32_t)__builtin_amdgcn_readlane((int)d, __builtin_ctzll(r0));
        m1 = __builtin_amdgcn_ballot_w64(ok && d == d1);
      }
      if (lane == 0) {
        if (m0 != 0) atomicAdd(&h[wave][d0], (uint32_t)__popcll(m0));
        if (m1 != 0) atomicAdd(&h[wave][d1], (uint32_t)__popcll(m1));
      }
      if (ok && d != d0 && d != d1) atomicAdd(&h[wave][d], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kThreads) {
    uint32_t s = 0;
    for (int w = 0; w < kWaves; ++w) s += h[w][d];
    hist[(size_t)d * nblocks + chunk] = s;
  }
}

// One pass of the stable LSD sort.  Each block ranks its 4096 elements by
// digit (wave ballots, stable), places them in LDS in block-local digit order,
// and writes them out so that consecutive threads store consecutive addresses
// of one digit's run: the global writes are coalesced.
static_assert(kThreads == kRadix, "one thread per digit in the offset scan");

__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, uint32_t n_max, const uint32_t* d_n, int shift, uint32_t nblocks,
    const uint32_t* __restrict__ hist_scanned) {
  __shared__ uint32_t cnt[kWaves][kRadix];
  __shared__ uint32_t gofs[kRadix];    // global position of local index 0 of digit d's run
  __shared__ uint32_t lstart[kRadix];  // block-local start of digit d
  __shared__ uint64_t scan_tmp[kWaves];
  __shared__ uint32_t sk[kChunk], sv[kChunk];
  const int wave = threadIdx.x / 64, lane = __lane_id();
  for (int d = threadIdx.x; d < kWaves * kRadix; d += kThreads) (&cnt[0][0])[d] = 0;
  const uint32_t n = load_n(n_max, d_n);
  // the runs that neighbouring chunks write for one digit, adjacent in the
  // output, meet in the same L2, and the cache lines they share are written
  // back whole
  const uint32_t chunk = xcd_chunk(nblocks);
  const uint32_t base = chunk * (uint32_t)kChunk + wave * 64 * kItems;
  if (chunk * (uint32_t)kChunk >= n) return;  // whole block empty (uniform)
  uint32_t key[kItems], val[kItems], rank[kItems];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t i = base + j * 64 + lane;
    const bool ok = i < n;
    key[j] = ok ? kin[i] : 0u;
    val[j] = ok ? (vin != nullptr ? vin[i] : i) : 0u;
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t i = base + j * 64 + lane;
    const bool ok = i < n;
    const uint32_t d = (key[j] >> shift) & 0xffu;
    // lanes with the same digit: for every bit, the ballot of the bit where the
    // lane's bit is set, its complement where it is clear, on the two 32-bit
    // halves (sbit: the bit sign-extended, 0 or all ones)
    const uint64_t okm = __builtin_amdgcn_ballot_w64(ok);
    uint32_t plo = (uint32_t)okm, phi = (uint32_t)(okm >> 32);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int32_t sbit = (int32_t)(d << (31 - b)) >> 31;
      const uint64_t bb = __builtin_amdgcn_ballot_w64(sbit != 0);
      plo &= ~((uint32_t)bb ^ (uint32_t)sbit);
      phi &= ~((uint32_t)(bb >> 32) ^ (uint32_t)sbit);
    }
    const uint64_t peers = ((uint64_t)phi << 32) | plo;
    uint32_t old = 0;
    const int leader = 63 - __clzll((long long)peers);
    if (ok && lane == leader) {
      old = cnt[wave][d];
      cnt[wave][d] = old + (uint32_t)__popcll(peers);
    }
    old = __shfl(old, ok ? leader : lane, 64);
    rank[j] = old + (uint32_t)__popcll(peers & lt);
  }
  __syncthreads();
  {
    // thread d: wave prefixes of digit d, the block-local start of d and its
    // global position (unsigned wrap-around is intended in gofs - start)
    const int d = threadIdx.x;
    uint32_t run = 0;
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = cnt[w][d];
      cnt[w][d] = run;
      run += c;
    }
    uint64_t total;
    const uint32_t start = (uint32_t)block_exclusive_scan(run, scan_tmp, total);
    lstart[d] = start;
    gofs[d] = hist_scanned[(size_t)d * nblocks + chunk] - start;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const uint32_t i = base + j * 64 + lane;
    if (i < n) {
      const uint32_t d = (key[j] >> shift) & 0xffu;
      const uint32_t lp = lstart[d] + cnt[wave][d] + rank[j];
      sk[lp] = key[j];
      sv[lp] = val[j];
    }
  }
  __syncthreads();
  const uint32_t nloc = min((uint32_t)kChunk, n - chunk * (uint32_t)kChunk);
  for (uint32_t t = threadIdx.x; t < nloc; t += kThreads) {
    const uint32_t k = sk[t];
    const uint32_t pos = gofs[(k >> shift) & 0xffu] + t;
    kout[pos] = k;
    vout[pos] = sv[t];
  }
}

// ---------------------------------------------------------------- emission
// Records of every (view, Gaussian) entry in depth order: (global tile, entry)
// for each tile of its rectangle, row by row.  A wave writes its 64 entries'
// records together: lane r of a pass takes the wave's record r (the owning
// entry found by a search over the wave's prefix sums of record counts), so
// each pass stores 64 consecutive records and no lane idles behind a large
// rectangle.  An entry whose records would pass the capacity writes none and
// sets the overflow word.
__global__ __launch_bounds__(256) void k_emit(ViewTable vt,
                                              const uint32_t* __restrict__ sidx,
                                              const uint32_t* __restrict__ srx,
                                              const uint32_t* __restrict__ sry,
                                              const uint32_t* __restrict__ offs, uint32_t count,
                                              uint32_t cap, uint32_t* __restrict__ tkey,
                                              uint32_t* __restrict__ tval,
                                              uint32_t* overflow) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = __lane_id();
  uint32_t need = 0, o = 0, idx = 0, key0 = 0, w = 1, tx = 0;
  if (i < count) {
    idx = sidx[i];
    const uint2 r = make_uint2(srx[i], sry[i]);  // rect[idx], gathered in depth order by k_counts
    const int x0 = (int)(r.x & 0xffffu), y0 = (int)(r.x >> 16);
    const int x1 = (int)(r.y & 0xffffu), y1 = (int)(r.y >> 16);
    if (x1 >= x0 && y1 >= y0) {
      const int v = view_of_entry(vt, idx);
      tx = (uint32_t)vt.v[v].tiles_x;
      o = offs[i];
      const uint32_t nd = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
      if ((uint64_t)o + nd > cap) {
        if (overflow != nullptr) *overflow = 1u;
      } else {
        need = nd;
        w = (uint32_t)(x1 - x0 + 1);
        key0 = (uint32_t)vt.v[v].tile_offset + (uint32_t)y0 * tx + (uint32_t)x0;
      }
    }
  }
  // exclusive prefix of the record counts over the wave, and the wave total
  uint32_t incl = need;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = (uint32_t)__shfl_up((int)incl, d, 64);
    if (lane >= d) incl += t;
  }
  const uint32_t excl = incl - need;
  const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
  // wave-uniform passes (every lane takes part in the shuffles)
  for (uint32_t base = 0; base < total; base += 64) {
    const uint32_t rr = base + (uint32_t)lane;
    const bool act = rr < total;
    // owner: the largest lane l with excl_l <= rr (never a lane without records)
    int l = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
      const int c = l + step;
      const uint32_t e = (uint32_t)__shfl((int)excl, c, 64);
      if (e <= rr) l = c;
    }
    const uint32_t li = rr - (uint32_t)__shfl((int)excl, l, 64);
    const uint32_t wl = (uint32_t)__shfl((int)w, l, 64);
    const uint32_t txl = (uint32_t)__shfl((int)tx, l, 64);
    const uint32_t k0 = (uint32_t)__shfl((int)key0, l, 64);
    const uint32_t ol = (uint32_t)__shfl((int)o, l, 64);
    const uint32_t il = (uint32_t)__shfl((int)idx, l, 64);
    if (act) {
      // row and column of the record in its rectangle: a float reciprocal
      // estimate of li / wl is off by at most one below 2^20, so one step
      // corrects it (exact integer division beyond)
      uint32_t yy;
      if (li < (1u << 20)) {
        yy = (uint32_t)((float)li * __builtin_amdgcn_rcpf((float)wl));
        const int32_t rem = (int32_t)(li - yy * wl);
        yy = rem < 0 ? yy - 1u : (rem >= (int32_t)wl ? yy + 1u : yy);
      } else {
        yy = li / wl;
      }
      const uint32_t xx = li - yy * wl;
      tkey[ol + li] = k0 + yy * txl + xx;
      tval[ol + li] = il;
    }
  }
}

// Per-tile [start, end) of the sorted keys: four keys per thread (one 16-byte
// read, plus the neighbours on either side); a run boundary sets the range.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tkey, uint32_t K_max,
                                                const uint32_t* d_K, uint2* __restrict__ ranges) {
  const uint32_t k0 = 4u * (blockIdx.x * blockDim.x + threadIdx.x);
  const uint32_t K = load_n(K_max, d_K);
  if (k0 >= K) return;
  uint32_t t[6];  // keys k0 - 1 .. k0 + 4 (~0 outside [0, K): differs from every tile)
  t[0] = k0 > 0 ? tkey[k0 - 1] : ~0u;
  if (k0 + 4 <= K) {
    const uint4 q = *reinterpret_cast<const uint4*>(tkey + k0);
    t[1] = q.x;
    t[2] = q.y;
    t[3] = q.z;
    t[4] = q.w;
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u + 1] = k0 + u < K ? tkey[k0 + u] : ~0u;
  }
  t[5] = k0 + 4 < K ? tkey[k0 + 4] : ~0u;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const uint32_t k = k0 + u;
    if (k >= K) break;
    if (t[u] != t[u + 1]) ranges[t[u + 1]].x = k;
    if (t[u + 2] != t[u + 1]) ranges[t[u + 1]].y = k + 1;
  }
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint32_t value, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_clamp_count(const uint64_t* __restrict__ total, uint32_t cap,
                              uint32_t* __restrict__ K, uint32_t* __restrict__ overflow) {
  const uint64_t t = *total;
  *K = t < cap ? (uint32_t)t : cap;
  if (t > cap) *overflow = 1u;
}

// Sort key of a tile for the longest-first work queue: 255 minus a log-scale
// length class (16 classes per octave of length + 1, lengths up to 2^16 - 1
// distinguished), so one 8-bit pass orders the tiles by length to within 1/16
// of an octave, which is all the schedule needs.
__global__ __launch_bounds__(256) void k_tile_len_keys(const uint2* __restrict__ ranges,
                                                       uint32_t tiles, uint32_t* __restrict__ key) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tiles) return;
  const uint2 r = ranges[t];
  const uint32_t x = r.y - r.x + 1u;                      // >= 1
  const uint32_t e = 31u - (uint32_t)__clz((int)x);       // floor(log2 x)
  const uint32_t m = ((x << (31u - e)) >> 27) & 15u;      // next four bits after the leading one
  const uint32_t cls = e * 16u + m;
  key[t] = 255u - (cls < 255u ? cls : 255u);
}

__global__ __launch_bounds__(256) void k_export_keys(const uint32_t* __restrict__ tkey,
                                                     const uint32_t* __restrict__ tval,
                                                     const uint32_t* __restrict__ dkey, uint32_t K,
                                                     uint64_t* __restrict__ out) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  out[k] = ((uint64_t)tkey[k] << 32) | (uint64_t)dkey[tval[k]];
}

inline uint32_t nblocks_of(uint32_t n) {
  return (uint32_t)(((uint64_t)n + kChunk - 1) / kChunk);
}

// The scanned digit table of a sort's last pass holds, at (digit d, chunk 0),
// the number of keys whose top byte is below d.  After a depth sort (positive
// float32 depths, untouched entries keyed 0xffffffff) the entry of digit 0xff
// is the count of touched entries; an empty table (every key below 0xff) gives n.
__global__ void k_visible_count(const uint32_t* __restrict__ hist_scanned, uint32_t nblocks,
                                uint32_t n, uint32_t* __restrict__ dst) {
  const uint32_t below = hist_scanned[(size_t)255 * nblocks];
  *dst = below <= n ? below : n;
}

}  // namespace

gs_status launch_fill_u32(void* p, uint32_t value, size_t count, hipStream_t s) {
  if (count == 0) return GS_OK;
  size_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, value,
                     count);
  GS_LAUNCHED("fill_u32");
  return GS_OK;
}

// Exclusive scan of f over n values into out (in place when out is f's array):
// block totals, then either the down-sweep summing its predecessors (up to
// kDirectBlocks blocks) or a one-block scan of the totals first.
constexpr uint32_t kDirectBlocks = 2048;

static gs_status scan_launch(ArrayIn f, uint32_t n, uint64_t* partial, uint32_t* out,
                             uint64_t* d_total, hipStream_t s) {
  const uint32_t nb = nblocks_of(n);
  hipLaunchKernelGGL(k_scan_reduce<ArrayIn>, dim3(nb), dim3(kThreads), 0, s, f, n, partial);
  GS_LAUNCHED("scan_reduce");
  const int pre = nb > kDirectBlocks ? 1 : 0;
  if (pre) {
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, s, partial, nb, d_total);
    GS_LAUNCHED("scan_partials");
  }
  hipLaunchKernelGGL(k_scan_down<ArrayIn>, dim3(nb), dim3(kThreads), 0, s, f, n,
                     (const uint64_t*)partial, out, d_total, pre);
  GS_LAUNCHED("scan_down");
  return GS_OK;
}

static gs_status ensure_scratch(Ctx* ctx, SortScratch& ss, uint32_t nb, size_t hist_entries,
                                hipStream_t s) {
  gs_status st = buf_ensure(ctx, ss.partial, sizeof(uint64_t) * (size_t)(nb + 1), s, ss.prior);
  if (st != GS_OK) return st;
  st = buf_ensure(ctx, ss.total, sizeof(uint64_t) * 2, s, ss.prior);
  if (st != GS_OK) return st;
  return buf_ensure(ctx, ss.hist, sizeof(uint32_t) * (hist_entries + 1), s, ss.prior);
}

gs_status scan_tile_counts(Ctx* ctx, SortScratch& ss, const uint32_t* sidx, const uint2* rect,
                           uint32_t n, uint32_t* offs, uint32_t* srx, uint32_t* sry,
                           uint64_t* d_total, hipStream_t s) {
  const uint32_t nb = nblocks_of(n);
  gs_status st = ensure_scratch(ctx, ss, nb, 0, s);
  if (st != GS_OK) return st;
  // gather the counts once (random rect reads), then scan them in place, coalesced
  hipLaunchKernelGGL(k_counts, dim3((n + 255) / 256), dim3(256), 0, s, sidx, rect, n, offs, srx,
                     sry);
  GS_LAUNCHED("counts");
  return scan_launch(ArrayIn{offs}, n, (uint64_t*)ss.partial.p, offs, d_total, s);
}

gs_status sort_pairs_u32(Ctx* ctx, SortScratch& ss, const uint32_t* kin, const uint32_t* vin,
                         uint32_t* kA, uint32_t* vA, uint32_t* kB, uint32_t* vB, uint32_t n,
                         const uint32_t* d_n, int bits, int* result_in_b, hipStream_t s) {
  *result_in_b = 0;
  if (n == 0) return GS_OK;
  const uint32_t nb = nblocks_of(n);
  const uint32_t hist_n = (uint32_t)kRadix * nb;
  const uint32_t hb = nblocks_of(hist_n);
  gs_status st = ensure_scratch(ctx, ss, hb > nb ? hb : nb, hist_n, s);
  if (st != GS_OK) return st;
  auto* hist = (uint32_t*)ss.hist.p;
  auto* partial = (uint64_t*)ss.partial.p;
  uint32_t* kb[2] = {kA, kB};
  uint32_t* vb[2] = {vA, vB};
  const uint32_t* ki = kin;
  const uint32_t* vi = vin;
  int out = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kThreads), 0, s, ki, n, d_n, shift, nb, hist);
    GS_LAUNCHED("radix_hist");
    st = scan_launch(ArrayIn{hist}, hist_n, partial, hist, nullptr, s);
    if (st != GS_OK) return st;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kThreads), 0, s, ki, vi, kb[out], vb[out],
                       n, d_n, shift, nb, hist);
    GS_LAUNCHED("radix_scatter");
    ki = kb[out];
    vi = vb[out];
    *result_in_b = out;
    out ^= 1;
  }
  return GS_OK;
}

gs_status launch_emit(const ViewTable& vt, Frame& f, const uint32_t* sidx, const uint32_t* srx,
                      const uint32_t* sry, uint32_t count, uint32_t* overflow, hipStream_t s) {
  if (count == 0) return GS_OK;
  const size_t cap_bytes = f.tkey[0].cap < f.tval[0].cap ? f.tkey[0].cap : f.tval[0].cap;
  const uint32_t cap = (uint32_t)(cap_bytes / sizeof(uint32_t));
  hipLaunchKernelGGL(k_emit, dim3((count + 255) / 256), dim3(256), 0, s, vt, sidx, srx,
                     sry, (const uint32_t*)f.offs.p, count, cap, (uint32_t*)f.tkey[0].p,
                     (uint32_t*)f.tval[0].p, overflow);
  GS_LAUNCHED("emit");
  return GS_OK;
}

gs_status launch_ranges(Frame& f, uint32_t n_rec, const uint32_t* d_K, hipStream_t s) {
  gs_status st = launch_fill_u32(f.ranges.p, 0u, (size_t)f.vt.total_tiles * 2, s);
  if (st != GS_OK) return st;
  if (n_rec == 0) return GS_OK;
  const uint32_t quads = (n_rec + 3) / 4;
  hipLaunchKernelGGL(k_ranges, dim3((quads + 255) / 256), dim3(256), 0, s,
                     (const uint32_t*)f.tkey[f.tkey_sel].p, n_rec, d_K, (uint2*)f.ranges.p);
  GS_LAUNCHED("ranges");
  return GS_OK;
}

gs_status launch_clamp_count(const uint64_t* total, uint32_t cap, uint32_t* K,
                             uint32_t* overflow, hipStream_t s) {
  hipLaunchKernelGGL(k_clamp_count, dim3(1), dim3(1), 0, s, total, cap, K, overflow);
  GS_LAUNCHED("clamp_count");
  return GS_OK;
}

gs_status sort_reserve(Ctx* ctx, SortScratch& ss, uint32_t n, hipStream_t s) {
  const uint32_t nb = nblocks_of(n);
  const uint32_t hist_n = (uint32_t)kRadix * nb;
  const uint32_t hb = nblocks_of(hist_n);
  return ensure_scratch(ctx, ss, hb > nb ? hb : nb, hist_n, s);
}

gs_status launch_visible_count(const SortScratch& ss, uint32_t n, uint32_t* dst, hipStream_t s) {
  if (n == 0) return launch_fill_u32(dst, 0u, 1, s);
  hipLaunchKernelGGL(k_visible_count, dim3(1), dim3(1), 0, s, (const uint32_t*)ss.hist.p,
                     nblocks_of(n), n, dst);
  GS_LAUNCHED("visible_count");
  return GS_OK;
}

gs_status launch_tile_order(Frame& f, hipStream_t s) {
  const uint32_t tiles = (uint32_t)f.vt.total_tiles;
  for (int k = 0; k < 2; ++k) {
    gs_status st = buf_ensure(f.ctx, f.okey[k], (size_t)tiles * 4, s, f.last_use);
    if (st == GS_OK) st = buf_ensure(f.ctx, f.oval[k], (size_t)tiles * 4, s, f.last_use);
    if (st != GS_OK) return st;
  }
  // keys into okey[1]; the sort reads them and ping-pongs okey[0] <-> okey[1]
  hipLaunchKernelGGL(k_tile_len_keys, dim3((tiles + 255) / 256), dim3(256), 0, s,
                     (const uint2*)f.ranges.p, tiles, (uint32_t*)f.okey[1].p);
  GS_LAUNCHED("tile_len_keys");
  int in_b = 0;
  gs_status st = sort_pairs_u32(f.ctx, f.ss, (const uint32_t*)f.okey[1].p, nullptr,
                                (uint32_t*)f.okey[0].p, (uint32_t*)f.oval[0].p,
                                (uint32_t*)f.okey[1].p, (uint32_t*)f.oval[1].p, tiles, nullptr,
                                8, &in_b, s);
  if (st != GS_OK) return st;
  f.tile_order = (const uint32_t*)f.oval[in_b].p;
  return GS_OK;
}

gs_status launch_export_keys(Frame& f, uint64_t* dst, hipStream_t s) {
  if (f.K == 0) return GS_OK;
  hipLaunchKernelGGL(k_export_keys, dim3((unsigned)((f.K + 255) / 256)), dim3(256), 0, s,
                     (const uint32_t*)f.tkey[f.tkey_sel].p, (const uint32_t*)f.tval[f.tkey_sel].p,
                     (const uint32_t*)f.dkey.p, (uint32_t)f.K, dst);
  GS_LAUNCHED("export_keys");
  return GS_OK;
}

}  // namespace isogs
