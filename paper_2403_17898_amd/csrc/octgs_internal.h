// Internal declarations shared by the HIP translation units of liboctgs.
// Written for gfx950 (CDNA4): 64-lane wavefronts, 256-thread blocks of four
// waves, MFMA for the decode GEMMs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstring>

#include "../../include/octgs.h"

namespace octgs {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per block in every kernel
constexpr int kTile = 16;            // screen tile edge in pixels
constexpr int kChunk = 1024;         // elements per block in the two-pass compactions
constexpr int kChunkPerThread = kChunk / kBlock;  // 4
constexpr int kGroups = kChunk / 64;              // 64-element ballot groups per block
constexpr int kGaussFields = 14;
constexpr int kProjVec = 3;          // float4 records per projected Gaussian
constexpr int kMaxK = 16;

// FP32 -> BF16 bit pattern, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint64_t ballot(int pred) { return __ballot(pred); }

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  int l = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (l >= o) v += t;
  }
  return v;
}

// Cross-lane moves without LDS: DPP within 16-lane rows, permlane swaps
// across rows (gfx950).  Controls: quad_perm [1,0,3,2] = lane ^ 1, quad_perm
// [2,3,0,1] = lane ^ 2, row_half_mirror = 7 - lane within 8, row_ror:8 =
// lane ^ 8 within 16.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppRor8 = 0x128;

// (x, y) -> (x with rows 1, 3 replaced by y's rows 0, 2; y with rows 0, 2
// replaced by x's rows 1, 3): x + y sums lanes L and L ^ 16, keeping x's
// value in rows 0 and 2 and y's in rows 1 and 3.
__device__ __forceinline__ void swap16(uint32_t &x, uint32_t &y) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}
// The same across halves: x + y sums lanes L and L ^ 32, x's value in the
// lower half and y's in the upper.
__device__ __forceinline__ void swap32(uint32_t &x, uint32_t &y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}

// Sum over the wave, the same bits in every lane.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  v += dpp_u<kDppXor1>(v);
  v += dpp_u<kDppXor2>(v);
  v += dpp_u<kDppHalfMirror>(v);
  v += dpp_u<kDppRor8>(v);
  uint32_t x = v, y = v;
  swap16(x, y);
  v = x + y;
  x = v; y = v;
  swap32(x, y);
  return x + y;
}

__device__ __forceinline__ float wave_sum_f(float v) {
  v += __uint_as_float(dpp_u<kDppXor1>(__float_as_uint(v)));
  v += __uint_as_float(dpp_u<kDppXor2>(__float_as_uint(v)));
  v += __uint_as_float(dpp_u<kDppHalfMirror>(__float_as_uint(v)));
  v += __uint_as_float(dpp_u<kDppRor8>(__float_as_uint(v)));
  uint32_t x = __float_as_uint(v), y = x;
  swap16(x, y);
  v = __uint_as_float(x) + __uint_as_float(y);
  x = __float_as_uint(v); y = x;
  swap32(x, y);
  return __uint_as_float(x) + __uint_as_float(y);
}

// Block-wide exclusive scan of one value per thread (256 threads); returns
// the exclusive prefix and writes the block total to *total.  `tmp` is LDS of
// at least 4 words.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *tmp, uint32_t *total) {
  int w = threadIdx.x / kWave, l = __lane_id();
  uint32_t inc = wave_incl_scan(v);
  if (l == 63) tmp[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kWave; ++i) {
    uint32_t s = tmp[i];
    if (i < w) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// Sum of v over the 256 threads of a block, returned to thread 0 (LDS
// scratch of 4 floats).
__device__ __forceinline__ float block_sum_f(float v, float *red) {
  v = wave_sum_f(v);
  if (__lane_id() == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Sum of a[0..b) by the 256 threads of a block, returned per thread
// (partial sums; the caller reduces).  Loads are unconditional at a clamped
// index, four per thread per step, so they are in flight together.
__device__ __forceinline__ uint32_t partial_sum_prefix(const uint32_t *a, int b) {
  uint32_t s = 0;
  const int t = threadIdx.x;
  for (int i0 = 0; i0 < b; i0 += 4 * kBlock) {
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = a[min(i0 + u * kBlock + t, b - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) s += i0 + u * kBlock + t < b ? v[u] : 0u;
  }
  return s;
}

// Relaxed device-scope (all XCDs) atomics for look-back status words.
__device__ __forceinline__ uint32_t ld_acq(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile scheduling of the per-tile kernels (one block per tile).  Blocks are
// dealt round-robin over the 8 XCDs, so block b runs on XCD b % 8.  Tiles
// are grouped in squares of kTileGroup x kTileGroup and group g goes to XCD
// g % 8: every XCD gets groups from all over the image, which balances the
// dense and sparse regions of a view across the XCDs, while the tiles of one
// group, which share most of their Gaussians, stay in one L2.  On request
// (OCTGS_RASTER_TILE_ORDER) the rasterizer then orders each XCD's tiles by
// list length, longest first (k_tile_order), so its last blocks are short.
constexpr uint32_t kXcds = 8;
constexpr uint32_t kTileGroup = 4;
// Largest number of 16x16 tiles per image (about 4.3 gigapixels): tile ids,
// sort keys and the per-tile grids stay well inside 32 bits.
constexpr int64_t kMaxTiles = int64_t(1) << 24;
inline bool image_tiles_ok(int32_t width, int32_t height) {
  if (width <= 0 || height <= 0) return false;
  return (int64_t)((width + 15) / 16) * ((height + 15) / 16) <= kMaxTiles;
}

// Blocks to launch: 8 x kTileGroup^2 x ceil(groups / 8); the blocks past the
// last group and those on tiles outside a partial edge group exit at once.
__host__ __device__ inline uint32_t tile_grid_blocks(int tiles_x, int tiles_y) {
  const uint32_t gx = (tiles_x + kTileGroup - 1) / kTileGroup;
  const uint32_t gy = (tiles_y + kTileGroup - 1) / kTileGroup;
  return (gx * gy + kXcds - 1) / kXcds * kXcds * kTileGroup * kTileGroup;
}

// The tile of block bid, or -1 for a block without one.  A bijection from
// the blocks that have a tile onto the tiles.
__device__ __forceinline__ int32_t tile_of_block(uint32_t bid, int tiles_x, int tiles_y) {
  const uint32_t gx = (tiles_x + kTileGroup - 1) / kTileGroup;
  const uint32_t gy = (tiles_y + kTileGroup - 1) / kTileGroup;
  const uint32_t xcd = bid % kXcds, slot = bid / kXcds;
  const uint32_t g = xcd + kXcds * (slot / (kTileGroup * kTileGroup));
  const uint32_t w = slot % (kTileGroup * kTileGroup);
  if (g >= gx * gy) return -1;
  const uint32_t tx = (g % gx) * kTileGroup + w % kTileGroup;
  const uint32_t ty = (g / gx) * kTileGroup + w / kTileGroup;
  if (tx >= (uint32_t)tiles_x || ty >= (uint32_t)tiles_y) return -1;
  return (int32_t)(ty * (uint32_t)tiles_x + tx);
}

// ---------------------------------------------------------------------------
// rasterizer workspace
// ---------------------------------------------------------------------------

constexpr int kTicketScan = 0, kTicketEmit = 1, kTicketDepth = 2, kTicketTile = 6;
constexpr int kTicketSlots = 10;

struct RasterHeader {
  uint32_t n_slots, n_visible, n_pairs, pair_overflow, sync_error;
  uint32_t n_candidates;  // rectangle tiles of the survivors (saturated at 2^32 - 1)
  uint32_t n_cand_listed; // candidates written (n_candidates, or 0 on overflow)
  uint32_t n_listed;      // pairs in the sorted list (n_pairs, or 0 on overflow)
  uint32_t tile_ordered;  // 1 if the forward wrote tile_order (OCTGS_RASTER_TILE_ORDER)
  // partition tickets of the kernels chained by look-back: candidate scan,
  // emission, then the depth sort's 4 passes and the tile sort's passes
  uint32_t ticket[kTicketSlots];
  uint32_t reserved[23 - kTicketSlots];
};

struct RasterWs {
  RasterHeader *hdr;
  uint64_t *vis_mask;     // [gcap / 64]
  uint32_t *blk_cnt;      // [nblk_g]
  float4 *proj;           // [gcap][3]: (mx, my, A, B) (C, log2 opacity, r, g) (b, qa, qb, qc);
                          // A, B, C = conic scaled for exp2: -0.5 log2e ca, -log2e cb, -0.5 log2e cc;
                          // qa, qb, qc = the conic itself (tile test)
  uint32_t *depth;        // [gcap] float bits of camera z
  uint64_t *rect;         // [gcap] packed u16 x0, y0, x1, y1
  uint32_t *dkey[2];      // [gcap] depth-sort keys (ping-pong)
  uint32_t *dval[2];      // [gcap] depth-sort values = slot ids
  uint32_t *pair_off;     // [gcap] exclusive prefix of rectangle tiles, depth order
  uint32_t *lb_emit;      // [nblk_g] look-back status of the candidate scan's chunks
  uint32_t *run_first;    // [nruns] depth-order index of the survivor holding candidate kEmitRun r
  uint32_t *lb_pair;      // [nruns] look-back status of the emission's runs
  uint32_t *tkey[2];      // [pcap] tile keys (ping-pong)
  uint32_t *tval[2];      // [pcap] slot ids
  uint32_t *tpair[2];     // [pcap] each pair's emission index, carried by the tile sort
  uint32_t *pair_slot;    // [pcap] slot of each pair in emission order (a Gaussian's pairs
                          // are contiguous there)
  uint32_t *ranges;       // [tiles][2]
  uint32_t *tile_order;   // [tile_grid_blocks] tile of each compositing block (~0u: none),
                          // written only with OCTGS_RASTER_TILE_ORDER
  uint32_t *hist;         // [kHistCopies][8][256] radix histograms (4 depth passes, then 1..4
                          // tile passes); block b adds into copy b % kHistCopies
  uint32_t *lookback;     // [4][ceil(gcap / kSortPart)][256] depth-sort look-back
  uint32_t *lookback_t;   // [tile passes][ceil(pcap / kTileSortPart)][256] tile-sort look-back
  float *dproj;           // [gcap][9] backward: d(mx, my, ca, cb, cc, opacity, r, g, b)
  float *gpair;           // [pcap][9] backward: the same per (tile, Gaussian) pair, emission order
  float *chunk_part;      // [ceil(pcap / 64)][2][9] backward: sums of a 64-pair chunk's first and
                          // last run where the run crosses the chunk's start or end
  uint32_t *chunk_info;   // [ceil(pcap / 64)] backward: which of those the chunk has
  int64_t gcap, pcap;
  int32_t tiles_x, tiles_y, nblk_g, nruns, tile_passes;
  float xmax, ymax;            // last pixel centre of the image: W - 0.5, H - 0.5
  size_t lb_words, lbt_words;  // look-back words of the depth and tile sorts (all passes)
  int64_t lb_parts, lbt_parts; // partitions per pass at capacity
  size_t bytes;
};

// Producers spread their histogram atomics over this many copies (one per
// XCD for round-robin dispatch), which the sort sums: atomics on global
// memory are performed at the memory side, and one copy served by every
// block serialises them.
constexpr int kHistCopies = 8;
constexpr uint32_t kHistStride = 8 * 256;

constexpr int kEmitThreads = 1024;  // pair emission: threads per block
constexpr int kEmitRun = 8192;      // candidate pairs per block of the emission

RasterWs raster_layout(void *base, int64_t gcap, int64_t pcap, int32_t W, int32_t H);

// dst[i] = BF16 bits of src[i] rounded to nearest even, i < count (device
// arrays); enqueues one kernel on s.
hipError_t launch_round_bf16(const float *src, uint16_t *dst, int64_t count, hipStream_t s);
int tile_sort_passes(int ntiles);

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

struct CamParams {
  float R[9], C[3], fx, fy, cx, cy, z_near;
  int W, H;
};

// ---------------------------------------------------------------------------
// radix sort (Onesweep: one histogram pass, then one pass per digit with
// decoupled look-back across the partitions)
// ---------------------------------------------------------------------------

constexpr int kSortItems = 8;
constexpr int kSortPart = kBlock * kSortItems;  // 2048 keys per partition (depth sort)
// The tile sort has ~10x more keys: 4096-key partitions halve its blocks,
// and with them the same-address ticket atomics and the look-back chain.
constexpr int kTileSortItems = 16;
constexpr int kTileSortPart = kBlock * kTileSortItems;
constexpr uint32_t kSpinLimit = 1u << 22;       // look-back wait bound
// Look-back status of one sort pass: a row of 2 x 256 words per partition
// (the digits' aggregate, upgraded to the inclusive prefix, and a copy of the
// aggregate), then one row of 256 words per group of kGroupParts partitions.
constexpr int kGroupParts = 16;
constexpr int kLbRow = 512;
__host__ __device__ inline size_t lookback_pass_words(int64_t nparts) {
  const int64_t np = nparts < 1 ? 1 : nparts;
  return (size_t)np * kLbRow + (size_t)((np + kGroupParts - 1) / kGroupParts) * 256;
}

// Sort (keys, vals) of length *count (device) by bits [0, 8 * passes) of the
// key, stably.  On return the sorted data is in buffers index `passes % 2`.
// tickets: one zeroed word per pass, from which the pass's blocks take their
// partition index in the order they start.
// hist: the digit histograms of the passes, [passes][256] words, as the sum
// of hist_copies (1..kHistCopies) copies hist_stride words apart (built by
// the producer of the keys; the first pass folds the later passes' copies
// into copy 0); items: keys per thread of a partition (kSortItems or
// kTileSortItems; a partition is 256 * items keys); lookback:
// passes * lookback_pass_words(ceil(cap / (256 * items))) words, cleared by
// the producer for the partitions in use (clear_partitions).
hipError_t radix_sort(uint32_t *keys[2], uint32_t *vals[2], uint32_t *const *vals2,
                      const uint32_t *count, int64_t cap, int items, int passes, uint32_t *hist,
                      int hist_copies, uint32_t hist_stride, uint32_t *lookback,
                      uint32_t *tickets, uint32_t *err_flag, hipStream_t stream);

// ---------------------------------------------------------------------------
// chained scan: decoupled look-back over one value per partition
// ---------------------------------------------------------------------------

constexpr uint32_t kLbAgg = 1u << 30;       // status flag: partition aggregate
constexpr uint32_t kLbInc = 2u << 30;       // status flag: inclusive prefix
constexpr uint32_t kLbVal = (1u << 30) - 1;  // value bits; values saturate here

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
  const uint32_t s = a + b;  // a, b <= kLbVal, so no wrap
  return s > kLbVal ? kLbVal : s;
}

// Called by all 64 lanes of one wave.  Publishes partition `part`'s
// aggregate `agg` (<= kLbVal), sums the predecessors' values back to the
// nearest inclusive one, 64 partitions per round trip, publishes the
// inclusive value and returns the exclusive prefix (saturating at kLbVal).
// status[] must be zero before the first partition publishes.  A wait that
// exceeds kSpinLimit sets *err and returns what it has.
__device__ __forceinline__ uint32_t chained_lookback(uint32_t *status, uint32_t part, uint32_t agg,
                                                     uint32_t *err, uint32_t spin_limit) {
  const int l = __lane_id();
  if (l == 0) st_rel(&status[part], (part == 0 ? kLbInc : kLbAgg) | agg);
  uint32_t excl = 0;
  int64_t p = (int64_t)part - 1;
  uint32_t spins = 0;
  while (p >= 0) {
    const int64_t q = p - l;
    const uint32_t s = q >= 0 ? ld_acq(&status[q]) : kLbInc;  // before partition 0: inclusive 0
    const uint64_t ready = ballot((s & ~kLbVal) != 0u);
    const uint64_t inc = ballot((s & ~kLbVal) == kLbInc);
    const int first = inc ? __builtin_ctzll(inc) : 64;
    const uint64_t need = first < 63 ? ((2ull << first) - 1ull) : ~0ull;
    if ((ready & need) != need) {
      if (++spins > spin_limit) {
        if (l == 0) atomicOr(err, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    uint32_t v = ((need >> l) & 1ull) ? (s & kLbVal) : 0u;
    // saturating wave sum: 64 values of 30 bits fit in 36 bits
    uint64_t v64 = v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v64 += __shfl_xor(v64, o, 64);
    excl = sat_add(excl, (uint32_t)(v64 > kLbVal ? kLbVal : v64));
    if (first < 64) break;
    p -= 64;
  }
  if (l == 0 && part > 0) st_rel(&status[part], kLbInc | sat_add(excl, agg));
  return excl;
}


}  // namespace octgs
