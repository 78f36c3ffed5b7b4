// Backward pass of the rasterizer: gradients of a loss on the image with
// respect to each Gaussian's mean, scale, rotation, opacity and colour
// (the training step of Octree-GS renders and back-propagates through the
// Eq. 2 blending and the EWA projection of Sec. III-A).
//
// composite backward: one wave per 16x16 tile, four pixels per thread.  Each
// pixel starts from its final transmittance and walks its tile list in
// reverse from the last entry the forward consumed, recovering
// T_i = T_{i+1} / (1 - a_i) instead of storing per-pixel lists; the colour
// behind each entry is accumulated on the way.  Per-Gaussian gradients are
// summed over the thread's pixels and over the wave by a halving exchange,
// stored once per (tile, Gaussian) pair at the pair's emission index (plain
// stores: float atomics on global memory are performed at the memory side
// on this chip and were most of the pass's time), then summed per Gaussian
// over its contiguous run of pairs.
//
// projection backward: one thread per Gaussian slot, recomputing the forward
// quantities (rotation, 3D covariance, Jacobian, 2D covariance) in FP32.
#include "octgs_internal.h"

namespace octgs {

namespace {

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

struct BwdArgs {
  RasterWs ws;
  int buf, W, H;
  float alpha_max, alpha_min, bg[3];
  const float *T_final, *dimg;
  const uint32_t *last;
};

// Sum of 8 values over the 64 lanes of a wave, by halving exchanges: a
// permlane32 swap, a permlane16 swap and a DPP row rotation leave each lane
// one partial sum of value 4 b5 + 2 b4 + b3 (b = lane bits), and three DPP
// steps finish it within 8 lanes.  Lane 8 q returns the total of value q.
__device__ __forceinline__ float wave_sum8(const float (&v)[8], int &q) {
  const int l = __lane_id();
  float a[4], b[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint32_t x = __float_as_uint(v[i]), y = __float_as_uint(v[4 + i]);
    swap32(x, y);
    a[i] = __uint_as_float(x) + __uint_as_float(y);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    uint32_t x = __float_as_uint(a[i]), y = __float_as_uint(a[2 + i]);
    swap16(x, y);
    b[i] = __uint_as_float(x) + __uint_as_float(y);
  }
  const bool h3 = (l >> 3) & 1;
  float c = (h3 ? b[1] : b[0]) + __uint_as_float(dpp_u<kDppRor8>(__float_as_uint(h3 ? b[0] : b[1])));
  c += __uint_as_float(dpp_u<kDppXor1>(__float_as_uint(c)));
  c += __uint_as_float(dpp_u<kDppXor2>(__float_as_uint(c)));
  c += __uint_as_float(dpp_u<kDppHalfMirror>(__float_as_uint(c)));
  q = 4 * ((l >> 5) & 1) + 2 * ((l >> 4) & 1) + (int)h3;
  return c;
}

// Reverse replay of one tile by one wave (64 threads), four vertically
// adjacent pixels per thread, replaying the forward's per-pixel exponent
// sequence operation for operation, so every a_i is bit-identical to the
// forward's and T_i = T_{i+1} / (1 - a_i) retraces its transmittances.
constexpr int kBwdThreads = 64;
constexpr int kBwdBatch = 64;
constexpr int kBPx = 4;

struct BwdLds {
  float4 sA[kBwdBatch], sB[kBwdBatch], sC[kBwdBatch];
  uint32_t s_pair[kBwdBatch];
  float sG[9][kBwdBatch];
};

// Per-pair gradients of list entries [e0, e1) that no pixel consumed are 0.
__device__ __forceinline__ void zero_pairs(const RasterWs &ws, const uint32_t *pidx, uint32_t e0,
                                           uint32_t e1) {
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    float *gp = ws.gpair + 9 * (size_t)pidx[e];
#pragma unroll
    for (int k = 0; k < 9; ++k) gp[k] = 0.0f;
  }
}

// The LDS lives in the kernel and is passed in, so the two AMIN
// instantiations share one allocation.
template <bool AMIN>
__device__ __forceinline__ void composite_bwd_tile(const BwdArgs &a, BwdLds &lds) {
  float4 *sA = lds.sA, *sB = lds.sB, *sC = lds.sC;
  uint32_t *s_pair = lds.s_pair;
  float (*sG)[kBwdBatch] = lds.sG;
  // the tile order the forward used: its per-view order (a permutation of
  // the group mapping) if it wrote one, else the group mapping
  const int32_t tile = a.ws.hdr->tile_ordered
                           ? (int32_t)a.ws.tile_order[blockIdx.x]
                           : tile_of_block(blockIdx.x, a.ws.tiles_x, a.ws.tiles_y);
  if (tile < 0 || tile >= a.ws.tiles_x * a.ws.tiles_y) return;
  const int tx = tile % a.ws.tiles_x, ty = tile / a.ws.tiles_x;
  const int t = threadIdx.x, l = __lane_id();
  const int px = tx * kTile + (t % kTile), py0 = ty * kTile + kBPx * (t / kTile);
  const float fx = (float)px + 0.5f, fy = (float)py0 + 0.5f;
  const uint32_t start = a.ws.ranges[2 * tile], end = a.ws.ranges[2 * tile + 1];
  const uint32_t *vals = a.ws.tval[a.buf];   // slot of each sorted pair
  const uint32_t *pidx = a.ws.tpair[a.buf];  // its emission index
  const float4 *proj = a.ws.proj;
  const size_t plane = (size_t)a.W * a.H;
  // per pixel: T, dL/dC, S = dL/dC . (colour behind) (starts as T_final
  // dL/dC . bg; dL/dC is fixed per pixel, so the dot product is accumulated
  // instead of the colour), entries used
  float T[kBPx], dr[kBPx], dg[kBPx], db[kBPx], S[kBPx];
  uint32_t last[kBPx];
  uint32_t mx = 0;
#pragma unroll
  for (int k = 0; k < kBPx; ++k) {
    T[k] = 1.0f; dr[k] = 0.0f; dg[k] = 0.0f; db[k] = 0.0f; last[k] = 0;
    if (px < a.W && py0 + k < a.H) {
      const size_t pix = (size_t)(py0 + k) * a.W + px;
      T[k] = a.T_final[pix];
      last[k] = a.last[pix];
      dr[k] = a.dimg[pix];
      dg[k] = a.dimg[plane + pix];
      db[k] = a.dimg[2 * plane + pix];
    }
    S[k] = T[k] * fma_(a.bg[0], dr[k], fma_(a.bg[1], dg[k], a.bg[2] * db[k]));
    mx = max(mx, last[k]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, kWave));
  const uint32_t n_used = min(mx, end - start);
  const float amax = a.alpha_max, amin = a.alpha_min;
  zero_pairs(a.ws, pidx, start + n_used, end);
  if (n_used == 0) return;
  for (int32_t b0 = (int32_t)((n_used - 1) / kBwdBatch) * kBwdBatch; b0 >= 0; b0 -= kBwdBatch) {
    const int nb = (int)min((uint32_t)kBwdBatch, n_used - (uint32_t)b0);
    __syncthreads();  // one wave: orders the reuse of the batch buffers
#pragma unroll
    for (int q = 0; q < kBwdBatch / kBwdThreads; ++q) {
      const int i = t + q * kBwdThreads;
      const uint32_t e = start + (uint32_t)b0 + (uint32_t)min(i, nb - 1);
      const uint32_t s = vals[e];
      s_pair[i] = pidx[e];
      sA[i] = proj[3 * (size_t)s];
      const float4 bv = proj[3 * (size_t)s + 1];
      sB[i] = bv;
      float4 cv = proj[3 * (size_t)s + 2];
      cv.y = __builtin_amdgcn_exp2f(-bv.y);  // 1 / opacity, for dL/dop = dL/da a / op
      sC[i] = cv;
#pragma unroll
      for (int g = 0; g < 9; ++g) sG[g][i] = 0.0f;
    }
    __syncthreads();
    for (int j = nb - 1; j >= 0; --j) {
      const uint32_t li = (uint32_t)b0 + (uint32_t)j;  // index in the tile list
      const float4 A = sA[j];
      const float4 B = sB[j];
      const float4 Cc = sC[j];
      // the forward's sequence, so each a0 (= op G') is bit-identical to it
      const float dx = fx - A.x;
      const float adx = fma_(A.z * dx, dx, B.y);
      const float bdx = A.w * dx;
      const float dy = fy - A.y;
      float p = fma_(B.x * dy, dy, fma_(bdx, dy, adx));
      float d = fma_(B.x, fma_(2.0f, dy, 1.0f), bdx);
      const float c2 = B.x + B.x;
      // raw per-lane sums, turned into gradients once per (tile, Gaussian):
      // dq = dL/da a0 (0 where alpha is clamped); over the thread's pixels
      // k = 0..3 (dy = dy0 + k), D = sum dq, E = sum k dq, F = sum k^2 dq,
      // so sum dq dy = dy0 D + E and sum dq dy^2 = dy0^2 D + 2 dy0 E + F;
      // colour weights
      float D = 0.0f, E = 0.0f, F = 0.0f, wr = 0.0f, wg = 0.0f, wb = 0.0f;
      bool any = false;
#pragma unroll
      for (int k = 0; k < kBPx; ++k) {
        if (k > 0) {
          p += d;
          d += c2;
        }
        const float a0 = __builtin_amdgcn_exp2f(p);
        const float al = fminf(amax, a0);
        bool valid = li < last[k];
        if (AMIN) valid = valid && !(al < amin);
        if (valid) {
          any = true;
          const float inv1 = __builtin_amdgcn_rcpf(1.0f - al);
          const float Ti = T[k] * inv1;
          const float w = al * Ti;
          wr = fma_(w, dr[k], wr);
          wg = fma_(w, dg[k], wg);
          wb = fma_(w, db[k], wb);
          const float cdot = fma_(B.z, dr[k], fma_(B.w, dg[k], Cc.x * db[k]));
          const float dLda = Ti * cdot - S[k] * inv1;
          S[k] = fma_(w, cdot, S[k]);
          T[k] = Ti;
          const float dq = a0 <= amax ? dLda * a0 : 0.0f;
          D += dq;
          if (k > 0) {
            E = fma_((float)k, dq, E);
            F = fma_((float)(k * k), dq, F);
          }
        }
      }
      if (ballot(any) != 0ull) {
        int q;
        const float Sy = fma_(dy, D, E);
        const float Qyy = fma_(dy, fma_(dy, D, 2.0f * E), F);
        const float v8[8] = {D, D * dx, D * dx * dx, Sy, Sy * dx, Qyy, wr, wg};
        const float s8 = wave_sum8(v8, q);
        const float s9 = wave_sum_f(wb);
        if ((l & 7) == 0) sG[q][j] = s8;
        if (l == 0) sG[8][j] = s9;
      }
    }
    __syncthreads();
    // raw sums -> dL/d(mx, my, ca, cb, cc, op, r, g, b).  With dpw = ln2 dq
    // and p = A' dx^2 + B' dx dy + C' dy^2 (dx = x - mx):
    //   dmx = -(2 A' Sx + B' Sy) ln2, dmy = -(B' Sx + 2 C' Sy) ln2,
    //   d(ca, cb, cc) = ln2 (-log2e / 2 Qxx, -log2e Qxy, -log2e / 2 Qyy),
    //   dop = D / op
#pragma unroll
    for (int q = 0; q < kBwdBatch / kBwdThreads; ++q) {
      const int i = t + q * kBwdThreads;
      if (i < nb) {
        const float4 A = sA[i], B = sB[i], Cc = sC[i];
        const float D = sG[0][i], Sx = sG[1][i], Qxx = sG[2][i], Sy = sG[3][i];
        const float Qxy = sG[4][i], Qyy = sG[5][i];
        float g[9];
        g[0] = -kLn2 * fma_(2.0f * A.z, Sx, A.w * Sy);
        g[1] = -kLn2 * fma_(A.w, Sx, 2.0f * B.x * Sy);
        g[2] = -0.5f * Qxx;  // ln2 * log2e = 1
        g[3] = -Qxy;
        g[4] = -0.5f * Qyy;
        g[5] = D * Cc.y;
        g[6] = sG[6][i];
        g[7] = sG[7][i];
        g[8] = sG[8][i];
        float *gp = a.ws.gpair + 9 * (size_t)s_pair[i];
#pragma unroll
        for (int k = 0; k < 9; ++k) gp[k] = g[k];
      }
    }
  }
}

__global__ __launch_bounds__(kBwdThreads) void k_composite_bwd(BwdArgs a) {
  __shared__ BwdLds lds;
  {
    // the reduction writes the per-slot rows of Gaussians with pairs only;
    // the others must read zero, and this kernel does not touch the rows,
    // so its blocks clear them
    const uint64_t nz = (uint64_t)min<int64_t>(a.ws.hdr->n_slots, a.ws.gcap) * 9u;
    for (uint64_t i = (uint64_t)blockIdx.x * kBwdThreads + threadIdx.x; i < nz;
         i += (uint64_t)gridDim.x * kBwdThreads)
      a.ws.dproj[i] = 0.0f;
  }
  if (a.alpha_min > 0.0f)
    composite_bwd_tile<true>(a, lds);
  else
    composite_bwd_tile<false>(a, lds);
}

// v[k] += (the DPP-moved v[k]) where take holds; lanes the move does not
// reach (past a row's start, or outside row_mask) receive 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ void seg_step(float (&v)[9], bool take) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float u = __uint_as_float(
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)__float_as_uint(v[k]), CTRL, ROWMASK, 0xF, true));
    v[k] += take ? u : 0.0f;
  }
}

// Per-Gaussian sums of the per-pair gradients.  A Gaussian's pairs are
// contiguous in emission order.  Each wave takes a chunk of 64 consecutive
// pairs and runs a segmented inclusive scan keyed by slot (six DPP steps);
// the last lane of each run then holds the run's sum.  A run that lies inside
// the chunk is stored.  A run that crosses the chunk's start or end leaves
// its sum in the chunk's two partial slots (the first and the last run; one
// run covering the whole chunk is its first), and k_pair_fix adds a crossing
// run's partials in chunk order: no atomics, the same sums on every run.
constexpr uint32_t kChunkFirst = 1u;   // the chunk's first run continues from the previous chunk
constexpr uint32_t kChunkLast = 2u;    // its last run continues into the next chunk
constexpr uint32_t kChunkWhole = 4u;   // one run covers the chunk and continues both ways
__global__ __launch_bounds__(kBlock) void k_pair_reduce(RasterWs ws) {
  // a full chunk's 64 records (2,304 bytes, 16-byte aligned) are read with
  // lane-contiguous float4 loads into LDS, then each lane takes its own 9
  // floats (odd stride: no bank conflicts)
  constexpr int kRec4 = kWave * 9 / 4;  // 144
  __shared__ float4 stage[kBlock / kWave][kRec4];
  const uint32_t P = ws.hdr->n_listed;
  const int l = __lane_id();
  const uint32_t nw = gridDim.x * (kBlock / kWave);
  float4 *sw = stage[threadIdx.x / kWave];
  for (uint32_t c0 = (blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) * (uint32_t)kWave; c0 < P;
       c0 += nw * kWave) {
    const uint32_t p = c0 + l;
    const bool valid = p < P;
    const uint32_t pc = valid ? p : P - 1;
    const uint32_t s = valid ? ws.pair_slot[pc] : 0xffffffffu;
    float v[9];
    if (c0 + kWave <= P) {
      const float4 *src = reinterpret_cast<const float4 *>(ws.gpair + 9 * (size_t)c0);
      float4 r[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) r[u] = src[min(l + kWave * u, kRec4 - 1)];
#pragma unroll
      for (int u = 0; u < 3; ++u)
        if (l + kWave * u < kRec4) sw[l + kWave * u] = r[u];
      // the wave's LDS writes are complete before any lane reads them
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const float *sf = reinterpret_cast<const float *>(sw) + 9 * l;
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = sf[k];
      // every lane has read before the next chunk overwrites the stage
      __builtin_amdgcn_wave_barrier();
    } else {
      const float *gp = ws.gpair + 9 * (size_t)pc;
#pragma unroll
      for (int k = 0; k < 9; ++k) v[k] = valid ? gp[k] : 0.0f;
    }
    // does the chunk's first (last) run continue from (into) its neighbour?
    const uint32_t s0 = __builtin_amdgcn_readfirstlane(s);
    const uint32_t s63 = (uint32_t)__builtin_amdgcn_readlane((int)s, kWave - 1);
    const bool first_cont = c0 > 0 && ws.pair_slot[c0 - 1] == s0;
    const bool last_cont = c0 + kWave < P && ws.pair_slot[c0 + kWave] == s63;
    const uint32_t sp = __shfl_up(s, 1, kWave);
    const bool head = l == 0 || sp != s;
    const uint64_t heads = ballot(head);
    // lane of this run's head within the wave
    const int hl = 63 - __builtin_clzll(heads & (lanemask_lt() | (1ull << l)));
    // segmented inclusive scan by DPP (no LDS round trips): shifts by 1, 2,
    // 4 and 8 within each 16-lane row, then the last lane of row 0 into row 1
    // and of row 2 into row 3, then lane 31 into rows 2 and 3; a lane adds a
    // partial only if the partial's lane lies in its own run
    seg_step<0x111, 0xF>(v, l - 1 >= hl);
    seg_step<0x112, 0xF>(v, l - 2 >= hl);
    seg_step<0x114, 0xF>(v, l - 4 >= hl);
    seg_step<0x118, 0xF>(v, l - 8 >= hl);
    seg_step<0x142, 0xA>(v, (l & ~15) - 1 >= hl);
    seg_step<0x143, 0xC>(v, 31 >= hl);
    const uint32_t sn = __shfl_down(s, 1, kWave);
    const bool tail = valid && (l == kWave - 1 || sn != s);
    const uint32_t chunk = c0 / kWave;
    const bool from_prev = hl == 0 && first_cont;
    const bool into_next = l == kWave - 1 && last_cont;
    if (tail) {
      float *d = ws.dproj + 9 * (size_t)s;
      if (from_prev) d = ws.chunk_part + 18 * (size_t)chunk;          // first run (or whole chunk)
      else if (into_next) d = ws.chunk_part + 18 * (size_t)chunk + 9;  // last run
#pragma unroll
      for (int k = 0; k < 9; ++k) d[k] = v[k];
    }
    if (l == kWave - 1)
      ws.chunk_info[chunk] = (first_cont ? kChunkFirst : 0u) | (last_cont ? kChunkLast : 0u) |
                             (first_cont && last_cont && hl == 0 ? kChunkWhole : 0u);
  }
}

// One thread per chunk whose last run starts in it and continues into the
// next chunk: that run's sum is its partial here, plus the partials of the
// following chunks in order (the whole-chunk ones, then the one where the
// run ends), stored once into the run's slot row.
__global__ __launch_bounds__(kBlock) void k_pair_fix(RasterWs ws) {
  const uint32_t P = ws.hdr->n_listed;
  const uint32_t nch = (P + kWave - 1) / kWave;
  for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < nch; c += gridDim.x * kBlock) {
    const uint32_t info = ws.chunk_info[c];
    if (!(info & kChunkLast) || (info & kChunkWhole)) continue;
    float t[9];
    const float *src = ws.chunk_part + 18 * (size_t)c + 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) t[k] = src[k];
    // a run that continues into the next chunk ends in some later chunk
    // (the last chunk's last run cannot continue), so the walk stops.  The
    // following chunks are read eight at a time (one round trip for most
    // runs, a few for a Gaussian listed in thousands of tiles) and added in
    // chunk order.
    constexpr int kAhead = 8;
    bool done = false;
    for (uint32_t j0 = c + 1; j0 < nch && !done; j0 += kAhead) {
      uint32_t inf[kAhead];
      float pv[kAhead][9];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const uint32_t j = min(j0 + (uint32_t)u, nch - 1);
        inf[u] = ws.chunk_info[j];
#pragma unroll
        for (int k = 0; k < 9; ++k) pv[u][k] = ws.chunk_part[18 * (size_t)j + k];
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        if (!done && j0 + (uint32_t)u < nch) {
#pragma unroll
          for (int k = 0; k < 9; ++k) t[k] += pv[u][k];
          done = !(inf[u] & kChunkWhole);
        }
      }
    }
    float *d = ws.dproj + 9 * (size_t)ws.pair_slot[c * (size_t)kWave + kWave - 1];
#pragma unroll
    for (int k = 0; k < 9; ++k) d[k] = t[k];
  }
}

struct PBwdArgs {
  CamParams cam;
  float dil, jc;
  const float *g;
  int64_t gstride;
  RasterWs ws;
  float *dg;
  int64_t dstride;
};

// Projection backward of one Gaussian (FP32).  Forward recap:
//   (xc, yc, zc) = R (mu - C); Rq = rotation of q; M = Rq diag(s); S = M M^T
//   tx = clamp(xc / zc) zc (same for y); J00 = fx / zc, J02 = -fx tx / zc^2, ...
//   T0 = J00 R0 + J02 R2, T1 = J11 R1 + J12 R2;  (a, b, c) = (T0 S T0, T1 S T0, T1 S T1) + dil
//   conic = (a, b; b, c)^-1;  mean2d = (fx xc / zc + cx, fy yc / zc + cy)
// dL/dSigma2D = -Q Gq Q with Q the conic and Gq the gradient on the
// symmetric conic (its off-diagonal gradient split over both entries).
__device__ void project_bwd_one(const PBwdArgs &a, const float *g, const float *dp, float *out) {
  const CamParams &k = a.cam;
  const float d0 = g[0] - k.C[0], d1 = g[1] - k.C[1], d2 = g[2] - k.C[2];
  const float xc = fma_(k.R[0], d0, fma_(k.R[1], d1, k.R[2] * d2));
  const float yc = fma_(k.R[3], d0, fma_(k.R[4], d1, k.R[5] * d2));
  const float zc = fma_(k.R[6], d0, fma_(k.R[7], d1, k.R[8] * d2));
  const float w = g[6], x = g[7], y = g[8], z = g[9];
  float Rq[9];
  Rq[0] = 1.0f - 2.0f * (y * y + z * z); Rq[1] = 2.0f * (x * y - w * z); Rq[2] = 2.0f * (x * z + w * y);
  Rq[3] = 2.0f * (x * y + w * z); Rq[4] = 1.0f - 2.0f * (x * x + z * z); Rq[5] = 2.0f * (y * z - w * x);
  Rq[6] = 2.0f * (x * z - w * y); Rq[7] = 2.0f * (y * z + w * x); Rq[8] = 1.0f - 2.0f * (x * x + y * y);
  float M[9], S[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * g[3 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      S[3 * i + j] = fma_(M[3 * i], M[3 * j], fma_(M[3 * i + 1], M[3 * j + 1], M[3 * i + 2] * M[3 * j + 2]));
  const float lx = a.jc * ((0.5f * (float)k.W) / k.fx), ly = a.jc * ((0.5f * (float)k.H) / k.fy);
  const float rx = xc / zc, ry = yc / zc;
  const bool clx = rx > lx || rx < -lx, cly = ry > ly || ry < -ly;
  const float txz = fminf(lx, fmaxf(-lx, rx)), tyz = fminf(ly, fmaxf(-ly, ry));
  const float tx = txz * zc, ty = tyz * zc;
  const float iz = 1.0f / zc, iz2 = iz * iz;
  const float J00 = k.fx * iz, J02 = -k.fx * tx * iz2, J11 = k.fy * iz, J12 = -k.fy * ty * iz2;
  float T0[3], T1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T0[c] = fma_(J00, k.R[c], J02 * k.R[6 + c]);
    T1[c] = fma_(J11, k.R[3 + c], J12 * k.R[6 + c]);
  }
  float ST0[3], ST1[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ST0[i] = fma_(S[3 * i], T0[0], fma_(S[3 * i + 1], T0[1], S[3 * i + 2] * T0[2]));
    ST1[i] = fma_(S[3 * i], T1[0], fma_(S[3 * i + 1], T1[1], S[3 * i + 2] * T1[2]));
  }
  const float ca = fma_(T0[0], ST0[0], fma_(T0[1], ST0[1], T0[2] * ST0[2])) + a.dil;
  const float cb = fma_(T1[0], ST0[0], fma_(T1[1], ST0[1], T1[2] * ST0[2]));
  const float cc = fma_(T1[0], ST1[0], fma_(T1[1], ST1[1], T1[2] * ST1[2])) + a.dil;
  const float idet = 1.0f / (ca * cc - cb * cb);
  const float Q0 = cc * idet, Q1 = -cb * idet, Q3 = ca * idet;
  const float G0 = dp[2], G1 = 0.5f * dp[3], G3 = dp[4];
  // H = -Q G Q (symmetric 2x2)
  const float QG0 = Q0 * G0 + Q1 * G1, QG1 = Q0 * G1 + Q1 * G3;
  const float QG2 = Q1 * G0 + Q3 * G1, QG3 = Q1 * G1 + Q3 * G3;
  const float H0 = -(QG0 * Q0 + QG1 * Q1), H1 = -(QG0 * Q1 + QG1 * Q3);
  const float H2 = -(QG2 * Q0 + QG3 * Q1), H3 = -(QG2 * Q1 + QG3 * Q3);
  const float da = H0, db = H1 + H2, dc = H3;
  float dT0[3], dT1[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    dT0[i] = 2.0f * da * ST0[i] + db * ST1[i];
    dT1[i] = db * ST0[i] + 2.0f * dc * ST1[i];
  }
  // dL/dSigma (general) then dM = (GS + GS^T) M
  float GS[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      GS[3 * i + j] = da * T0[i] * T0[j] + db * T1[i] * T0[j] + dc * T1[i] * T1[j];
  float ds[3] = {0.0f, 0.0f, 0.0f}, dR[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float sum = 0.0f;
#pragma unroll
      for (int l = 0; l < 3; ++l) sum = fma_(GS[3 * i + l] + GS[3 * l + i], M[3 * l + j], sum);
      ds[j] = fma_(sum, Rq[3 * i + j], ds[j]);
      dR[3 * i + j] = sum * g[3 + j];
    }
  float dw = 0.0f, dx = 0.0f, dy = 0.0f, dz = 0.0f;
  dy += -4.0f * y * dR[0]; dz += -4.0f * z * dR[0];
  dx += 2.0f * y * dR[1]; dy += 2.0f * x * dR[1]; dw += -2.0f * z * dR[1]; dz += -2.0f * w * dR[1];
  dx += 2.0f * z * dR[2]; dz += 2.0f * x * dR[2]; dw += 2.0f * y * dR[2]; dy += 2.0f * w * dR[2];
  dx += 2.0f * y * dR[3]; dy += 2.0f * x * dR[3]; dw += 2.0f * z * dR[3]; dz += 2.0f * w * dR[3];
  dx += -4.0f * x * dR[4]; dz += -4.0f * z * dR[4];
  dy += 2.0f * z * dR[5]; dz += 2.0f * y * dR[5]; dw += -2.0f * x * dR[5]; dx += -2.0f * w * dR[5];
  dx += 2.0f * z * dR[6]; dz += 2.0f * x * dR[6]; dw += -2.0f * y * dR[6]; dy += -2.0f * w * dR[6];
  dy += 2.0f * z * dR[7]; dz += 2.0f * y * dR[7]; dw += 2.0f * x * dR[7]; dx += 2.0f * w * dR[7];
  dx += -4.0f * x * dR[8]; dy += -4.0f * y * dR[8];
  float dJ00 = 0.0f, dJ02 = 0.0f, dJ11 = 0.0f, dJ12 = 0.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    dJ00 = fma_(dT0[i], k.R[i], dJ00);
    dJ02 = fma_(dT0[i], k.R[6 + i], dJ02);
    dJ11 = fma_(dT1[i], k.R[3 + i], dJ11);
    dJ12 = fma_(dT1[i], k.R[6 + i], dJ12);
  }
  float dxc = 0.0f, dyc = 0.0f, dzc = 0.0f;
  dzc += -(dJ00 * k.fx + dJ11 * k.fy) * iz2;
  const float dtx = -dJ02 * k.fx * iz2, dty = -dJ12 * k.fy * iz2;
  dzc += 2.0f * (dJ02 * k.fx * tx + dJ12 * k.fy * ty) * iz2 * iz;
  if (clx) dzc += dtx * txz; else dxc += dtx;
  if (cly) dzc += dty * tyz; else dyc += dty;
  dxc += dp[0] * k.fx * iz;
  dzc += -dp[0] * k.fx * xc * iz2;
  dyc += dp[1] * k.fy * iz;
  dzc += -dp[1] * k.fy * yc * iz2;
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c] = fma_(k.R[c], dxc, fma_(k.R[3 + c], dyc, k.R[6 + c] * dzc));
  out[3] = ds[0]; out[4] = ds[1]; out[5] = ds[2];
  out[6] = dw; out[7] = dx; out[8] = dy; out[9] = dz;
  out[10] = dp[5];
  out[11] = dp[6]; out[12] = dp[7]; out[13] = dp[8];
}

__global__ __launch_bounds__(kBlock) void k_project_bwd(PBwdArgs a) {
  const uint32_t n = a.ws.hdr->n_slots;
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < n; s += gridDim.x * kBlock) {
    float out[kGaussFields];
    const bool vis = (a.ws.vis_mask[s >> 6] >> (s & 63)) & 1ull;
    if (vis) {
      float g[kGaussFields], dp[9];
#pragma unroll
      for (int f = 0; f < kGaussFields; ++f) g[f] = a.g[f * a.gstride + s];
#pragma unroll
      for (int q = 0; q < 9; ++q) dp[q] = a.ws.dproj[9 * (size_t)s + q];
      project_bwd_one(a, g, dp, out);
    } else {
#pragma unroll
      for (int f = 0; f < kGaussFields; ++f) out[f] = 0.0f;
    }
#pragma unroll
    for (int f = 0; f < kGaussFields; ++f) a.dg[f * a.dstride + s] = out[f];
  }
}

}  // namespace

}  // namespace octgs

using namespace octgs;

extern "C" int octgs_rasterize_bwd(const octgs_gaussians *g, const octgs_camera *cam,
                                   const octgs_raster_params *p, int64_t pair_capacity,
                                   const float *T_final, const uint32_t *last,
                                   const float *dL_drgb, float *d_gauss, void *wsp,
                                   size_t ws_bytes, void *const *stage_events,
                                   octgs_stream stream) {
  if (!g || !cam || !p || !T_final || !last || !dL_drgb || !d_gauss || !wsp) return OCTGS_EINVAL;
  // the pair indices of the forward's tile sort are kept only in training mode
  if (!(p->flags & OCTGS_RASTER_TRAIN)) return OCTGS_EINVAL;
  if (!g->data || !g->count || g->capacity < 0 || g->capacity >= (int64_t(1) << 31))
    return OCTGS_EINVAL;
  if (pair_capacity < 0 || pair_capacity >= (int64_t(1) << 30)) return OCTGS_EINVAL;
  if (!image_tiles_ok(cam->width, cam->height) || !(cam->fx > 0.0f) || !(cam->fy > 0.0f))
    return OCTGS_EINVAL;
  if (ws_bytes < octgs_raster_workspace_bytes(g->capacity, pair_capacity, cam->width, cam->height))
    return OCTGS_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  RasterWs ws = raster_layout(wsp, g->capacity, pair_capacity, cam->width, cam->height);
  auto mark = [&](int i) {
    if (stage_events && stage_events[i]) (void)hipEventRecord((hipEvent_t)stage_events[i], s);  // timing only
  };
  const int ntiles = ws.tiles_x * ws.tiles_y;
  BwdArgs b;
  b.ws = ws;
  b.buf = tile_sort_passes(ntiles) % 2;
  b.W = cam->width;
  b.H = cam->height;
  b.alpha_max = p->alpha_max;
  b.alpha_min = p->alpha_min;
  for (int i = 0; i < 3; ++i) b.bg[i] = p->bg[i];
  b.T_final = T_final;
  b.dimg = dL_drgb;
  b.last = last;
  mark(0);
  hipLaunchKernelGGL(k_composite_bwd, dim3(tile_grid_blocks(ws.tiles_x, ws.tiles_y)),
                     dim3(kBwdThreads), 0, s, b);
  mark(1);
  mark(2);
  const int rgrid = (int)std::min<int64_t>(std::max<int64_t>((ws.pcap + kBlock - 1) / kBlock, 1), 2048);
  hipLaunchKernelGGL(k_pair_reduce, dim3(rgrid), dim3(kBlock), 0, s, ws);
  const int fgrid = (int)std::min<int64_t>(std::max<int64_t>((ws.pcap + 64 * kBlock - 1) / (64 * kBlock), 1), 1024);
  hipLaunchKernelGGL(k_pair_fix, dim3(fgrid), dim3(kBlock), 0, s, ws);
  PBwdArgs pa;
  for (int i = 0; i < 9; ++i) pa.cam.R[i] = cam->R[i];
  for (int i = 0; i < 3; ++i) pa.cam.C[i] = cam->C[i];
  pa.cam.fx = cam->fx; pa.cam.fy = cam->fy; pa.cam.cx = cam->cx; pa.cam.cy = cam->cy;
  pa.cam.z_near = cam->z_near; pa.cam.W = cam->width; pa.cam.H = cam->height;
  pa.dil = p->dilation;
  pa.jc = p->jac_clamp;
  pa.g = g->data;
  pa.gstride = g->capacity;
  pa.ws = ws;
  pa.dg = d_gauss;
  pa.dstride = g->capacity;
  const int pgrid = (int)std::min<int64_t>(std::max<int64_t>((ws.gcap + kBlock - 1) / kBlock, 1), 4096);
  hipLaunchKernelGGL(k_project_bwd, dim3(pgrid), dim3(kBlock), 0, s, pa);
  mark(3);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}
