// Forward rasterizer (Octree-GS Sec. III-A: EWA projection of each 3D
// Gaussian to a 2D one, tile-based front-to-back depth ordering, and the
// alpha blending of Eq. 2).
//
// Stages, all on one stream with device-resident counts:
//   init      zero counters, tile ranges, radix histograms
//   project   per Gaussian slot: culls, 2D covariance, conic, 3-sigma tile
//             rectangle, depth key; ballot of survivors
//   compact   survivors in slot order -> (depth key, slot)
//   sort      Onesweep on the 32-bit depth keys (4 passes over Gaussians)
//   emit      candidates in depth order: per Gaussian its rectangle's
//             tiles, offsets by a two-pass scan, writers balanced over
//             candidates; each candidate is kept iff the 3-sigma ellipse
//             meets the tile (tile_meets_ellipse); ordered compaction of
//             the kept ones by ballots and a scan over runs
//   sort      Onesweep on the tile id (1-3 passes over pairs); stable, so
//             each tile keeps depth order, ties by slot index
//   ranges    [start, end) per tile
//   composite one wave per 16x16 tile (four pixels of a column per lane),
//             batches of 128 Gaussians staged in LDS, exit once every pixel
//             is done
//
// Sorting depth once per Gaussian and then only the tile id per pair gives
// the same (tile, depth, slot) order as one sort of 64-bit tile|depth keys
// while moving far fewer bytes: a pair list is typically several times
// longer than the Gaussian list.
//
// Decisions (culls, rectangle, depth key, tile test) use the fixed FP32
// operation sequences documented at project_decide and tile_meets_ellipse;
// continuous values are FP32.
#include "octgs_internal.h"

namespace octgs {

namespace {

typedef CamParams Cam;

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Canonical FP32 projection decisions and FP32 continuous outputs for one
// Gaussian (attributes g[14]).  Sequence:
//   cull unless opacity > 0
//   d = mean - C; (xc, yc, zc) rows fmaf(R0, d0, fmaf(R1, d1, R2 * d2)); cull unless zc > z_near
//   yy=y*y zz=z*z xx=x*x xy=x*y xz=x*z yz=y*z wx=w*x wy=w*y wz=w*z
//   Rq = [1-2(yy+zz), 2(xy-wz), 2(xz+wy); 2(xy+wz), 1-2(xx+zz), 2(yz-wx); 2(xz-wy), 2(yz+wx), 1-2(xx+yy)]
//   M_ab = Rq_ab * s_b; S_ab = fmaf(M_a0, M_b0, fmaf(M_a1, M_b1, M_a2 * M_b2))
//   lx = jac_clamp * ((0.5 * W) / fx); rx = xc / zc; tx = min(lx, max(-lx, rx)) * zc (y alike)
//   zc2 = zc * zc; J00 = fx / zc; J02 = -((fx * tx) / zc2); J11 = fy / zc; J12 = -((fy * ty) / zc2)
//   T0_c = fmaf(J00, R_0c, J02 * R_2c); T1_c = fmaf(J11, R_1c, J12 * R_2c)
//   u_a = fmaf(S_a0, T0_0, fmaf(S_a1, T0_1, S_a2 * T0_2)); v_a likewise with T1
//   a = dot(T0, u) + dil; b = dot(T1, u); c = dot(T1, v) + dil;  dot = fmaf chain
//   det = a * c - b * b; cull unless det > 0
//   mid = 0.5 * (a + c); lam = mid + sqrtf(fmaxf(mid * mid - det, 0)); r = ceilf(3 * sqrtf(lam))
//   px = fmaf(fx, rx, cx); py = fmaf(fy, ry, cy)
//   x0 = clamp(floorf((px - r) * 0.0625)), x1 = clamp(floorf((px + r) * 0.0625) + 1) to [0, tiles]
//   cull if x0 >= x1 or y0 >= y1
struct ProjOut {
  float mx, my, ca, cb, cc, zc;
  int x0, y0, x1, y1;
};

__device__ __forceinline__ bool project_decide(const Cam &k, float dil, float jc, int tiles_x,
                                               int tiles_y, const float *g, ProjOut &o) {
  if (!(g[10] > 0.0f)) return false;
  const float d0 = g[0] - k.C[0], d1 = g[1] - k.C[1], d2 = g[2] - k.C[2];
  const float xc = fma_(k.R[0], d0, fma_(k.R[1], d1, k.R[2] * d2));
  const float yc = fma_(k.R[3], d0, fma_(k.R[4], d1, k.R[5] * d2));
  const float zc = fma_(k.R[6], d0, fma_(k.R[7], d1, k.R[8] * d2));
  if (!(zc > k.z_near)) return false;
  const float w = g[6], x = g[7], y = g[8], z = g[9];
  const float yy = y * y, zz = z * z, xx = x * x, xy = x * y, xz = x * z, yz = y * z;
  const float wx = w * x, wy = w * y, wz = w * z;
  float Rq[9];
  Rq[0] = 1.0f - 2.0f * (yy + zz); Rq[1] = 2.0f * (xy - wz); Rq[2] = 2.0f * (xz + wy);
  Rq[3] = 2.0f * (xy + wz); Rq[4] = 1.0f - 2.0f * (xx + zz); Rq[5] = 2.0f * (yz - wx);
  Rq[6] = 2.0f * (xz - wy); Rq[7] = 2.0f * (yz + wx); Rq[8] = 1.0f - 2.0f * (xx + yy);
  float M[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * g[3 + b];
  float S[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      const float v = fma_(M[3 * a], M[3 * b], fma_(M[3 * a + 1], M[3 * b + 1], M[3 * a + 2] * M[3 * b + 2]));
      S[3 * a + b] = v;
      S[3 * b + a] = v;
    }
  const float lx = jc * ((0.5f * (float)k.W) / k.fx);
  const float ly = jc * ((0.5f * (float)k.H) / k.fy);
  const float rx = xc / zc, ry = yc / zc;
  const float tx = fminf(lx, fmaxf(-lx, rx)) * zc;
  const float ty = fminf(ly, fmaxf(-ly, ry)) * zc;
  const float zc2 = zc * zc;
  const float J00 = k.fx / zc, J02 = -((k.fx * tx) / zc2);
  const float J11 = k.fy / zc, J12 = -((k.fy * ty) / zc2);
  float T0[3], T1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T0[c] = fma_(J00, k.R[c], J02 * k.R[6 + c]);
    T1[c] = fma_(J11, k.R[3 + c], J12 * k.R[6 + c]);
  }
  float u[3], v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = fma_(S[3 * a], T0[0], fma_(S[3 * a + 1], T0[1], S[3 * a + 2] * T0[2]));
    v[a] = fma_(S[3 * a], T1[0], fma_(S[3 * a + 1], T1[1], S[3 * a + 2] * T1[2]));
  }
  const float ca = fma_(T0[0], u[0], fma_(T0[1], u[1], T0[2] * u[2])) + dil;
  const float cb = fma_(T1[0], u[0], fma_(T1[1], u[1], T1[2] * u[2]));
  const float cc = fma_(T1[0], v[0], fma_(T1[1], v[1], T1[2] * v[2])) + dil;
  const float det = ca * cc - cb * cb;
  if (!(det > 0.0f)) return false;
  const float mid = 0.5f * (ca + cc);
  const float lam = mid + sqrtf(fmaxf(mid * mid - det, 0.0f));
  const float r = ceilf(3.0f * sqrtf(lam));
  const float px = fma_(k.fx, rx, k.cx), py = fma_(k.fy, ry, k.cy);
  const float fx0 = floorf((px - r) * 0.0625f), fx1 = floorf((px + r) * 0.0625f) + 1.0f;
  const float fy0 = floorf((py - r) * 0.0625f), fy1 = floorf((py + r) * 0.0625f) + 1.0f;
  const float tX = (float)tiles_x, tY = (float)tiles_y;
  const int x0 = (int)fminf(fmaxf(fx0, 0.0f), tX), x1 = (int)fminf(fmaxf(fx1, 0.0f), tX);
  const int y0 = (int)fminf(fmaxf(fy0, 0.0f), tY), y1 = (int)fminf(fmaxf(fy1, 0.0f), tY);
  if (x0 >= x1 || y0 >= y1) return false;
  const float inv = 1.0f / det;
  o.mx = px; o.my = py;
  o.ca = cc * inv; o.cb = -cb * inv; o.cc = ca * inv;
  o.zc = zc;
  o.x0 = x0; o.y0 = y0; o.x1 = x1; o.y1 = y1;
  return true;
}

// Tile test, canonical FP32: does the 3-sigma ellipse q(p) <= 9,
// q = qa dx^2 + 2 qb dx dy + qc dy^2 around (mx, my), meet the box of the
// tile's pixel centres inside the image, [16 tx + 0.5, min(16 tx + 15.5,
// W - 0.5)] x [16 ty + 0.5, min(16 ty + 15.5, H - 0.5)]?  (Pixels of a
// partial edge tile past the image are not drawn, so they do not list a
// Gaussian.)  The convex quadratic's minimum over the box is 0 with the mean
// inside; otherwise it lies on an edge facing the mean, at the 1D minimiser
// clamped to the edge:
//   X0 = (float)(16 tx) + 0.5, X1 = fminf(X0 + 15, xmax) (Y alike)
//   mean's x outside [X0, X1]: xe = nearer of X0, X1; dx = xe - mx;
//     ys = min(max(my - (qb * dx) / qc, Y0), Y1); dy = ys - my;
//     q1 = fmaf(qa * dx, dx, fmaf(2 * qb * dx, dy, qc * dy * dy))
//   mean's y outside [Y0, Y1]: the same with the roles of x and y swapped
//   keep iff min(q1, q2) <= 9.
__device__ __forceinline__ bool tile_meets_ellipse(float mx, float my, float qa, float qb, float qc,
                                                   uint32_t tx, uint32_t ty, float xmax,
                                                   float ymax) {
  const float X0 = (float)(16u * tx) + 0.5f, X1 = fminf(X0 + 15.0f, xmax);
  const float Y0 = (float)(16u * ty) + 0.5f, Y1 = fminf(Y0 + 15.0f, ymax);
  const bool in_x = !(mx < X0) && !(mx > X1), in_y = !(my < Y0) && !(my > Y1);
  float q = INFINITY;
  if (!in_x) {
    const float xe = mx < X0 ? X0 : X1;
    const float dx = xe - mx;
    const float ys = fminf(fmaxf(my - (qb * dx) / qc, Y0), Y1);
    const float dy = ys - my;
    q = fma_(qa * dx, dx, fma_(2.0f * qb * dx, dy, qc * dy * dy));
  }
  if (!in_y) {
    const float ye = my < Y0 ? Y0 : Y1;
    const float dy = ye - my;
    const float xs = fminf(fmaxf(mx - (qb * dy) / qa, X0), X1);
    const float dx = xs - mx;
    q = fminf(q, fma_(qa * dx, dx, fma_(2.0f * qb * dx, dy, qc * dy * dy)));
  }
  return (in_x && in_y) || q <= 9.0f;
}

// Clears, for each of `passes` sort passes (pass_words apart), the look-back
// rows of the partitions that start in [a, b) (partitions of `part` keys,
// nparts of them at capacity) and the group rows of the groups they open;
// called by whole blocks of 256 threads, one digit's words per thread.
__device__ __forceinline__ void clear_partitions(uint32_t *lb, size_t pass_words, uint32_t a,
                                                 uint32_t b, int passes, int64_t nparts,
                                                 uint32_t part) {
  const uint32_t j0 = (a + part - 1) / part;
  const uint32_t j1 = (uint32_t)std::min<uint64_t>(((uint64_t)b + part - 1) / part, (uint64_t)nparts);
  for (int p = 0; p < passes; ++p) {
    uint32_t *base = lb + p * pass_words;
    for (uint32_t j = j0; j < j1; ++j) {
      base[(size_t)j * kLbRow + threadIdx.x] = 0u;
      base[(size_t)j * kLbRow + 256 + threadIdx.x] = 0u;
      if (j % kGroupParts == 0)
        base[(size_t)nparts * kLbRow + (size_t)(j / kGroupParts) * 256 + threadIdx.x] = 0u;
    }
  }
}

__device__ __forceinline__ uint64_t pack_rect(int x0, int y0, int x1, int y1) {
  return (uint64_t)(uint16_t)x0 | ((uint64_t)(uint16_t)y0 << 16) | ((uint64_t)(uint16_t)x1 << 32) |
         ((uint64_t)(uint16_t)y1 << 48);
}

__device__ __forceinline__ uint32_t rect_tiles(uint64_t r) {
  const uint32_t x0 = r & 0xffff, y0 = (r >> 16) & 0xffff, x1 = (r >> 32) & 0xffff, y1 = r >> 48;
  return (x1 - x0) * (y1 - y0);
}

struct ProjArgs {
  Cam cam;
  float dil, jc;
  int tiles_x, tiles_y;
  const float *g;
  int64_t gstride;
  const uint32_t *count;
  int64_t gcap;
  RasterWs ws;
  float *gauss_w;
};

// Also clears the per-call state of the later stages (header, tile ranges,
// radix histograms, the scans' look-back status words), which the kernel
// itself never reads.
__global__ __launch_bounds__(kBlock) void k_project_mark(ProjArgs a) {
  __shared__ uint32_t wsum[4];
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const uint32_t n = (uint32_t)min<int64_t>(*a.count, a.gcap);
  {
    const RasterWs &ws = a.ws;
    const size_t gi = (size_t)blockIdx.x * kBlock + t, gs = (size_t)gridDim.x * kBlock;
    if (blockIdx.x == 0 && t < (int)(sizeof(RasterHeader) / 4))
      reinterpret_cast<uint32_t *>(ws.hdr)[t] = t == 0 ? n : 0u;  // n_slots is word 0
    const size_t nr = 2 * (size_t)ws.tiles_x * ws.tiles_y;
    for (size_t i = gi; i < nr; i += gs) ws.ranges[i] = 0u;
    for (size_t i = gi; i < kHistCopies * kHistStride; i += gs) ws.hist[i] = 0u;
    for (size_t i = gi; i < (size_t)ws.nblk_g; i += gs) ws.lb_emit[i] = 0u;
    for (size_t i = gi; i < (size_t)ws.nruns; i += gs) ws.lb_pair[i] = 0u;
  }
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  if (base >= n) return;
  // every field of the thread's four slots is loaded up front (clamped
  // index, so the loads are unconditional and all in flight together)
  float gg[kChunkPerThread][kGaussFields];
#pragma unroll
  for (int i = 0; i < kChunkPerThread; ++i) {
    const int64_t s = min(base + i * kBlock + t, (int64_t)n - 1);
#pragma unroll
    for (int f = 0; f < kGaussFields; ++f) gg[i][f] = a.g[f * a.gstride + s];
  }
  uint32_t cnt = 0;
#pragma unroll
  for (int i = 0; i < kChunkPerThread; ++i) {
    const int64_t s = base + i * kBlock + t;
    bool vis = false;
    if (s < n) {
      const float *g = gg[i];
      ProjOut o;
      vis = project_decide(a.cam, a.dil, a.jc, a.tiles_x, a.tiles_y, g, o);
      if (vis) {
        float4 *p = a.ws.proj + 3 * s;
        p[0] = make_float4(o.mx, o.my, -0.5f * kLog2e * o.ca, -kLog2e * o.cb);
        p[1] = make_float4(-0.5f * kLog2e * o.cc, log2f(g[10]), g[11], g[12]);
        p[2] = make_float4(g[13], o.ca, o.cb, o.cc);
        a.ws.depth[s] = __float_as_uint(o.zc);
        a.ws.rect[s] = pack_rect(o.x0, o.y0, o.x1, o.y1);
      }
      if (a.gauss_w) a.gauss_w[s] = 0.0f;
    }
    const uint64_t m = ballot(vis);
    const int64_t gidx = base + i * kBlock + w * kWave;
    if (l == 0 && gidx < n) a.ws.vis_mask[gidx >> 6] = m;
    cnt += (uint32_t)__popcll(m);
  }
  if (l == 0) wsum[w] = cnt;
  __syncthreads();
  if (t == 0) a.ws.blk_cnt[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Ordered compaction of the survivors: (depth key, slot) in slot order.
// It also accumulates the four 8-bit digit histograms of the depth keys for
// the radix sort.
__global__ __launch_bounds__(kBlock) void k_project_compact(RasterWs ws, const uint32_t *count) {
  __shared__ uint32_t red[4];
  __shared__ uint32_t gpre[64];
  __shared__ uint64_t gmask[64];
  __shared__ uint32_t h[4][256];
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const uint32_t n = (uint32_t)min<int64_t>(*count, ws.gcap);
  const int b = blockIdx.x;
  const int64_t base = (int64_t)b * kChunk;
  if (n == 0) {
    if (b == 0 && t == 0) ws.hdr->n_visible = 0;
    return;
  }
  if (base >= n) return;
  uint32_t s = 0;
  s = partial_sum_prefix(ws.blk_cnt, b);
  s = wave_sum(s);
  if (l == 0) red[w] = s;
  const int ngroups = (int)min<int64_t>(kGroups, ((int64_t)n - base + 63) / 64);
  if (w == 0) {
    const uint64_t m = l < ngroups ? ws.vis_mask[(base >> 6) + l] : 0ull;
    const uint32_t c = (uint32_t)__popcll(m);
    const uint32_t inc = wave_incl_scan(c);
    gpre[l] = inc - c;
    gmask[l] = m;
  }
  __syncthreads();
  for (int i = t; i < 4 * 256; i += kBlock) (&h[0][0])[i] = 0u;
  __syncthreads();
  const uint32_t prefix = red[0] + red[1] + red[2] + red[3];
  // wave w owns groups w, w + 4, w + 8, w + 12; their depth keys are loaded
  // up front (clamped index), so the loads are in flight together
  uint32_t keys[kGroups / 4];
#pragma unroll
  for (int q = 0; q < kGroups / 4; ++q)
    keys[q] = ws.depth[min(base + 64 * (w + 4 * q) + l, (int64_t)n - 1)];
#pragma unroll
  for (int q = 0; q < kGroups / 4; ++q) {
    const int gi = w + 4 * q;
    const uint64_t m = gi < ngroups ? gmask[gi] : 0ull;
    if ((m >> l) & 1ull) {
      const uint32_t pos = prefix + gpre[gi] + (uint32_t)__popcll(m & lanemask_lt());
      const uint32_t slot = (uint32_t)(base + 64 * gi + l);
      const uint32_t key = keys[q];
      ws.dkey[0][pos] = key;
      ws.dval[0][pos] = slot;
#pragma unroll
      for (int d = 0; d < 4; ++d) atomicAdd(&h[d][(key >> (8 * d)) & 255u], 1u);
    }
  }
  const uint32_t mine = gpre[ngroups - 1] + (uint32_t)__popcll(gmask[ngroups - 1]);
  if ((int64_t)b == ((int64_t)n - 1) / kChunk && t == 0) ws.hdr->n_visible = prefix + mine;
  // clear the depth sort's look-back words of the partitions that start in
  // this block's output range [prefix, prefix + mine), for all four passes
  clear_partitions(ws.lookback, ws.lb_words / 4, prefix, prefix + mine, 4, ws.lb_parts, kSortPart);
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const uint32_t v = h[d][t];
    if (v) atomicAdd(&ws.hist[(blockIdx.x % kHistCopies) * kHistStride + d * 256 + t], v);
  }
}

// Candidate scan over the depth-ordered survivors (one chunk of 1024 per
// block, offsets chained by decoupled look-back): pair_off[s] = rectangle
// tiles of the survivors before s, and run_first[r] = the survivor that
// holds candidate kEmitRun r.  The chunk
// holding the last survivor publishes the total and the overflow flag.
// Values saturate at 2^30 - 1, above any admissible pair capacity, so they
// are exact whenever the candidates fit.
__global__ __launch_bounds__(kBlock) void k_emit_scan(RasterWs ws) {
  __shared__ uint32_t tmp[8];
  __shared__ uint64_t red[4];
  __shared__ uint32_t s_excl;
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const uint32_t n = ws.hdr->n_visible;
  const uint32_t nch = (n + kChunk - 1) / kChunk;
  if (blockIdx.x >= nch) return;  // n == 0: the cleared header already says 0
  // chunk id = ticket, taken in the order blocks start, so every chunk a
  // block waits on belongs to a block that is already running
  __shared__ uint32_t s_c;
  if (t == 0) s_c = atomicAdd(&ws.hdr->ticket[kTicketScan], 1u);
  __syncthreads();
  const uint32_t c = s_c;
  const int64_t base = (int64_t)c * kChunk;
  uint32_t cnt[kChunkPerThread], slot[kChunkPerThread];
  uint64_t mine = 0;
  // two batches of unconditional loads at clamped indices: slots, then
  // their rectangles
#pragma unroll
  for (int i = 0; i < kChunkPerThread; ++i)
    slot[i] = ws.dval[0][min(base + i * kBlock + t, (int64_t)n - 1)];
#pragma unroll
  for (int i = 0; i < kChunkPerThread; ++i) {
    const int64_t sidx = base + i * kBlock + t;
    const uint32_t c = min(rect_tiles(ws.rect[slot[i]]), kLbVal);
    cnt[i] = sidx < n ? c : 0u;
    mine += cnt[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o, 64);
  if (l == 0) red[w] = mine;
  __syncthreads();
  const uint64_t total64 = red[0] + red[1] + red[2] + red[3];
  const uint32_t agg = (uint32_t)std::min<uint64_t>(total64, kLbVal);
  if (w == 0) {
    const uint32_t ex = chained_lookback(ws.lb_emit, c, agg, &ws.hdr->sync_error, kSpinLimit);
    if (l == 0) s_excl = ex;
  }
  __syncthreads();
  const uint32_t excl = s_excl;
  const bool exact = total64 < kLbVal && excl < kLbVal;  // else the call overflows
  // the tile sort's partitions start inside the candidate range of some
  // chunk (kept pairs are a prefix-closed subset of the positions)
  if (excl < kLbVal)
    clear_partitions(ws.lookback_t, ws.lbt_words / max(ws.tile_passes, 1), excl,
                     sat_add(excl, agg), ws.tile_passes, ws.lbt_parts, kTileSortPart);
  // consecutive 256-entry rows of the chunk, scanned in order (32-bit sums
  // are exact when the chunk total is below 2^30)
  uint32_t carry = 0;
#pragma unroll
  for (int i = 0; i < kChunkPerThread; ++i) {
    const int64_t sidx = base + i * kBlock + t;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(cnt[i], tmp, &tot);
    if (exact && sidx < n) {
      const uint32_t o = excl + carry + ex;
      ws.pair_off[sidx] = o;
      // runs whose first candidate falls in [o, o + cnt)
      for (uint32_t r = (o + kEmitRun - 1) / kEmitRun; (uint64_t)r * kEmitRun < (uint64_t)o + cnt[i] &&
                                                       r < (uint32_t)ws.nruns; ++r)
        ws.run_first[r] = (uint32_t)sidx;
    }
    carry += tot;
  }
  if (c == nch - 1 && t == 0) {
    const uint32_t total = sat_add(excl, agg);
    const bool over = total > (uint64_t)ws.pcap;
    ws.hdr->n_candidates = total;
    ws.hdr->pair_overflow = over ? 1u : 0u;
    ws.hdr->n_cand_listed = over ? 0u : total;
  }
}

// Pair emission with the ellipse test and ordered compaction in one pass.
// Block r (1024 threads) takes the run of 8192 consecutive candidate
// positions from 8192 r; runs this long keep the look-back chain short, as
// each step of it is a device-scope round trip
// (r is a ticket taken in the order blocks start, so the runs a block waits
// on belong to blocks already running); it locates the survivors covering the positions (run_first, then a
// binary search of their offsets in LDS), tests each candidate tile, ranks
// the kept ones by ballots, gets the run's output offset by decoupled
// look-back over the preceding runs and writes (tile id, slot) in order.
// It also accumulates the digit histograms of the kept tile ids.
__global__ __launch_bounds__(kEmitThreads) void k_emit_pairs(RasterWs ws, int tile_passes, int train) {
  constexpr int kW = kEmitThreads / kWave;     // waves per block
  constexpr int kG = kEmitRun / 64;            // ballot groups per run
  constexpr int kC = kEmitRun / kEmitThreads;  // candidates per thread (8)
  static_assert(kEmitThreads >= 256 && kC * kEmitThreads == kEmitRun, "emission shape");
  __shared__ uint32_t offs[kEmitRun + 1];
  __shared__ uint16_t owner[kEmitRun];
  __shared__ uint32_t wmax[kW];
  __shared__ uint32_t gpre[kG];
  __shared__ uint64_t gmask[kG];
  __shared__ uint32_t h[4][256];
  __shared__ uint32_t s_agg, s_excl;
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const uint32_t P = ws.hdr->n_cand_listed;
  const uint32_t n = ws.hdr->n_visible;
  const uint32_t R = (P + kEmitRun - 1) / kEmitRun;
  if (blockIdx.x >= R) return;
  __shared__ uint32_t s_r;
  if (t == 0) s_r = atomicAdd(&ws.hdr->ticket[kTicketEmit], 1u);
  for (int i = t; i < 4 * 256; i += kEmitThreads) (&h[0][0])[i] = 0u;
  __syncthreads();
  const uint32_t r = s_r;
  const uint32_t p0 = r * kEmitRun, p1 = min(P, p0 + kEmitRun);
  const uint32_t lo = ws.run_first[r];
  const uint32_t cnt = min((uint32_t)kEmitRun + 1, n - lo);
  {
    // all loads in flight before the first LDS store (clamped, so the code
    // stays straight-line); a thread past the end rewrites the last entry
    // with the value it holds
    constexpr int kU = (kEmitRun + 1 + kEmitThreads - 1) / kEmitThreads;  // 9
    uint32_t v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = ws.pair_off[lo + min((uint32_t)(t + u * kEmitThreads), cnt - 1)];
#pragma unroll
    for (int u = 0; u < kU; ++u) offs[min((uint32_t)(t + u * kEmitThreads), cnt - 1)] = v[u];
  }
  // owner[i]: local index of the survivor holding position p0 + i.  Each
  // survivor that starts inside the run marks its first position (offsets
  // strictly increase), then a prefix maximum fills the gaps.
#pragma unroll
  for (int u = 0; u < kC; ++u) owner[t + u * kEmitThreads] = 0;
  __syncthreads();
  for (uint32_t a = 1 + t; a < cnt; a += kEmitThreads) {
    const uint32_t st = offs[a];
    if (st < p0 + kEmitRun) owner[st - p0] = (uint16_t)a;
  }
  __syncthreads();
  {
    uint32_t v[kC], m = 0;  // thread t holds positions [8 t, 8 t + 8)
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      m = max(m, (uint32_t)owner[t * kC + u]);
      v[u] = m;
    }
    uint32_t inc = m;  // inclusive max-scan over the wave, then over waves
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, 64);
      if (l >= o) inc = max(inc, y);
    }
    if (l == 63) wmax[w] = inc;
    __syncthreads();
    uint32_t before = __shfl_up(inc, 1, 64);
    if (l == 0) before = 0;
#pragma unroll
    for (int i = 0; i < kW; ++i)
      if (i < w) before = max(before, wmax[i]);
#pragma unroll
    for (int u = 0; u < kC; ++u) owner[t * kC + u] = (uint16_t)max(before, v[u]);
  }
  __syncthreads();
  // three phases over the thread's 8 candidates, so that each phase's
  // global loads are all in flight together: locate (slot), fetch
  // (rectangle, 2D mean and conic), test
  uint32_t key[kC], val[kC], loc[kC];
#pragma unroll
  for (int k = 0; k < kC; ++k) {
    const uint32_t i = min((uint32_t)(k * kEmitThreads + t), p1 - 1 - p0);  // clamped; masked below
    const uint32_t a = owner[i];
    loc[k] = p0 + i - offs[a];
    val[k] = ws.dval[0][lo + a];
  }
  uint64_t rc[kC];
  float4 pa[kC], pc[kC];
#pragma unroll
  for (int k = 0; k < kC; ++k) {
    rc[k] = ws.rect[val[k]];
    pa[k] = ws.proj[3 * (size_t)val[k]];
    pc[k] = ws.proj[3 * (size_t)val[k] + 2];
  }
#pragma unroll
  for (int k = 0; k < kC; ++k) {
    const uint32_t x0 = rc[k] & 0xffff, y0 = (rc[k] >> 16) & 0xffff, x1 = (rc[k] >> 32) & 0xffff;
    const uint32_t wdt = x1 - x0;
    // row and column of the candidate in its rectangle: a float quotient,
    // exact after one correction step while loc < 2^24
    uint32_t row;
    if (loc[k] < (1u << 24)) {
      row = (uint32_t)((float)loc[k] * __builtin_amdgcn_rcpf((float)wdt));
      const int32_t rem = (int32_t)(loc[k] - row * wdt);
      row = rem < 0 ? row - 1 : (rem >= (int32_t)wdt ? row + 1 : row);
    } else {
      row = loc[k] / wdt;
    }
    const uint32_t ty = y0 + row, tx = x0 + (loc[k] - row * wdt);
    const bool keep = p0 + k * kEmitThreads + t < p1 &&
                      tile_meets_ellipse(pa[k].x, pa[k].y, pc[k].y, pc[k].z, pc[k].w, tx, ty,
                                         ws.xmax, ws.ymax);
    key[k] = ty * (uint32_t)ws.tiles_x + tx;
    const uint64_t m = ballot(keep);
    if (l == 0) gmask[k * kW + w] = m;
  }
  __syncthreads();
  if (w == 0) {
    // exclusive prefix over the kG ballot groups, up to one per lane per step
    uint32_t agg = 0;
#pragma unroll
    for (int q = 0; q < (kG + 63) / 64; ++q) {
      const int gi = q * 64 + l;
      const uint32_t c = gi < kG ? (uint32_t)__popcll(gmask[gi]) : 0u;
      const uint32_t inc = wave_incl_scan(c);
      if (gi < kG) gpre[gi] = agg + inc - c;
      agg += __shfl(inc, 63, 64);
    }
    const uint32_t ex = chained_lookback(ws.lb_pair, r, agg, &ws.hdr->sync_error, kSpinLimit);
    if (l == 0) {
      s_excl = ex;
      s_agg = agg;
    }
  }
  __syncthreads();
  const uint32_t excl = s_excl;
#pragma unroll
  for (int k = 0; k < kC; ++k) {
    const int g = k * kW + w;
    const uint64_t m = gmask[g];
    if ((m >> l) & 1ull) {
      const uint32_t dst = excl + gpre[g] + (uint32_t)__popcll(m & lanemask_lt());
      if (dst < P) {  // always true unless a look-back wait hit its bound
        ws.tkey[0][dst] = key[k];
        ws.tval[0][dst] = val[k];
        if (train) {  // what the backward needs: emission index and slot per pair
          ws.tpair[0][dst] = dst;
          ws.pair_slot[dst] = val[k];
        }
      }
      for (int d = 0; d < tile_passes; ++d) atomicAdd(&h[d][(key[k] >> (8 * d)) & 255u], 1u);
    }
  }
  if (r == R - 1 && t == 0) {
    ws.hdr->n_listed = sat_add(excl, s_agg);
    ws.hdr->n_pairs = sat_add(excl, s_agg);
  }
  __syncthreads();
  if (t < 256)
    for (int d = 0; d < tile_passes; ++d) {
      const uint32_t v = h[d][t];
      if (v) atomicAdd(&ws.hist[(blockIdx.x % kHistCopies) * kHistStride + (4 + d) * 256 + t], v);
    }
}

__global__ __launch_bounds__(kBlock) void k_ranges(RasterWs ws, int buf) {
  const uint32_t P = ws.hdr->n_listed;
  const uint32_t *key = ws.tkey[buf];
  for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < P; p += gridDim.x * kBlock) {
    const uint32_t k = key[p];
    if (p == 0 || key[p - 1] != k) ws.ranges[2 * k] = p;
    if (p == P - 1 || key[p + 1] != k) ws.ranges[2 * k + 1] = p + 1;
  }
}

constexpr int kOrderBuckets = 64;  // = kWave: one scan lane per bucket

// Half-octave bucket of a tile's list length, longest lists first; empty
// tiles and blocks without a tile go last (kOrderBuckets - 1).
__device__ __forceinline__ uint32_t order_bucket(int32_t tile, const uint32_t *ranges) {
  if (tile < 0) return kOrderBuckets - 1;
  const uint32_t len = ranges[2 * tile + 1] - ranges[2 * tile];
  if (len == 0) return kOrderBuckets - 1;
  const uint32_t lg = 31u - (uint32_t)__clz(len);
  const uint32_t half = lg > 0 ? (len >> (lg - 1)) & 1u : 0u;
  return (uint32_t)(kOrderBuckets - 2) - min(2u * lg + half, (uint32_t)(kOrderBuckets - 2));
}

// Block x takes the slots that the group mapping gives XCD x and writes
// their tiles to tile_order[x + 8 * position] in a stable order by bucket
// (longest lists first):
// a counting pass, then chunks of 1024 slots ranked per wave with ballots
// (match-any on the bucket bits), each wave owning a contiguous run.  Every
// position of the XCD is written once, so tile_order is a permutation of the
// group mapping.
__global__ __launch_bounds__(kBlock) void k_tile_order(RasterWs ws) {
  constexpr int kItems = 4;
  constexpr int kWaves = kBlock / kWave;
  __shared__ uint32_t cnt[kOrderBuckets];
  __shared__ uint32_t wcnt[kWaves][kOrderBuckets];
  __shared__ uint32_t run[kOrderBuckets];
  const uint32_t xcd = blockIdx.x;
  const uint32_t nslots = tile_grid_blocks(ws.tiles_x, ws.tiles_y) / kXcds;
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const uint64_t lt = lanemask_lt();
  if (xcd == 0 && t == 0) ws.hdr->tile_ordered = 1u;
  if (t < kOrderBuckets) cnt[t] = 0u;
  __syncthreads();
  for (uint32_t q = t; q < nslots; q += kBlock)
    atomicAdd(&cnt[order_bucket(tile_of_block(xcd + kXcds * q, ws.tiles_x, ws.tiles_y),
                                ws.ranges)], 1u);
  __syncthreads();
  if (w == 0) {
    const uint32_t v = cnt[l];
    run[l] = wave_incl_scan(v) - v;
  }
  for (uint32_t c0 = 0; c0 < nslots; c0 += kBlock * kItems) {
    (&wcnt[0][0])[t] = 0u;  // kWaves * kOrderBuckets == kBlock
    int32_t tl[kItems];
    uint32_t key[kItems], rank[kItems];
    bool ok[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint32_t q = c0 + (uint32_t)(w * kWave * kItems + j * kWave + l);
      ok[j] = q < nslots;
      tl[j] = ok[j] ? tile_of_block(xcd + kXcds * q, ws.tiles_x, ws.tiles_y) : -1;
      key[j] = order_bucket(tl[j], ws.ranges);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      uint64_t peers = ballot(ok[j]);
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const int bit = (key[j] >> b) & 1;
        const uint64_t bal = ballot(bit);
        peers &= bit ? bal : ~bal;
      }
      uint32_t before = 0;
      if (ok[j]) before = wcnt[w][key[j]];
      // all lanes of the wave have read before any leader writes
      __builtin_amdgcn_wave_barrier();
      if (ok[j]) {
        rank[j] = before + (uint32_t)__popcll(peers & lt);
        if ((peers & lt) == 0) wcnt[w][key[j]] = before + (uint32_t)__popcll(peers);
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (t < kOrderBuckets) {
      uint32_t base = run[t];
#pragma unroll
      for (int v = 0; v < kWaves; ++v) {
        const uint32_t c = wcnt[v][t];
        wcnt[v][t] = base;
        base += c;
      }
      run[t] = base;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kItems; ++j)
      if (ok[j]) ws.tile_order[xcd + kXcds * (wcnt[w][key[j]] + rank[j])] = (uint32_t)tl[j];
    __syncthreads();
  }
}

struct CompArgs {
  RasterWs ws;
  int buf, W, H;
  int ordered;  // blocks take their tile from ws.tile_order
  float alpha_max, alpha_min, t_min, bg[3];
  float *rgb, *T_final;
  uint32_t *last;
  float *gauss_w;
  uint32_t *status;  // nullable: the frame's pair-overflow / look-back bits are OR-ed in
};

// One 16x16 tile per block of one wave (64 threads); each thread owns four
// vertically adjacent pixels of one column, so the Gaussian's column terms
// are shared four ways.  Batches of kFwdBatch list entries are staged in LDS
// as three float4 per Gaussian.  Per entry the exponent of the first pixel
// is evaluated directly and the next three by finite differences of the
// quadratic in dy (exact in real arithmetic; in FP32 within a few ulps of
// |p|):
//   dx = x - mx; dy = y0 - my
//   p0 = fma(C' dy, dy, fma(B' dx, dy, fma(A' dx, dx, log2 op)))
//   d0 = p(dy + 1) - p(dy) = fma(C', 2 dy + 1, B' dx);  d(k+1) = d(k) + 2 C'
//   p(k+1) = p(k) + d(k)
//   a = min(alpha_max, exp2(p)) = min(alpha_max, op G')
// The loop is branch-free (lanes that are done blend alpha 0), so the wave
// only branches on wave-uniform conditions; the tile stops when all of its
// pixels have.
constexpr int kFwdThreads = 64;   // forward composite: one wave per tile, 4 pixels per thread
constexpr int kFwdBatch = 128;    // list entries staged in LDS per batch
constexpr int kPx = 4;

template <bool LOG>
struct CompLds {
  float4 sA[kFwdBatch], sB[kFwdBatch], sC[kFwdBatch];
  uint32_t s_slot[LOG ? kFwdBatch : 1];
  float s_w[LOG ? kFwdBatch : 1];
};

// The LDS lives in the kernel and is passed in, so the two AMIN
// instantiations share one allocation.
template <bool LOG, bool AMIN, bool LAST>
__device__ __forceinline__ void composite_tile(const CompArgs &a, CompLds<LOG> &lds) {
  float4 *sA = lds.sA, *sB = lds.sB, *sC = lds.sC;
  uint32_t *s_slot = lds.s_slot;
  float *s_w = lds.s_w;
  const int32_t tile = a.ordered ? (int32_t)a.ws.tile_order[blockIdx.x]
                                 : tile_of_block(blockIdx.x, a.ws.tiles_x, a.ws.tiles_y);
  if (tile < 0) return;
  const int tx = tile % a.ws.tiles_x, ty = tile / a.ws.tiles_x;
  const int t = threadIdx.x;
  const int px = tx * kTile + (t % kTile), py0 = ty * kTile + kPx * (t / kTile);
  bool in[kPx];
#pragma unroll
  for (int k = 0; k < kPx; ++k) in[k] = px < a.W && py0 + k < a.H;
  const float fx = (float)px + 0.5f, fy = (float)py0 + 0.5f;
  const uint32_t start = __builtin_amdgcn_readfirstlane(a.ws.ranges[2 * tile]);
  const uint32_t end = __builtin_amdgcn_readfirstlane(a.ws.ranges[2 * tile + 1]);
  const uint32_t *vals = a.ws.tval[a.buf];
  const float4 *proj = a.ws.proj;
  const float amax = a.alpha_max, amin = a.alpha_min, tmin = a.t_min;
  float T[kPx], cr[kPx], cg[kPx], cb[kPx];
  uint32_t last[kPx];
  bool done[kPx];
#pragma unroll
  for (int k = 0; k < kPx; ++k) {
    T[k] = in[k] ? 1.0f : 0.0f;
    cr[k] = 0.0f; cg[k] = 0.0f; cb[k] = 0.0f;
    last[k] = end - start;
    done[k] = !in[k];
  }
  for (uint32_t b0 = start; b0 < end; b0 += kFwdBatch) {
    // one wave: the barrier only orders LDS reuse across batches
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kFwdBatch / kFwdThreads; ++q) {
      const int i = t + q * kFwdThreads;
      const uint32_t e = min(b0 + i, end - 1u);
      const uint32_t s = vals[e];
      if (LOG) s_slot[i] = s;
      sA[i] = proj[3 * (size_t)s];
      sB[i] = proj[3 * (size_t)s + 1];
      sC[i] = proj[3 * (size_t)s + 2];
    }
    __syncthreads();
    const int nb = __builtin_amdgcn_readfirstlane((int)min((uint32_t)kFwdBatch, end - b0));
    const uint32_t base = b0 - start + 1u;
    auto step = [&](int j) {
      const float4 A = sA[j];
      const float4 B = sB[j];
      const float cbl = sC[j].x;
      const float dx = fx - A.x;
      const float adx = fma_(A.z * dx, dx, B.y);
      const float bdx = A.w * dx;
      const float dy = fy - A.y;
      float p = fma_(B.x * dy, dy, fma_(bdx, dy, adx));
      float d = fma_(B.x, fma_(2.0f, dy, 1.0f), bdx);
      const float c2 = B.x + B.x;
      const uint32_t li = base + (uint32_t)j;
      float wsum = 0.0f;
#pragma unroll
      for (int k = 0; k < kPx; ++k) {
        if (k > 0) {
          p += d;
          d += c2;
        }
        float al = fminf(amax, __builtin_amdgcn_exp2f(p));
        if (AMIN) al = al < amin ? 0.0f : al;
        al = done[k] ? 0.0f : al;
        const float w = al * T[k];
        cr[k] = fma_(w, B.z, cr[k]);
        cg[k] = fma_(w, B.w, cg[k]);
        cb[k] = fma_(w, cbl, cb[k]);
        T[k] = T[k] - w;
        // `last` follows every entry a live pixel blends and freezes once the
        // pixel is done: the entry that took T below t_min, else the list
        // length (a live pixel keeps the wave going to the end).  A done lane
        // blends nothing more, so its T stays below t_min; an outside lane
        // starts at T = 0.
        if (LAST) last[k] = done[k] ? last[k] : li;
        done[k] = T[k] < tmin;
        if (LOG) wsum += w;
      }
      if (LOG) {
        const float ws = wave_sum_f(wsum);
        if (__lane_id() == 0) s_w[j] = ws;
      }
    };
    // groups of 16 entries, with a wave-uniform exit check between groups
    for (int j0 = 0; j0 < nb; j0 += 16) {
      if (!LOG && __all(done[0] && done[1] && done[2] && done[3])) break;
      if (j0 + 16 <= nb) {
#pragma unroll
        for (int k = 0; k < 16; ++k) step(j0 + k);
      } else {
        for (int j = j0; j < nb; ++j) step(j);
      }
    }
    if (LOG) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kFwdBatch / kFwdThreads; ++q) {
        const int i = t + q * kFwdThreads;
        if (i < nb && s_w[i] != 0.0f) atomicAdd(&a.gauss_w[s_slot[i]], s_w[i]);
      }
    }
    if (__all(done[0] && done[1] && done[2] && done[3])) break;
  }
  const size_t plane = (size_t)a.W * a.H;
#pragma unroll
  for (int k = 0; k < kPx; ++k) {
    if (in[k]) {
      const size_t pix = (size_t)(py0 + k) * a.W + px;
      a.rgb[pix] = fma_(T[k], a.bg[0], cr[k]);
      a.rgb[plane + pix] = fma_(T[k], a.bg[1], cg[k]);
      a.rgb[2 * plane + pix] = fma_(T[k], a.bg[2], cb[k]);
      a.T_final[pix] = T[k];
      if (LAST) a.last[pix] = last[k];
    }
  }
}

template <bool LOG>
__global__ __launch_bounds__(kFwdThreads) void k_composite(CompArgs a) {
  __shared__ CompLds<LOG> lds;
  // the conditions of the earlier stages are final here: one thread adds
  // them to the caller's status word
  if (a.status && blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t f = (a.ws.hdr->pair_overflow ? OCTGS_STATUS_PAIR_OVERFLOW : 0u) |
                       (a.ws.hdr->sync_error ? OCTGS_STATUS_SYNC_ERROR : 0u);
    if (f) atomicOr(a.status, f);
  }
  // a render that no backward follows may leave out the per-pixel entry
  // count, one select per pixel and entry
  if (a.alpha_min > 0.0f) {
    if (a.last)
      composite_tile<LOG, true, true>(a, lds);
    else
      composite_tile<LOG, true, false>(a, lds);
  } else {
    if (a.last)
      composite_tile<LOG, false, true>(a, lds);
    else
      composite_tile<LOG, false, false>(a, lds);
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

RasterWs raster_layout(void *base, int64_t gcap, int64_t pcap, int32_t W, int32_t H) {
  RasterWs ws;
  char *p = (char *)base;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void * {
    void *r = p ? (void *)(p + off) : nullptr;
    off += align256(bytes);
    return r;
  };
  const int64_t g = std::max<int64_t>(gcap, 1), pc = std::max<int64_t>(pcap, 1);
  ws.gcap = g;
  ws.pcap = pc;
  ws.xmax = (float)W - 0.5f;
  ws.ymax = (float)H - 0.5f;
  ws.tiles_x = (W + kTile - 1) / kTile;
  ws.tiles_y = (H + kTile - 1) / kTile;
  ws.nblk_g = (int)((g + kChunk - 1) / kChunk);
  ws.hdr = (RasterHeader *)take(sizeof(RasterHeader));
  ws.vis_mask = (uint64_t *)take((size_t)ws.nblk_g * kGroups * 8);
  ws.blk_cnt = (uint32_t *)take((size_t)ws.nblk_g * 4);
  ws.proj = (float4 *)take((size_t)kProjVec * g * 16);
  ws.depth = (uint32_t *)take((size_t)g * 4);
  ws.rect = (uint64_t *)take((size_t)g * 8);
  for (int i = 0; i < 2; ++i) ws.dkey[i] = (uint32_t *)take((size_t)g * 4);
  for (int i = 0; i < 2; ++i) ws.dval[i] = (uint32_t *)take((size_t)g * 4);
  ws.pair_off = (uint32_t *)take((size_t)g * 4);
  ws.lb_emit = (uint32_t *)take((size_t)ws.nblk_g * 4);
  ws.nruns = (int)((pc + kEmitRun - 1) / kEmitRun);
  ws.run_first = (uint32_t *)take((size_t)ws.nruns * 4);
  ws.lb_pair = (uint32_t *)take((size_t)ws.nruns * 4);
  for (int i = 0; i < 2; ++i) ws.tkey[i] = (uint32_t *)take((size_t)pc * 4);
  for (int i = 0; i < 2; ++i) ws.tval[i] = (uint32_t *)take((size_t)pc * 4);
  for (int i = 0; i < 2; ++i) ws.tpair[i] = (uint32_t *)take((size_t)pc * 4);
  ws.pair_slot = (uint32_t *)take((size_t)pc * 4);
  ws.ranges = (uint32_t *)take((size_t)ws.tiles_x * ws.tiles_y * 8);
  ws.tile_order = (uint32_t *)take((size_t)tile_grid_blocks(ws.tiles_x, ws.tiles_y) * 4);
  ws.hist = (uint32_t *)take(kHistCopies * kHistStride * 4);
  ws.tile_passes = tile_sort_passes(ws.tiles_x * ws.tiles_y);
  ws.lb_parts = (g + kSortPart - 1) / kSortPart;
  ws.lbt_parts = (pc + kTileSortPart - 1) / kTileSortPart;
  ws.lb_words = (size_t)4 * lookback_pass_words(ws.lb_parts);
  ws.lbt_words = (size_t)ws.tile_passes * lookback_pass_words(ws.lbt_parts);
  ws.lookback = (uint32_t *)take(ws.lb_words * 4);
  ws.lookback_t = (uint32_t *)take(ws.lbt_words * 4);
  ws.dproj = (float *)take((size_t)g * 9 * 4);
  ws.gpair = (float *)take((size_t)pc * 9 * 4);
  ws.chunk_part = (float *)take((size_t)((pc + 63) / 64) * 18 * 4);
  ws.chunk_info = (uint32_t *)take((size_t)((pc + 63) / 64) * 4);
  ws.bytes = off;
  return ws;
}

int tile_sort_passes(int ntiles) {
  int bits = 1;
  while ((1 << bits) < ntiles) ++bits;
  return (bits + 7) / 8;
}

}  // namespace octgs

using namespace octgs;

extern "C" {

size_t octgs_raster_workspace_bytes(int64_t gauss_capacity, int64_t pair_capacity, int32_t width,
                                    int32_t height) {
  if (gauss_capacity < 0 || pair_capacity < 0 || !image_tiles_ok(width, height)) return 0;
  return raster_layout(nullptr, gauss_capacity, pair_capacity, width, height).bytes;
}

int octgs_rasterize_fwd(const octgs_gaussians *g, const octgs_camera *cam,
                        const octgs_raster_params *p, int64_t pair_capacity, float *rgb,
                        float *T_final, uint32_t *last, float *gauss_w, void *wsp,
                        size_t ws_bytes, void *const *stage_events, octgs_stream stream) {
  if (!g || !cam || !p || !rgb || !T_final || !wsp) return OCTGS_EINVAL;
  if (!g->data || !g->count || g->capacity < 0 || g->capacity >= (int64_t(1) << 31))
    return OCTGS_EINVAL;
  // candidate counts saturate at 2^30 - 1, which must exceed the capacity
  if (pair_capacity < 0 || pair_capacity >= (int64_t(1) << 30) - 1) return OCTGS_EINVAL;
  if (!image_tiles_ok(cam->width, cam->height)) return OCTGS_EINVAL;
  if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f)) return OCTGS_EINVAL;
  // z_near > 0 keeps every listed depth positive (the depth keys are float bits)
  if (!(cam->z_near > 0.0f)) return OCTGS_EINVAL;
  if (!(p->dilation >= 0.0f) || !(p->jac_clamp > 0.0f)) return OCTGS_EINVAL;
  if (ws_bytes < octgs_raster_workspace_bytes(g->capacity, pair_capacity, cam->width, cam->height))
    return OCTGS_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  RasterWs ws = raster_layout(wsp, g->capacity, pair_capacity, cam->width, cam->height);
  auto mark = [&](int i) {
    if (stage_events && stage_events[i]) (void)hipEventRecord((hipEvent_t)stage_events[i], s);  // timing only
  };
  ProjArgs pa;
  for (int i = 0; i < 9; ++i) pa.cam.R[i] = cam->R[i];
  for (int i = 0; i < 3; ++i) pa.cam.C[i] = cam->C[i];
  pa.cam.fx = cam->fx; pa.cam.fy = cam->fy; pa.cam.cx = cam->cx; pa.cam.cy = cam->cy;
  pa.cam.z_near = cam->z_near; pa.cam.W = cam->width; pa.cam.H = cam->height;
  pa.dil = p->dilation;
  pa.jc = p->jac_clamp;
  pa.tiles_x = ws.tiles_x;
  pa.tiles_y = ws.tiles_y;
  pa.g = g->data;
  pa.gstride = g->capacity;
  pa.count = g->count;
  pa.gcap = g->capacity;
  pa.ws = ws;
  pa.gauss_w = gauss_w;
  mark(0);
  hipLaunchKernelGGL(k_project_mark, dim3(ws.nblk_g), dim3(kBlock), 0, s, pa);
  hipLaunchKernelGGL(k_project_compact, dim3(ws.nblk_g), dim3(kBlock), 0, s, ws, g->count);
  mark(1);
  mark(2);
  // histograms and cleared look-back words come from the kernels above
  hipError_t e = radix_sort(ws.dkey, ws.dval, nullptr, &ws.hdr->n_visible, ws.gcap, kSortItems, 4, ws.hist,
                            kHistCopies, kHistStride, ws.lookback,
                            &ws.hdr->ticket[kTicketDepth], &ws.hdr->sync_error, s);
  if (e != hipSuccess) return OCTGS_EHIP;
  mark(3);
  mark(4);
  hipLaunchKernelGGL(k_emit_scan, dim3(ws.nblk_g), dim3(kBlock), 0, s, ws);
  hipLaunchKernelGGL(k_emit_pairs, dim3(std::max(ws.nruns, 1)), dim3(kEmitThreads), 0, s, ws,
                     ws.tile_passes, (p->flags & OCTGS_RASTER_TRAIN) ? 1 : 0);
  mark(5);
  mark(6);
  const int passes = ws.tile_passes;
  e = radix_sort(ws.tkey, ws.tval, (p->flags & OCTGS_RASTER_TRAIN) ? ws.tpair : nullptr,
                 &ws.hdr->n_listed, ws.pcap, kTileSortItems, passes, ws.hist + 4 * 256, kHistCopies,
                 kHistStride, ws.lookback_t, &ws.hdr->ticket[kTicketTile],
                 &ws.hdr->sync_error, s);
  if (e != hipSuccess) return OCTGS_EHIP;
  const int buf = passes % 2;
  const int rgrid = (int)std::min<int64_t>(std::max<int64_t>((ws.pcap + kBlock - 1) / kBlock, 1), 8192);
  hipLaunchKernelGGL(k_ranges, dim3(rgrid), dim3(kBlock), 0, s, ws, buf);
  const bool ordered = (p->flags & OCTGS_RASTER_TILE_ORDER) != 0;
  if (ordered) hipLaunchKernelGGL(k_tile_order, dim3(kXcds), dim3(kBlock), 0, s, ws);
  mark(7);
  CompArgs ca;
  ca.ws = ws;
  ca.buf = buf;
  ca.ordered = ordered ? 1 : 0;
  ca.W = cam->width;
  ca.H = cam->height;
  ca.alpha_max = p->alpha_max;
  ca.alpha_min = p->alpha_min;
  ca.t_min = p->t_min;
  for (int i = 0; i < 3; ++i) ca.bg[i] = p->bg[i];
  ca.rgb = rgb;
  ca.T_final = T_final;
  ca.last = last;
  ca.gauss_w = gauss_w;
  ca.status = g->status;
  mark(8);
  if (gauss_w)
    hipLaunchKernelGGL(k_composite<true>, dim3(tile_grid_blocks(ws.tiles_x, ws.tiles_y)),
                       dim3(kFwdThreads), 0, s, ca);
  else
    hipLaunchKernelGGL(k_composite<false>, dim3(tile_grid_blocks(ws.tiles_x, ws.tiles_y)),
                       dim3(kFwdThreads), 0, s, ca);
  mark(9);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_raster_views(const void *wsp, int64_t gauss_capacity, int64_t pair_capacity,
                       int32_t width, int32_t height, const octgs_raster_stats **stats,
                       const uint32_t **pair_tile, const uint32_t **pair_slot,
                       const uint32_t **tile_ranges) {
  if (!wsp || width <= 0 || height <= 0 || gauss_capacity < 0 || pair_capacity < 0)
    return OCTGS_EINVAL;
  RasterWs ws = raster_layout(const_cast<void *>(wsp), gauss_capacity, pair_capacity, width, height);
  const int buf = tile_sort_passes(ws.tiles_x * ws.tiles_y) % 2;
  if (stats) *stats = (const octgs_raster_stats *)ws.hdr;
  if (pair_tile) *pair_tile = ws.tkey[buf];
  if (pair_slot) *pair_slot = ws.tval[buf];
  if (tile_ranges) *tile_ranges = ws.ranges;
  return OCTGS_OK;
}

const char *octgs_strerror(int status) {
  switch (status) {
    case OCTGS_OK: return "ok";
    case OCTGS_EINVAL: return "invalid argument";
    case OCTGS_ENOSPC: return "workspace too small";
    case OCTGS_EHIP: return "HIP launch or runtime error";
    case OCTGS_EUNSUPPORTED: return "unsupported shape";
    default: return "unknown status";
  }
}

int octgs_version(void) { return 1; }

}  // extern "C"
