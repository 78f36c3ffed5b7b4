// Learned anchor skip: a small per-anchor contribution predictor that lets
// the render path leave out, before decoding, anchors the view would blend
// with negligible weight.  It extends the paper's per-view anchor selection
// (Sec. IV-A): Eq. 7 picks anchors by distance and level; the predictor
// drops, among those, anchors whose Gaussians would add almost nothing.
//
//   input  z = [feature (32), viewing direction in the camera frame (3),
//               log2(d / d_max), level]
//   net    37 -> 64 -> ReLU -> 64 -> ReLU -> 1 (logit of "contributes")
//   label  the anchor's blend weight sum_pixels sum_{its Gaussians} a_i T_i,
//          logged by the forward rasterizer, above a threshold
//
// Inference runs the two 64-wide layers on BF16 MFMA (16x16x16) with FP32
// accumulation and keeps an anchor iff its logit >= the threshold; the kept
// anchors are compacted in ascending order so decoding is unchanged.
// Training (binary cross-entropy) runs forward and backward on BF16 MFMA
// with FP32 master weights.
#include "octgs_internal.h"

namespace octgs {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int kZ = 37;
constexpr int kZPad = 48;
constexpr int kH = 64;

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

struct FeatArgs {
  const float *pos, *feat;
  const uint8_t *level;
  float R[9], C[3];
  float inv_dmax;
  const uint32_t *idx, *count;
  int64_t cap;
};

// Predictor input of one anchor, FP32: z[0..31] feature, z[32..34] unit
// direction from the camera in camera coordinates, z[35] log2(d / d_max),
// z[36] level.
__device__ __forceinline__ void skip_input(const FeatArgs &a, uint32_t j, float *z) {
  for (int f = 0; f < 32; ++f) z[f] = a.feat[(size_t)j * 32 + f];
  const float d0 = a.pos[3 * (size_t)j] - a.C[0], d1 = a.pos[3 * (size_t)j + 1] - a.C[1];
  const float d2 = a.pos[3 * (size_t)j + 2] - a.C[2];
  const float dist = sqrtf(__builtin_fmaf(d0, d0, __builtin_fmaf(d1, d1, d2 * d2)));
  const float inv = 1.0f / dist;
  // viewing direction in the camera frame: where in the image the anchor lies
  z[32] = __builtin_fmaf(a.R[0], d0, __builtin_fmaf(a.R[1], d1, a.R[2] * d2)) * inv;
  z[33] = __builtin_fmaf(a.R[3], d0, __builtin_fmaf(a.R[4], d1, a.R[5] * d2)) * inv;
  z[34] = __builtin_fmaf(a.R[6], d0, __builtin_fmaf(a.R[7], d1, a.R[8] * d2)) * inv;
  z[35] = log2f(dist * a.inv_dmax);
  z[36] = (float)a.level[j];
}

__global__ __launch_bounds__(kBlock) void k_skip_features(FeatArgs a, float *z) {
  const uint32_t M = (uint32_t)min<int64_t>(*a.count, a.cap);
  for (uint32_t m = blockIdx.x * kBlock + threadIdx.x; m < M; m += gridDim.x * kBlock)
    skip_input(a, a.idx[m], z + (size_t)m * kZ);
}

__global__ __launch_bounds__(kBlock) void k_anchor_weights(const float *gw, const uint32_t *count,
                                                           int k, int64_t cap, float *w) {
  const uint32_t M = (uint32_t)min<int64_t>(*count, cap);
  for (uint32_t m = blockIdx.x * kBlock + threadIdx.x; m < M; m += gridDim.x * kBlock) {
    float s = 0.0f;
    for (int i = 0; i < k; ++i) s += gw[(size_t)m * k + i];
    w[m] = s;
  }
}

struct PredArgs {
  FeatArgs f;
  const float *w1, *b1, *w2, *b2, *w3, *b3;
  float thr;
  uint8_t *flag;
  float *logit;
};

constexpr int kTM = 32;  // anchors per block iteration

// BF16 MFMA forward of the predictor over the listed anchors; writes a keep
// flag (logit >= thr) per list position and, optionally, the logits.
__global__ __launch_bounds__(kBlock) void k_skip_predict(PredArgs a) {
  __shared__ alignas(16) uint16_t sZ[kTM][kZPad + 4];
  __shared__ alignas(16) uint16_t sH1[kTM][kH + 4];
  __shared__ float sH2[kTM][kH + 1];
  const int t = threadIdx.x, w = t / kWave, l = __lane_id(), g = l / 16, lc = l % 16;
  // weight fragments of this wave's 16 output columns, BF16
  s4 B1[3], B2[4];
  const int n = w * 16 + lc;
#pragma unroll
  for (int ks = 0; ks < 3; ++ks) {
    s4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = ks * 16 + g * 4 + j;
      v[j] = (short)f2bf(kk < kZ ? a.w1[kk * kH + n] : 0.0f);
    }
    B1[ks] = v;
  }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    s4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = (short)f2bf(a.w2[(ks * 16 + g * 4 + j) * kH + n]);
    B2[ks] = v;
  }
  const float bias1 = a.b1[n], bias2 = a.b2[n];
  // layer 3 in FP32 on BF16-rounded weights: lane l of each group of 8 owns 8 hidden units
  const uint32_t M = (uint32_t)min<int64_t>(*a.f.count, a.f.cap);
  for (uint32_t tile = blockIdx.x; tile * kTM < M; tile += gridDim.x) {
    const uint32_t r0 = tile * kTM;
    const int rows = (int)min((uint32_t)kTM, M - r0);
    if (t < kTM) {
      float z[kZ];
      if (t < rows) skip_input(a.f, a.f.idx[r0 + t], z);
      else
        for (int q = 0; q < kZ; ++q) z[q] = 0.0f;
      for (int q = 0; q < kZPad; ++q) sZ[t][q] = q < kZ ? f2bf(z[q]) : (uint16_t)0;
    }
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < kTM / 16; ++rt) {
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 3; ++ks) {
        const s4 av = *(const s4 *)&sZ[rt * 16 + lc][ks * 16 + g * 4];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, B1[ks], acc, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) sH1[rt * 16 + 4 * g + i][n] = f2bf(fmaxf(acc[i] + bias1, 0.0f));
    }
    __syncthreads();
#pragma unroll
    for (int rt = 0; rt < kTM / 16; ++rt) {
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const s4 av = *(const s4 *)&sH1[rt * 16 + lc][ks * 16 + g * 4];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, B2[ks], acc, 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) sH2[rt * 16 + 4 * g + i][n] = fmaxf(acc[i] + bias2, 0.0f);
    }
    __syncthreads();
    {
      // 8 lanes per anchor, 8 hidden units each
      const int r = t / 8, part = t % 8;
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int u = part * 8 + q;
        s = __builtin_fmaf(sH2[r][u], bf2f(f2bf(a.w3[u])), s);
      }
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      if (part == 0 && r < rows) {
        const float lg = s + a.b3[0];
        a.flag[r0 + r] = lg >= a.thr ? 1 : 0;
        if (a.logit) a.logit[r0 + r] = lg;
      }
    }
    __syncthreads();
  }
}

// Ordered compaction of flagged list positions (two passes, 1024 positions
// per block): out[q] = src[p] for the q-th flagged p.
__global__ __launch_bounds__(kBlock) void k_flag_mark(const uint8_t *flag, const uint32_t *count,
                                                      int64_t cap, uint64_t *masks,
                                                      uint32_t *blk) {
  __shared__ uint32_t wsum[4];
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const int64_t n = min<int64_t>(*count, cap);
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  if (base >= n) return;
  uint32_t c = 0;
  for (int i = 0; i < kChunkPerThread; ++i) {
    const int64_t p = base + i * kBlock + t;
    const uint64_t m = ballot(p < n && flag[p] != 0);
    const int64_t gi = base + i * kBlock + w * kWave;
    if (l == 0 && gi < n) masks[gi >> 6] = m;
    c += (uint32_t)__popcll(m);
  }
  if (l == 0) wsum[w] = c;
  __syncthreads();
  if (t == 0) blk[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(kBlock) void k_flag_scatter(const uint32_t *count, int64_t cap,
                                                         const uint64_t *masks, const uint32_t *blk,
                                                         const uint32_t *src, uint32_t *out,
                                                         uint32_t *out_count) {
  __shared__ uint32_t red[4];
  __shared__ uint32_t gpre[64];
  __shared__ uint64_t gmask[64];
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const int64_t n = min<int64_t>(*count, cap);
  const int b = blockIdx.x;
  const int64_t base = (int64_t)b * kChunk;
  if (n == 0) {
    if (b == 0 && t == 0) *out_count = 0;
    return;
  }
  if (base >= n) return;
  uint32_t s = 0;
  s = partial_sum_prefix(blk, b);
  s = wave_sum(s);
  if (l == 0) red[w] = s;
  const int ng = (int)min<int64_t>(kGroups, (n - base + 63) / 64);
  if (w == 0) {
    const uint64_t m = l < ng ? masks[(base >> 6) + l] : 0ull;
    const uint32_t c = (uint32_t)__popcll(m);
    gpre[l] = wave_incl_scan(c) - c;
    gmask[l] = m;
  }
  __syncthreads();
  const uint32_t prefix = red[0] + red[1] + red[2] + red[3];
  for (int gi = w; gi < ng; gi += 4) {
    const uint64_t m = gmask[gi];
    if ((m >> l) & 1ull) {
      const uint32_t q = prefix + gpre[gi] + (uint32_t)__popcll(m & lanemask_lt());
      out[q] = src[base + 64 * gi + l];
    }
  }
  if ((int64_t)b == (n - 1) / kChunk && t == 0)
    *out_count = prefix + gpre[ng - 1] + (uint32_t)__popcll(gmask[ng - 1]);
}

// ---- training: one fused BF16 MFMA pass per batch ----------------------
// Weighted binary cross-entropy on the logit x of a row with label y:
//   loss = wgt (softplus(x) - y x),  dloss/dx = wgt (sigmoid(x) - y),
// wgt = pos_weight for positives and 1 otherwise, averaged over the batch.
// Forward and backward of the three layers run per tile of 64 rows: the two
// 64-wide layers, dH1 = dH2 W2^T and both weight gradients dW = X^T dY (the
// tile's rows being the reduction dimension) are BF16 MFMA products with
// FP32 accumulation on BF16 copies of the FP32 master weights; layer 3, the
// loss and the bias gradients stay in FP32.  Each block keeps its gradient
// sums in registers over its tiles and writes them once; a second kernel adds
// the block partials in block order, so the result does not depend on timing.
constexpr int kTR = 64;            // batch rows per tile
constexpr int kTrainBlocks = 256;  // partial-sum blocks at most
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kZ * kH;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH;
constexpr int kOffLoss = kOffB3 + 1;
constexpr int kPartLen = kOffLoss + 1;  // floats per block partial

struct TrainArgs {
  const float *w1, *b1, *w2, *b2, *w3, *b3;
  const float *z, *y;
  const uint32_t *rows;  // nullable: batch row b is row rows[b] of z and y
  int B;
  uint64_t in_mask;      // bit i clear: input i reads as zero
  float pw;
  float *part;           // [gridDim.x][kPartLen]
};

struct TrainLds {
  alignas(16) uint16_t z[kTR][kZPad + 8];  // BF16 inputs of the tile
  alignas(16) uint16_t h1[kTR][kH + 8];    // BF16 ReLU(layer 1)
  alignas(16) uint16_t d2[kTR][kH + 8];    // BF16 dloss/d(layer-2 pre-activation)
  alignas(16) uint16_t d1[kTR][kH + 8];    // BF16 dloss/d(layer-1 pre-activation)
  float h2[kTR][kH + 1];       // FP32 ReLU(layer 2)
  float dx[kTR];               // dloss/dlogit per row (0 on padding rows)
  float yv[kTR];
  float red[4][kH];
};

__device__ __forceinline__ f4 mfma16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(kBlock) void k_skip_train(TrainArgs a) {
  __shared__ TrainLds s;
  const int t = threadIdx.x, w = t / kWave, l = __lane_id(), g = l / 16, lc = l % 16;
  const int n = w * 16 + lc;  // this lane's column in every 16x16 MFMA tile
  // BF16 fragments of W1 and W2 (forward) and of W2^T (for dH1)
  s4 B1[3], B2[4], B2t[4];
#pragma unroll
  for (int ks = 0; ks < 3; ++ks)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = ks * 16 + g * 4 + j;
      B1[ks][j] = (short)f2bf(kk < kZ ? a.w1[kk * kH + n] : 0.0f);
    }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = ks * 16 + g * 4 + j;
      B2[ks][j] = (short)f2bf(a.w2[kk * kH + n]);
      B2t[ks][j] = (short)f2bf(a.w2[n * kH + kk]);
    }
  const float bias1 = a.b1[n], bias2 = a.b2[n];
  // elementwise work: thread t owns hidden column c for rows q*16 .. q*16+15
  const int c = t & 63, q = t >> 6;
  const float w3c = a.w3[c];
  // layer 3: four threads per row, 16 hidden units each
  const int r3 = t >> 2, p3 = t & 3;
  float w3p[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) w3p[u] = a.w3[p3 * 16 + u];
  const float b3 = a.b3[0], invB = 1.0f / (float)a.B;

  f4 gW1[3], gW2[4];
#pragma unroll
  for (int m = 0; m < 3; ++m) gW1[m] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int m = 0; m < 4; ++m) gW2[m] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  float gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f, gloss = 0.0f;

  const int ntiles = (a.B + kTR - 1) / kTR;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int r0 = tile * kTR, rows = min(kTR, a.B - r0);
    for (int e = t; e < kTR * kZPad; e += kBlock) {
      const int r = e / kZPad, col = e % kZPad;
      float v = 0.0f;
      if (r < rows && col < kZ && ((a.in_mask >> col) & 1u)) {
        const size_t row = a.rows ? (size_t)a.rows[r0 + r] : (size_t)(r0 + r);
        v = a.z[row * kZ + col];
      }
      s.z[r][col] = f2bf(v);
    }
    if (t < kTR) s.yv[t] = t < rows ? a.y[a.rows ? (size_t)a.rows[r0 + t] : (size_t)(r0 + t)] : 0.0f;
    __syncthreads();
    // layer 1
#pragma unroll
    for (int rt = 0; rt < kTR / 16; ++rt) {
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 3; ++ks) acc = mfma16(*(const s4 *)&s.z[rt * 16 + lc][ks * 16 + g * 4], B1[ks], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) s.h1[rt * 16 + 4 * g + i][n] = f2bf(fmaxf(acc[i] + bias1, 0.0f));
    }
    __syncthreads();
    // layer 2
#pragma unroll
    for (int rt = 0; rt < kTR / 16; ++rt) {
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) acc = mfma16(*(const s4 *)&s.h1[rt * 16 + lc][ks * 16 + g * 4], B2[ks], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) s.h2[rt * 16 + 4 * g + i][n] = fmaxf(acc[i] + bias2, 0.0f);
    }
    __syncthreads();
    // layer 3, the loss and its derivative per row
    {
      float x = 0.0f;
#pragma unroll
      for (int u = 0; u < 16; ++u) x = __builtin_fmaf(s.h2[r3][p3 * 16 + u], w3p[u], x);
      x += __shfl_xor(x, 1, 64);
      x += __shfl_xor(x, 2, 64);
      if (p3 == 0) {
        float d = 0.0f;
        if (r3 < rows) {
          x += b3;
          const float yy = s.yv[r3], wgt = yy > 0.5f ? a.pw : 1.0f;
          d = wgt * (1.0f / (1.0f + expf(-x)) - yy) * invB;
          gloss += wgt * (fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))) - yy * x);
          gb3 += d;
        }
        s.dx[r3] = d;
      }
    }
    __syncthreads();
    // dH2 = dx w3 where layer 2 is active; dW3 and db2 in FP32
#pragma unroll 4
    for (int i = 0; i < kTR / 4; ++i) {
      const int r = q * (kTR / 4) + i;
      const float h = s.h2[r][c], dx = s.dx[r];
      const float d = h > 0.0f ? dx * w3c : 0.0f;
      gw3 = __builtin_fmaf(h, dx, gw3);
      gb2 += d;
      s.d2[r][c] = f2bf(d);
    }
    __syncthreads();
    // dH1 = dH2 W2^T where layer 1 is active
#pragma unroll
    for (int rt = 0; rt < kTR / 16; ++rt) {
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) acc = mfma16(*(const s4 *)&s.d2[rt * 16 + lc][ks * 16 + g * 4], B2t[ks], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rt * 16 + 4 * g + i;
        const float d = bf2f(s.h1[r][n]) > 0.0f ? acc[i] : 0.0f;
        gb1 += d;
        s.d1[r][n] = f2bf(d);
      }
    }
    // dW2 += H1^T dH2 over the tile's rows
#pragma unroll
    for (int ks = 0; ks < kTR / 16; ++ks) {
      s4 bv;
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = (short)s.d2[ks * 16 + g * 4 + j][n];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        s4 av;
#pragma unroll
        for (int j = 0; j < 4; ++j) av[j] = (short)s.h1[ks * 16 + g * 4 + j][mt * 16 + lc];
        gW2[mt] = mfma16(av, bv, gW2[mt]);
      }
    }
    __syncthreads();
    // dW1 += Z^T dH1 over the tile's rows
#pragma unroll
    for (int ks = 0; ks < kTR / 16; ++ks) {
      s4 bv;
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = (short)s.d1[ks * 16 + g * 4 + j][n];
#pragma unroll
      for (int mt = 0; mt < 3; ++mt) {
        s4 av;
#pragma unroll
        for (int j = 0; j < 4; ++j) av[j] = (short)s.z[ks * 16 + g * 4 + j][mt * 16 + lc];
        gW1[mt] = mfma16(av, bv, gW1[mt]);
      }
    }
    __syncthreads();
  }

  // this block's partial sums
  float *P = a.part + (size_t)blockIdx.x * kPartLen;
#pragma unroll
  for (int mt = 0; mt < 3; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = mt * 16 + 4 * g + i;
      if (r < kZ) P[kOffW1 + r * kH + n] = gW1[mt][i];
    }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) P[kOffW2 + (mt * 16 + 4 * g + i) * kH + n] = gW2[mt][i];
  // db1: the four lane groups g of a wave share column n
  gb1 += __shfl_xor(gb1, 16, 64);
  gb1 += __shfl_xor(gb1, 32, 64);
  if (g == 0) P[kOffB1 + n] = gb1;
  // db2 and dW3: the four row quarters q share column c
  s.red[q][c] = gb2;
  __syncthreads();
  if (t < kH) P[kOffB2 + t] = s.red[0][t] + s.red[1][t] + s.red[2][t] + s.red[3][t];
  __syncthreads();
  s.red[q][c] = gw3;
  __syncthreads();
  if (t < kH) P[kOffW3 + t] = s.red[0][t] + s.red[1][t] + s.red[2][t] + s.red[3][t];
  __syncthreads();
  // db3 and the loss sit on the threads with p3 == 0
  const float sb3 = wave_sum_f(gb3), sl = wave_sum_f(gloss);
  if (l == 0) {
    s.red[0][w] = sb3;
    s.red[1][w] = sl;
  }
  __syncthreads();
  if (t == 0) {
    P[kOffB3] = s.red[0][0] + s.red[0][1] + s.red[0][2] + s.red[0][3];
    P[kOffLoss] = (s.red[1][0] + s.red[1][1] + s.red[1][2] + s.red[1][3]) * invB;
  }
}

// Sum of the block partials in block order; gradients are overwritten and
// the loss is added to *loss.
__global__ __launch_bounds__(kBlock) void k_skip_train_reduce(const float *part, int nblk,
                                                              octgs_skip_net_grads gr,
                                                              float *loss) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= kPartLen) return;
  float acc = 0.0f;
  for (int b = 0; b < nblk; ++b) acc += part[(size_t)b * kPartLen + j];
  if (j < kOffB1) gr.w1[j - kOffW1] = acc;
  else if (j < kOffW2) gr.b1[j - kOffB1] = acc;
  else if (j < kOffB2) gr.w2[j - kOffW2] = acc;
  else if (j < kOffW3) gr.b2[j - kOffB2] = acc;
  else if (j < kOffB3) gr.w3[j - kOffW3] = acc;
  else if (j < kOffLoss) gr.b3[0] = acc;
  else *loss += acc;
}

int train_blocks(int32_t batch) {
  return (int)std::min<int64_t>(((int64_t)batch + kTR - 1) / kTR, kTrainBlocks);
}

FeatArgs feat_args(const octgs_anchors *an, const octgs_camera *cam, const uint32_t *idx,
                   const uint32_t *count, int64_t cap) {
  FeatArgs f;
  f.pos = an->pos;
  f.feat = an->feat;
  f.level = an->level;
  for (int c = 0; c < 3; ++c) f.C[c] = cam->C[c];
  for (int c = 0; c < 9; ++c) f.R[c] = cam->R[c];
  f.inv_dmax = 1.0f / an->d_max;
  f.idx = idx;
  f.count = count;
  f.cap = cap;
  return f;
}

}  // namespace

}  // namespace octgs

using namespace octgs;

extern "C" {

int octgs_anchor_weights(const float *gauss_w, const uint32_t *count, int32_t k,
                         int64_t cap_anchors, float *w_out, octgs_stream stream) {
  if (!gauss_w || !count || !w_out || k < 1 || k > kMaxK || cap_anchors < 0) return OCTGS_EINVAL;
  const int grid = (int)std::min<int64_t>(std::max<int64_t>((cap_anchors + kBlock - 1) / kBlock, 1), 2048);
  hipLaunchKernelGGL(k_anchor_weights, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, gauss_w,
                     count, k, cap_anchors, w_out);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_skip_features(const octgs_anchors *an, const octgs_camera *cam, const uint32_t *idx,
                        const uint32_t *count, int64_t cap, float *z, octgs_stream stream) {
  if (!an || !cam || !idx || !count || !z || cap < 0) return OCTGS_EINVAL;
  if (an->feat_dim != 32 || !an->pos || !an->feat || !an->level || !(an->d_max > 0.0f))
    return OCTGS_EINVAL;
  const int grid = (int)std::min<int64_t>(std::max<int64_t>((cap + kBlock - 1) / kBlock, 1), 2048);
  hipLaunchKernelGGL(k_skip_features, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream,
                     feat_args(an, cam, idx, count, cap), z);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

size_t octgs_skip_predict_workspace_bytes(int64_t cap) {
  if (cap < 0) return 0;
  const int64_t nblk = (std::max<int64_t>(cap, 1) + kChunk - 1) / kChunk;
  return (size_t)(((cap + 255) / 256) * 256 + nblk * kGroups * 8 + nblk * 4 + 1024);
}

int octgs_skip_predict(const octgs_anchors *an, const octgs_camera *cam, const octgs_skip_net *net,
                       float logit_threshold, const uint32_t *sel_idx, const uint32_t *sel_count,
                       int64_t cap, uint32_t *keep_idx, uint32_t *keep_count, float *logits,
                       void *ws, size_t ws_bytes, octgs_stream stream) {
  if (!an || !cam || !net || !sel_idx || !sel_count || !keep_idx || !keep_count || !ws || cap < 0)
    return OCTGS_EINVAL;
  if (an->feat_dim != 32 || !an->pos || !an->feat || !an->level || !(an->d_max > 0.0f))
    return OCTGS_EINVAL;
  if (!net->w1 || !net->b1 || !net->w2 || !net->b2 || !net->w3 || !net->b3) return OCTGS_EINVAL;
  if (ws_bytes < octgs_skip_predict_workspace_bytes(cap)) return OCTGS_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  const int64_t c = std::max<int64_t>(cap, 1);
  const int64_t nblk = (c + kChunk - 1) / kChunk;
  uint8_t *flag = (uint8_t *)ws;
  uint64_t *masks = (uint64_t *)((char *)ws + ((c + 255) / 256) * 256);
  uint32_t *blk = (uint32_t *)((char *)masks + nblk * kGroups * 8);
  PredArgs a;
  a.f = feat_args(an, cam, sel_idx, sel_count, cap);
  a.w1 = net->w1; a.b1 = net->b1; a.w2 = net->w2; a.b2 = net->b2; a.w3 = net->w3; a.b3 = net->b3;
  a.thr = logit_threshold;
  a.flag = flag;
  a.logit = logits;
  const int grid = (int)std::min<int64_t>((c + kTM - 1) / kTM, 1024);
  hipLaunchKernelGGL(k_skip_predict, dim3(grid), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_flag_mark, dim3((unsigned)nblk), dim3(kBlock), 0, s, flag, sel_count, cap,
                     masks, blk);
  hipLaunchKernelGGL(k_flag_scatter, dim3((unsigned)nblk), dim3(kBlock), 0, s, sel_count, cap,
                     masks, blk, sel_idx, keep_idx, keep_count);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

size_t octgs_skip_train_workspace_bytes(int32_t batch) {
  if (batch < 1) return 0;
  return (size_t)train_blocks(batch) * kPartLen * sizeof(float);
}

int octgs_skip_train_grad(const octgs_skip_net *net, const float *z, const float *y,
                          const uint32_t *rows, int32_t batch, uint64_t input_mask,
                          float pos_weight, const octgs_skip_net_grads *gr, float *loss, void *ws,
                          size_t ws_bytes, octgs_stream stream) {
  if (!net || !z || !y || !gr || !loss || !ws || batch < 1) return OCTGS_EINVAL;
  if (!net->w1 || !net->b1 || !net->w2 || !net->b2 || !net->w3 || !net->b3) return OCTGS_EINVAL;
  if (!gr->w1 || !gr->b1 || !gr->w2 || !gr->b2 || !gr->w3 || !gr->b3) return OCTGS_EINVAL;
  if (ws_bytes < octgs_skip_train_workspace_bytes(batch)) return OCTGS_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  TrainArgs a;
  a.w1 = net->w1; a.b1 = net->b1; a.w2 = net->w2; a.b2 = net->b2; a.w3 = net->w3; a.b3 = net->b3;
  a.z = z;
  a.y = y;
  a.rows = rows;
  a.B = batch;
  a.in_mask = input_mask;
  a.pw = pos_weight;
  a.part = (float *)ws;
  const int nblk = train_blocks(batch);
  hipLaunchKernelGGL(k_skip_train, dim3(nblk), dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_skip_train_reduce, dim3((kPartLen + kBlock - 1) / kBlock), dim3(kBlock), 0,
                     s, (const float *)ws, nblk, *gr, loss);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

}  // extern "C"
