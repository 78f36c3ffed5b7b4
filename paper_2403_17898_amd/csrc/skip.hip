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
// Training (FP32, binary cross-entropy) runs on the tiled GEMM.
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

// Binary cross-entropy on logits, mean over the batch, positives weighted:
// d = wgt (sigmoid(x) - y) / B; loss += wgt * (softplus(x) - y x) / B.
__global__ __launch_bounds__(kBlock) void k_bce(const float *x, const float *y, int B, float pw,
                                                float *d, float *loss) {
  __shared__ float red[4];
  float acc = 0.0f;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < B; i += gridDim.x * kBlock) {
    const float xi = x[i], yi = y[i];
    const float wgt = yi > 0.5f ? pw : 1.0f;
    const float sg = 1.0f / (1.0f + __expf(-xi));
    d[i] = wgt * (sg - yi) / (float)B;
    const float sp = fmaxf(xi, 0.0f) + log1pf(__expf(-fabsf(xi)));
    acc += wgt * (sp - yi * xi);
  }
  acc = block_sum_f(acc, red);  // one atomic per block on the loss
  if (threadIdx.x == 0 && acc != 0.0f) atomicAdd(loss, acc / (float)B);
}

struct TrainLayout {
  float *H1, *H2, *X3, *dX3, *dH2, *dH1;
  size_t bytes;
};

TrainLayout train_layout(void *base, int B) {
  TrainLayout L;
  char *p = (char *)base;
  size_t off = 0;
  auto take = [&](size_t b) -> float * {
    float *r = p ? (float *)(p + off) : nullptr;
    off += (b + 255) & ~(size_t)255;
    return r;
  };
  const size_t m = (size_t)std::max(B, 1);
  L.H1 = take(m * kH * 4);
  L.H2 = take(m * kH * 4);
  L.X3 = take(m * 4);
  L.dX3 = take(m * 4);
  L.dH2 = take(m * kH * 4);
  L.dH1 = take(m * kH * 4);
  L.bytes = off;
  return L;
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
  return train_layout(nullptr, batch).bytes;
}

int octgs_skip_train_grad(const octgs_skip_net *net, const float *z, const float *y, int32_t batch,
                          float pos_weight, const octgs_skip_net_grads *gr, float *loss, void *ws,
                          size_t ws_bytes, octgs_stream stream) {
  if (!net || !z || !y || !gr || !loss || !ws || batch < 1) return OCTGS_EINVAL;
  if (!net->w1 || !net->b1 || !net->w2 || !net->b2 || !net->w3 || !net->b3) return OCTGS_EINVAL;
  if (!gr->w1 || !gr->b1 || !gr->w2 || !gr->b2 || !gr->w3 || !gr->b3) return OCTGS_EINVAL;
  if (ws_bytes < octgs_skip_train_workspace_bytes(batch)) return OCTGS_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  TrainLayout L = train_layout(ws, batch);
  const int B = batch;
  const int splitk = std::max(1, std::min(64, B / 256));
  hipError_t e = hipSuccess;
  // gradients are overwritten
  e = fill(gr->w1, kZ * kH, 0.0f, s);
  if (e == hipSuccess) e = fill(gr->b1, kH, 0.0f, s);
  if (e == hipSuccess) e = fill(gr->w2, kH * kH, 0.0f, s);
  if (e == hipSuccess) e = fill(gr->b2, kH, 0.0f, s);
  if (e == hipSuccess) e = fill(gr->w3, kH, 0.0f, s);
  if (e == hipSuccess) e = fill(gr->b3, 1, 0.0f, s);
  if (e != hipSuccess) return OCTGS_EHIP;
  Gemm g = gemm_base();
  g.A = z; g.lda = kZ; g.B = net->w1; g.ldb = kH; g.C = L.H1; g.ldc = kH;
  g.M = B; g.N = kH; g.K = kZ; g.bias = net->b1;
  if ((e = gemm(g, B, s)) != hipSuccess) return OCTGS_EHIP;
  g = gemm_base();
  g.A = L.H1; g.lda = kH; g.reluA = 1; g.B = net->w2; g.ldb = kH; g.C = L.H2; g.ldc = kH;
  g.M = B; g.N = kH; g.K = kH; g.bias = net->b2;
  if ((e = gemm(g, B, s)) != hipSuccess) return OCTGS_EHIP;
  g = gemm_base();
  g.A = L.H2; g.lda = kH; g.reluA = 1; g.B = net->w3; g.ldb = 1; g.C = L.X3; g.ldc = 1;
  g.M = B; g.N = 1; g.K = kH; g.bias = net->b3;
  if ((e = gemm(g, B, s)) != hipSuccess) return OCTGS_EHIP;
  hipLaunchKernelGGL(k_bce, dim3(std::min(1024, (B + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     L.X3, y, B, pos_weight, L.dX3, loss);
  // layer 3
  g = gemm_base();
  g.A = L.H2; g.lda = kH; g.transA = 1; g.reluA = 1; g.B = L.dX3; g.ldb = 1; g.C = gr->w3; g.ldc = 1;
  g.M = kH; g.N = 1; g.K = B; g.accumulate = 1; g.splitk = splitk;
  if ((e = gemm(g, kH, s)) != hipSuccess) return OCTGS_EHIP;
  if ((e = colsum(L.dX3, 1, 1, nullptr, B, gr->b3, s)) != hipSuccess) return OCTGS_EHIP;
  g = gemm_base();
  g.A = L.dX3; g.lda = 1; g.B = net->w3; g.ldb = 1; g.transB = 1; g.C = L.dH2; g.ldc = kH;
  g.M = B; g.N = kH; g.K = 1; g.mask = L.H2; g.ldm = kH;
  if ((e = gemm(g, B, s)) != hipSuccess) return OCTGS_EHIP;
  // layer 2
  g = gemm_base();
  g.A = L.H1; g.lda = kH; g.transA = 1; g.reluA = 1; g.B = L.dH2; g.ldb = kH; g.C = gr->w2; g.ldc = kH;
  g.M = kH; g.N = kH; g.K = B; g.accumulate = 1; g.splitk = splitk;
  if ((e = gemm(g, kH, s)) != hipSuccess) return OCTGS_EHIP;
  if ((e = colsum(L.dH2, kH, kH, nullptr, B, gr->b2, s)) != hipSuccess) return OCTGS_EHIP;
  g = gemm_base();
  g.A = L.dH2; g.lda = kH; g.B = net->w2; g.ldb = kH; g.transB = 1; g.C = L.dH1; g.ldc = kH;
  g.M = B; g.N = kH; g.K = kH; g.mask = L.H1; g.ldm = kH;
  if ((e = gemm(g, B, s)) != hipSuccess) return OCTGS_EHIP;
  // layer 1
  g = gemm_base();
  g.A = z; g.lda = kZ; g.transA = 1; g.B = L.dH1; g.ldb = kH; g.C = gr->w1; g.ldc = kH;
  g.M = kZ; g.N = kH; g.K = B; g.accumulate = 1; g.splitk = splitk;
  if ((e = gemm(g, kZ, s)) != hipSuccess) return OCTGS_EHIP;
  if ((e = colsum(L.dH1, kH, kH, nullptr, B, gr->b1, s)) != hipSuccess) return OCTGS_EHIP;
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

}  // extern "C"
