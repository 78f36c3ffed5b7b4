// Neural-Gaussian decode (Octree-GS Sec. III-B, Eq. 3 and Eq. 4): each
// selected anchor emits k Gaussians whose positions are x_v + O_i * l_v and
// whose opacity, colour, scale and rotation come from three 2-layer MLPs fed
// with the anchor feature, the relative viewing distance and the viewing
// direction.
//
// Mapping to CDNA4: a block (4 waves) decodes 32 anchors per iteration.  The
// two layers are GEMMs [32 x 36] x [36 x 3W] and, per head, [32 x W] x [W x out]
// run on MFMA; the block's waves split the output columns, so each wave keeps
// its slice of the weights (the B operands) in registers for the whole
// persistent loop, and only the activations go through LDS.  A first small
// kernel writes those B operands once per call into the caller's workspace,
// already rounded to the path's precision and in the lane order the MFMA
// reads them, so each block loads its slices with a few fully coalesced loads
// instead of staging and converting every weight itself.  Two variants:
//   FP32: v_mfma_f32_16x16x4_f32 on FP32 inputs and weights;
//   BF16: v_mfma_f32_16x16x16_bf16 on BF16 features, inputs and weights,
//         FP32 accumulation; biases, activations and the Gaussian assembly
//         stay FP32.
// Operand layouts (16x16xK, 64 lanes in four groups g = lane / 16):
//   A[m][k]: lane holds row m = lane % 16, k = g * K/4 + j
//   B[k][n]: lane holds col n = lane % 16, k = g * K/4 + j
//   D[m][n]: lane holds col n = lane % 16, rows m = 4 g + i, i = 0..3
#include "octgs_internal.h"

namespace octgs {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int kTM = 32;          // anchors per block iteration
constexpr int kIn = 36;          // feat (32) + distance + direction (3)
constexpr int kInPad = 48;       // layer-1 K padded to a multiple of 16
constexpr int kMaxW = 64;
constexpr int kMaxN1 = 3 * kMaxW;  // 192
constexpr int kMaxNO = 176;        // 16 + 48 + 112 for k = 16
constexpr int kXS = kInPad + 4;    // LDS row strides (elements)
constexpr int kHS = kMaxN1 + 4;
constexpr int kYS = kMaxNO + 1;


__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + __expf(-x)); }

struct DecodeArgs {
  int64_t n;
  int k, W, cap_anchors;
  float inv_dmax;
  float C[3];
  // LOD transition blending: opacity factor min(1, max(0, L* - L + 1))
  int blend, n_levels;
  float d_max, s;
  const uint8_t *level;
  const float *lod_bias;
  const float *pos, *feat, *offsets, *oscale, *bscale;
  const uint16_t *feat_bf16;
  const void *frag;  // weight fragments (Frag layout), written by k_decode_prep
  const uint32_t *idx, *count;
  float *out;
  int64_t cap;
  uint32_t *out_count;
  uint32_t *status;  // nullable: OCTGS_STATUS_TRUNCATED when the listed anchors exceed the capacity
};

// layer-2 column tile c -> (head, first output column of the tile in that head)
__device__ __forceinline__ void l2_tile(int c, int k, int &head, int &col0, int &ncol) {
  const int t0 = (k + 15) / 16, t1 = (3 * k + 15) / 16;
  if (c < t0) { head = 0; col0 = c * 16; ncol = k; }
  else if (c < t0 + t1) { head = 1; col0 = (c - t0) * 16; ncol = 3 * k; }
  else { head = 2; col0 = (c - t0 - t1) * 16; ncol = 7 * k; }
}

template <bool BF16>
struct alignas(16) Smem {
  typedef typename std::conditional<BF16, uint16_t, float>::type T;
  T X[kTM][kXS];
  T H[kTM][kHS];
  float Y[kTM][kYS];
  uint32_t aidx[kTM];
  float ofac[kTM];  // opacity factor per anchor (1 without blending)
};

// One of three pointers by a lane-varying index, without indexing the
// kernel-argument array through memory.
__device__ __forceinline__ const float *pick3(const float *const p[3], int h) {
  return h == 0 ? p[0] : (h == 1 ? p[1] : p[2]);
}

// Weight fragments in the workspace, per wave w (0..3) and column-tile slot
// q (0..2, tile w + 4 q), one 64-lane vector each:
//   B1[w][q][ks] (ks < KS1), B2[w][q][ks] (ks < KS2), bias1[w][q], bias2[w][q]
// An operand is one float (FP32 path) or four BF16 values (BF16 path).
template <bool BF16>
struct Frag {
  static constexpr int KS1 = BF16 ? kInPad / 16 : kIn / 4;   // 3 or 9 k-steps
  static constexpr int KS2 = BF16 ? kMaxW / 16 : kMaxW / 4;  // 4 or 16 k-steps (W <= 64)
  static constexpr int KV = BF16 ? 4 : 1;                     // k values per lane per step
  typedef typename std::conditional<BF16, s4, float>::type Op;
  static constexpr size_t n1 = 4 * 3 * KS1 * kWave, n2 = 4 * 3 * KS2 * kWave, nb = 4 * 3 * kWave;
  static constexpr size_t bytes = (n1 + n2) * sizeof(Op) + 2 * nb * sizeof(float);
};

struct PrepArgs {
  int k, W;
  const float *w1[3], *b1[3], *w2[3], *b2[3];
  void *ws;
};

// One thread per fragment lane: the operand element(s) the MFMA lane reads,
// zero outside the real rows and columns.
//   layer 1, tile ct = w + 4 q of the 3W columns: column n = 16 ct + lane % 16,
//     head n / W; k index ks * 4 KV + (lane / 16) KV + j of the 36 inputs
//   layer 2, tile c = w + 4 q of the padded output columns (l2_tile)
template <bool BF16>
__global__ __launch_bounds__(kBlock) void k_decode_prep(PrepArgs a) {
  typedef Frag<BF16> F;
  typedef typename F::Op Op;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int k = a.k, W = a.W;
  const int n1tiles = 3 * W / 16;
  const int n2tiles = (k + 15) / 16 + (3 * k + 15) / 16 + (7 * k + 15) / 16;
  Op *f1 = reinterpret_cast<Op *>(a.ws);
  Op *f2 = f1 + F::n1;
  float *fb1 = reinterpret_cast<float *>(f2 + F::n2);
  float *fb2 = fb1 + F::nb;
  const int l = i % kWave, g = l / 16, lc = l % 16;
  auto put = [&](Op *dst, const float (&v)[F::KV]) {
    if constexpr (BF16) {
      s4 s;
      s[0] = (short)f2bf(v[0]); s[1] = (short)f2bf(v[1]);
      s[2] = (short)f2bf(v[2]); s[3] = (short)f2bf(v[3]);
      *dst = s;
    } else {
      *dst = v[0];
    }
  };
  if (i < (int)F::n1) {
    const int ks = (i / kWave) % F::KS1, q = (i / kWave / F::KS1) % 3, w = i / kWave / F::KS1 / 3;
    const int ct = w + 4 * q;
    const int n = ct * 16 + lc;
    const bool on = ct < n1tiles;
    const int head = on ? n / W : 0, hc = on ? n - head * W : 0;
    float v[F::KV];
#pragma unroll
    for (int j = 0; j < F::KV; ++j) {
      const int kk = ks * (4 * F::KV) + g * F::KV + j;
      v[j] = (on && kk < kIn) ? pick3(a.w1, head)[kk * W + hc] : 0.0f;
    }
    put(f1 + i, v);
  } else if (i < (int)(F::n1 + F::n2)) {
    const int r = i - (int)F::n1;
    const int ks = (r / kWave) % F::KS2, q = (r / kWave / F::KS2) % 3, w = r / kWave / F::KS2 / 3;
    const int c = w + 4 * q;
    const bool on = c < n2tiles;
    int head = 0, col0 = 0, ncol = 0;
    if (on) l2_tile(c, k, head, col0, ncol);
    const int col = col0 + lc;
    const bool cv = on && col < ncol;
    float v[F::KV];
#pragma unroll
    for (int j = 0; j < F::KV; ++j) {
      const int kk = ks * (4 * F::KV) + g * F::KV + j;
      v[j] = (cv && kk < W) ? pick3(a.w2, head)[kk * ncol + col] : 0.0f;
    }
    put(f2 + r, v);
  } else if (i < (int)(F::n1 + F::n2 + F::nb)) {
    const int r = i - (int)(F::n1 + F::n2);
    const int q = (r / kWave) % 3, w = r / kWave / 3;
    const int ct = w + 4 * q;
    const int n = ct * 16 + lc;
    const bool on = ct < n1tiles;
    const int head = on ? n / W : 0, hc = on ? n - head * W : 0;
    fb1[r] = on ? pick3(a.b1, head)[hc] : 0.0f;
    const int c = w + 4 * q;
    const bool on2 = c < n2tiles;
    int h2 = 0, col0 = 0, ncol = 0;
    if (on2) l2_tile(c, k, h2, col0, ncol);
    const int col = col0 + lc;
    fb2[r] = (on2 && col < ncol) ? pick3(a.b2, h2)[col] : 0.0f;
  }
}

template <bool BF16>
__global__ __launch_bounds__(kBlock) void k_decode(DecodeArgs a) {
  typedef Frag<BF16> F;
  __shared__ Smem<BF16> sm;
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const int g = l / 16, lc = l % 16;
  const int k = a.k, W = a.W;
  const int n1tiles = 3 * W / 16;
  const int t0 = (k + 15) / 16, t1 = (3 * k + 15) / 16, t2 = (7 * k + 15) / 16;
  const int n2tiles = t0 + t1 + t2;
  const int off_c = t0 * 16, off_s = (t0 + t1) * 16;

  // blocks beyond the listed anchors exit before loading any weights
  const uint32_t m_total = min(*a.count, (uint32_t)a.cap_anchors);
  if (blockIdx.x == 0 && t == 0) {
    *a.out_count = m_total * (uint32_t)k;
    if (a.status && *a.count > (uint32_t)a.cap_anchors) atomicOr(a.status, OCTGS_STATUS_TRUNCATED);
  }
  if ((uint64_t)blockIdx.x * kTM >= m_total) return;

  // ---- weights of this wave's column tiles, kept in registers ----
  constexpr int KS1 = F::KS1, KS2 = F::KS2;
  const int ks2 = BF16 ? W / 16 : W / 4;
  typedef typename F::Op Op;
  const Op *f1 = reinterpret_cast<const Op *>(a.frag);
  const Op *f2 = f1 + F::n1;
  const float *fb1 = reinterpret_cast<const float *>(f2 + F::n2);
  const float *fb2 = fb1 + F::nb;
  Op B1[3][KS1], B2[3][KS2];
  float b1r[3], b2r[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int ks = 0; ks < KS1; ++ks) B1[q][ks] = f1[((w * 3 + q) * KS1 + ks) * kWave + l];
#pragma unroll
    for (int ks = 0; ks < KS2; ++ks) B2[q][ks] = f2[((w * 3 + q) * KS2 + ks) * kWave + l];
    b1r[q] = fb1[(w * 3 + q) * kWave + l];
    b2r[q] = fb2[(w * 3 + q) * kWave + l];
  }

  const int64_t cap = a.cap;

  for (uint32_t tile = blockIdx.x; tile * kTM < m_total; tile += gridDim.x) {
    const uint32_t r0 = tile * kTM;
    const int rows = (int)min((uint32_t)kTM, m_total - r0);
    // ---- gather the network inputs ----
    {
      const int r = t / 8, part = t % 8;  // 8 threads per anchor, 4 features each
      if (r < rows) {
        const uint32_t j = a.idx[r0 + r];
        if (part == 0) sm.aidx[r] = j;
        if constexpr (BF16) {
          const uint2 v = *(const uint2 *)(a.feat_bf16 + (size_t)j * 32 + part * 4);
          *(uint2 *)&sm.X[r][part * 4] = v;
        } else {
          const float4 v = *(const float4 *)(a.feat + (size_t)j * 32 + part * 4);
          sm.X[r][part * 4 + 0] = v.x; sm.X[r][part * 4 + 1] = v.y;
          sm.X[r][part * 4 + 2] = v.z; sm.X[r][part * 4 + 3] = v.w;
        }
        if (part == 0) {
          const float d0 = a.pos[3 * (size_t)j] - a.C[0];
          const float d1 = a.pos[3 * (size_t)j + 1] - a.C[1];
          const float d2 = a.pos[3 * (size_t)j + 2] - a.C[2];
          const float dist = sqrtf(__builtin_fmaf(d0, d0, __builtin_fmaf(d1, d1, d2 * d2)));
          const float inv = 1.0f / dist;
          float of = 1.0f;
          if (a.blend) {
            // fractional level L* = clamp(log2(d_max / (d s)) + Delta L, 0, K - 1)
            const float ls = fminf(fmaxf(log2f(a.d_max / (dist * a.s)) + a.lod_bias[j], 0.0f),
                                   (float)(a.n_levels - 1));
            of = fminf(fmaxf(ls - (float)a.level[j] + 1.0f, 0.0f), 1.0f);
          }
          sm.ofac[r] = of;
          float e[kInPad - 32];
          e[0] = dist * a.inv_dmax;
          e[1] = d0 * inv; e[2] = d1 * inv; e[3] = d2 * inv;
#pragma unroll
          for (int q = 4; q < kInPad - 32; ++q) e[q] = 0.0f;
#pragma unroll
          for (int q = 0; q < kInPad - 32; ++q) {
            if constexpr (BF16) sm.X[r][32 + q] = f2bf(e[q]);
            else sm.X[r][32 + q] = e[q];
          }
        }
      } else if (r < kTM) {
#pragma unroll
        for (int q = 0; q < 4; ++q) sm.X[r][part * 4 + q] = 0;
        if (part == 0)
          for (int q = 32; q < kInPad; ++q) sm.X[r][q] = 0;
      }
    }
    __syncthreads();

    // ---- layer 1: H = relu(X W1 + b1) ----
#pragma unroll
    for (int rt = 0; rt < kTM / 16; ++rt) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int ct = w + 4 * q;
        if (ct < n1tiles) {
          f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int ks = 0; ks < KS1; ++ks) {
            if constexpr (BF16) {
              const s4 av = *(const s4 *)&sm.X[rt * 16 + lc][ks * 16 + g * 4];
              acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, B1[q][ks], acc, 0, 0, 0);
            } else {
              const float av = sm.X[rt * 16 + lc][ks * 4 + g];
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, B1[q][ks], acc, 0, 0, 0);
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float h = fmaxf(acc[i] + b1r[q], 0.0f);
            if constexpr (BF16) sm.H[rt * 16 + 4 * g + i][ct * 16 + lc] = f2bf(h);
            else sm.H[rt * 16 + 4 * g + i][ct * 16 + lc] = h;
          }
        }
      }
    }
    __syncthreads();

    // ---- layer 2: Y_head = H_head W2_head + b2 ----
#pragma unroll
    for (int rt = 0; rt < kTM / 16; ++rt) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int c = w + 4 * q;
        if (c < n2tiles) {
          int head, col0, ncol;
          l2_tile(c, k, head, col0, ncol);
          const int hb = head * W;
          f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int ks = 0; ks < KS2; ++ks) {
            if (ks < ks2) {
              if constexpr (BF16) {
                const s4 av = *(const s4 *)&sm.H[rt * 16 + lc][hb + ks * 16 + g * 4];
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, B2[q][ks], acc, 0, 0, 0);
              } else {
                const float av = sm.H[rt * 16 + lc][hb + ks * 4 + g];
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, B2[q][ks], acc, 0, 0, 0);
              }
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) sm.Y[rt * 16 + 4 * g + i][c * 16 + lc] = acc[i] + b2r[q];
        }
      }
    }
    __syncthreads();

    // ---- activations and Gaussian assembly, coalesced planar stores ----
    const int items = rows * k;
    const size_t slot0 = (size_t)r0 * k;
    for (int it = t; it < items; it += kBlock) {
      const int r = it / k, i = it - r * k;
      const uint32_t j = sm.aidx[r];
      const size_t s = slot0 + it;
      const float *o = a.offsets + ((size_t)j * k + i) * 3;
      const float *ls = a.oscale + 3 * (size_t)j;
      const float *bs = a.bscale + 3 * (size_t)j;
      const float *p = a.pos + 3 * (size_t)j;
#pragma unroll
      for (int c = 0; c < 3; ++c) a.out[c * cap + s] = __builtin_fmaf(o[c], ls[c], p[c]);
#pragma unroll
      for (int c = 0; c < 3; ++c) a.out[(3 + c) * cap + s] = bs[c] * sigmoidf(sm.Y[r][off_s + 7 * i + c]);
      const float qw = sm.Y[r][off_s + 7 * i + 3], qx = sm.Y[r][off_s + 7 * i + 4];
      const float qy = sm.Y[r][off_s + 7 * i + 5], qz = sm.Y[r][off_s + 7 * i + 6];
      const float n2 = __builtin_fmaf(qw, qw, __builtin_fmaf(qx, qx, __builtin_fmaf(qy, qy, qz * qz)));
      float nw = 1.0f, nx = 0.0f, ny = 0.0f, nz = 0.0f;
      if (n2 > 0.0f) {
        const float inv = 1.0f / sqrtf(n2);
        nw = qw * inv; nx = qx * inv; ny = qy * inv; nz = qz * inv;
      }
      a.out[6 * cap + s] = nw; a.out[7 * cap + s] = nx;
      a.out[8 * cap + s] = ny; a.out[9 * cap + s] = nz;
      a.out[10 * cap + s] = tanhf(sm.Y[r][i]) * sm.ofac[r];
#pragma unroll
      for (int c = 0; c < 3; ++c) a.out[(11 + c) * cap + s] = sigmoidf(sm.Y[r][off_c + 3 * i + c]);
    }
    __syncthreads();
  }
}

__global__ void k_zero_count(uint32_t *p) { *p = 0u; }

}  // namespace

}  // namespace octgs

using namespace octgs;

extern "C" size_t octgs_decode_workspace_bytes(int32_t precision) {
  if (precision == OCTGS_BF16) return Frag<true>::bytes;
  if (precision == OCTGS_FP32) return Frag<false>::bytes;
  return 0;
}

extern "C" int octgs_decode(const octgs_anchors *an, const octgs_mlp *mlp,
                            const octgs_camera *cam, const uint32_t *idx, const uint32_t *count,
                            int precision, const octgs_gaussians *out, void *ws, size_t ws_bytes,
                            octgs_stream stream) {
  if (!an || !mlp || !cam || !idx || !count || !out) return OCTGS_EINVAL;
  if (!out->data || !out->count || out->capacity < 0) return OCTGS_EINVAL;
  if (an->feat_dim != 32) return OCTGS_EUNSUPPORTED;
  if (an->k < 1 || an->k > kMaxK) return OCTGS_EUNSUPPORTED;
  if (mlp->width < 16 || mlp->width > kMaxW || mlp->width % 16) return OCTGS_EUNSUPPORTED;
  if (precision != OCTGS_FP32 && precision != OCTGS_BF16) return OCTGS_EINVAL;
  if (!ws || ((uintptr_t)ws & 15) || ws_bytes < octgs_decode_workspace_bytes(precision))
    return OCTGS_EINVAL;
  if (an->n == 0) {  // nothing can be listed: the output is empty
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, (hipStream_t)stream, out->count);
    return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
  }
  if (!an->pos || !an->offsets || !an->offset_scale || !an->base_scale) return OCTGS_EINVAL;
  if (precision == OCTGS_FP32 && !an->feat) return OCTGS_EINVAL;
  if (precision == OCTGS_BF16 && !an->feat_bf16) return OCTGS_EINVAL;
  if (!(an->d_max > 0.0f)) return OCTGS_EINVAL;
  for (int h = 0; h < 3; ++h)
    if (!mlp->w1[h] || !mlp->b1[h] || !mlp->w2[h] || !mlp->b2[h]) return OCTGS_EINVAL;
  if (out->capacity / an->k > 0x7fffffff) return OCTGS_EINVAL;
  PrepArgs pa;
  pa.k = an->k;
  pa.W = mlp->width;
  for (int h = 0; h < 3; ++h) {
    pa.w1[h] = mlp->w1[h]; pa.b1[h] = mlp->b1[h]; pa.w2[h] = mlp->w2[h]; pa.b2[h] = mlp->b2[h];
  }
  pa.ws = ws;
  DecodeArgs a{};
  a.n = an->n;
  a.k = an->k;
  a.W = mlp->width;
  a.cap_anchors = (int)(out->capacity / an->k);
  a.inv_dmax = 1.0f / an->d_max;
  for (int c = 0; c < 3; ++c) a.C[c] = cam->C[c];
  a.pos = an->pos; a.feat = an->feat; a.feat_bf16 = an->feat_bf16;
  a.offsets = an->offsets; a.oscale = an->offset_scale; a.bscale = an->base_scale;
  a.frag = ws;
  a.blend = cam->lod_blend ? 1 : 0;
  if (a.blend) {
    if (!an->level || !an->lod_bias || an->n_levels < 1 || !(cam->lod_scale2 > 0.0f))
      return OCTGS_EINVAL;
  }
  a.n_levels = an->n_levels;
  a.d_max = an->d_max;
  a.s = sqrtf(cam->lod_scale2);
  a.level = an->level;
  a.lod_bias = an->lod_bias;
  a.idx = idx; a.count = count; a.out = out->data; a.cap = out->capacity;
  a.out_count = out->count;
  a.status = out->status;
  const int64_t tiles = std::max<int64_t>(1, (a.cap_anchors + kTM - 1) / kTM);
  // persistent blocks: each loads its weight slices once and loops over
  // tiles; as many as stay resident at once (2 FP32 or 4 BF16 blocks per
  // CU); blocks without a tile exit before loading weights
  const int grid = (int)std::min<int64_t>(tiles, precision == OCTGS_BF16 ? 1024 : 512);
  hipStream_t s = (hipStream_t)stream;
  if (precision == OCTGS_BF16) {
    constexpr size_t n = Frag<true>::n1 + Frag<true>::n2 + Frag<true>::nb;
    hipLaunchKernelGGL(k_decode_prep<true>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pa);
    hipLaunchKernelGGL(k_decode<true>, dim3(grid), dim3(kBlock), 0, s, a);
  } else {
    constexpr size_t n = Frag<false>::n1 + Frag<false>::n2 + Frag<false>::nb;
    hipLaunchKernelGGL(k_decode_prep<false>, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, pa);
    hipLaunchKernelGGL(k_decode<false>, dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}
