// Backward pass of the neural-Gaussian decode (Octree-GS Sec. III-B, Eq. 3
// and Eq. 4): from the gradients of the decoded Gaussian attributes to the
// gradients of the anchor features, positions, offsets, scalings and of the
// three MLP heads' weights and biases.
//
// Structure: the forward activations are recomputed (hidden pre-activations
// and head outputs), the activation derivatives give dY, and the products of
// each head's backward (dW2 = relu(H)^T dY, dH = dY W2^T masked by relu',
// dW1 = X^T dH, dX = dH W1^T) run on one tiled FP32 GEMM kernel, the three
// heads of a product in one grouped launch.  Weight gradients reduce over
// anchors with split-K blocks and atomics.  The anchor count lives on the
// device; every kernel reads it.
#include "octgs_internal.h"

namespace octgs {

namespace {

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + __expf(-x)); }

struct BwdDecodeArgs {
  int k, W, OT, F;
  int off[3], outs[3];
  float inv_dmax;
  float C[3];
  const float *pos, *feat, *offsets, *oscale, *bscale;
  const uint32_t *idx, *count;
  int cap_anchors;
  const float *dgauss;
  int64_t dstride;
  float *X, *Dn, *Y, *dY, *dX;
  float *gpos, *gfeat, *goff, *gosc, *gbsc;
};

// network input per listed anchor: X = [feature, dist / d_max, dir], Dn = (dist, dir)
// Network inputs of the listed anchors, 32 lanes per anchor (one feature
// each, coalesced 128-byte rows); lane 0 adds distance and direction.
constexpr int kGatherLanes = 32;

__global__ __launch_bounds__(kBlock) void k_bwd_gather(BwdDecodeArgs a) {
  const uint32_t M = min(*a.count, (uint32_t)a.cap_anchors);
  const int f = threadIdx.x % kGatherLanes;
  const uint32_t per = kBlock / kGatherLanes;
  for (uint32_t m = blockIdx.x * per + threadIdx.x / kGatherLanes; m < M; m += gridDim.x * per) {
    const uint32_t j = a.idx[m];
    float *x = a.X + (size_t)m * 36;
    x[f] = a.feat[(size_t)j * 32 + f];
    if (f == 0) {
      const float d0 = a.pos[3 * (size_t)j] - a.C[0], d1 = a.pos[3 * (size_t)j + 1] - a.C[1];
      const float d2 = a.pos[3 * (size_t)j + 2] - a.C[2];
      const float dist = sqrtf(fma_(d0, d0, fma_(d1, d1, d2 * d2)));
      const float inv = 1.0f / dist;
      x[32] = dist * a.inv_dmax;
      x[33] = d0 * inv; x[34] = d1 * inv; x[35] = d2 * inv;
      float *dn = a.Dn + (size_t)m * 4;
      dn[0] = dist; dn[1] = x[33]; dn[2] = x[34]; dn[3] = x[35];
    }
  }
}

// Sum over the 16 lanes of a DPP row (every lane of the row gets it).
__device__ __forceinline__ float row16_sum(float v) {
  v += __uint_as_float(dpp_u<kDppXor1>(__float_as_uint(v)));
  v += __uint_as_float(dpp_u<kDppXor2>(__float_as_uint(v)));
  v += __uint_as_float(dpp_u<kDppHalfMirror>(__float_as_uint(v)));
  v += __uint_as_float(dpp_u<kDppRor8>(__float_as_uint(v)));
  return v;
}

// Activation derivatives and the anchor-array gradients of Eq. 3 and the
// scale bound: one 16-lane row per anchor, lane i for Gaussian i (k <= 16),
// the anchor's sums over its Gaussians reduced within the row.
__global__ __launch_bounds__(kBlock) void k_act_bwd(BwdDecodeArgs a) {
  const uint32_t M = min(*a.count, (uint32_t)a.cap_anchors);
  const int k = a.k;
  const int i = threadIdx.x & 15;
  const uint32_t per = kBlock / 16;
  // every lane of a row runs the same iterations, so the row sums stay whole
  for (uint32_t m = blockIdx.x * per + threadIdx.x / 16; m < M; m += gridDim.x * per) {
    const uint32_t j = a.idx[m];
    const bool act = i < k;
    const int ii = act ? i : 0;
    const float *y = a.Y + (size_t)m * a.OT;
    float *dy = a.dY + (size_t)m * a.OT;
    const float *l = a.oscale + 3 * (size_t)j;
    const float *bs = a.bscale + 3 * (size_t)j;
    const size_t s = (size_t)m * k + ii;
    const float *o = a.offsets + ((size_t)j * k + ii) * 3;
    float *go = a.goff + ((size_t)j * k + ii) * 3;
    float dp[3], dl[3], dbs[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float dm = act ? a.dgauss[c * a.dstride + s] : 0.0f;
      dp[c] = dm;
      if (act) go[c] += dm * l[c];
      dl[c] = dm * o[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float sg = sigm(y[a.off[2] + 7 * ii + c]);
      const float dsc = act ? a.dgauss[(3 + c) * a.dstride + s] : 0.0f;
      dbs[c] = dsc * sg;
      if (act) dy[a.off[2] + 7 * ii + c] = dsc * bs[c] * sg * (1.0f - sg);
    }
    if (act) {
      const float q0 = y[a.off[2] + 7 * ii + 3], q1 = y[a.off[2] + 7 * ii + 4];
      const float q2 = y[a.off[2] + 7 * ii + 5], q3 = y[a.off[2] + 7 * ii + 6];
      const float n2 = fma_(q0, q0, fma_(q1, q1, fma_(q2, q2, q3 * q3)));
      float dq[4] = {0, 0, 0, 0};
      if (n2 > 0.0f) {
        const float inv = 1.0f / sqrtf(n2);
        const float u[4] = {q0 * inv, q1 * inv, q2 * inv, q3 * inv};
        float gq[4], dot = 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          gq[c] = a.dgauss[(6 + c) * a.dstride + s];
          dot = fma_(u[c], gq[c], dot);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) dq[c] = (gq[c] - u[c] * dot) * inv;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) dy[a.off[2] + 7 * ii + 3 + c] = dq[c];
      const float op = tanhf(y[a.off[0] + ii]);
      dy[a.off[0] + ii] = a.dgauss[10 * a.dstride + s] * (1.0f - op * op);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float sg = sigm(y[a.off[1] + 3 * ii + c]);
        dy[a.off[1] + 3 * ii + c] = a.dgauss[(11 + c) * a.dstride + s] * sg * (1.0f - sg);
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dp[c] = row16_sum(dp[c]);
      dl[c] = row16_sum(dl[c]);
      dbs[c] = row16_sum(dbs[c]);
    }
    if (i == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a.gpos[3 * (size_t)j + c] += dp[c];
        a.gosc[3 * (size_t)j + c] += dl[c];
        a.gbsc[3 * (size_t)j + c] += dbs[c];
      }
    }
  }
}

// Input gradients back to the anchor: features (32 lanes per anchor), and
// the position through the relative distance and the viewing direction.
__global__ __launch_bounds__(kBlock) void k_x_bwd(BwdDecodeArgs a) {
  const uint32_t M = min(*a.count, (uint32_t)a.cap_anchors);
  const int f = threadIdx.x % kGatherLanes;
  const uint32_t per = kBlock / kGatherLanes;
  for (uint32_t m = blockIdx.x * per + threadIdx.x / kGatherLanes; m < M; m += gridDim.x * per) {
    const uint32_t j = a.idx[m];
    const float *dx = a.dX + (size_t)m * 36;
    a.gfeat[(size_t)j * 32 + f] += dx[f];
    if (f == 0) {
      const float *dn = a.Dn + (size_t)m * 4;
      const float dist = dn[0], u0 = dn[1], u1 = dn[2], u2 = dn[3];
      const float dot = fma_(u0, dx[33], fma_(u1, dx[34], u2 * dx[35]));
      const float sd = dx[32] * a.inv_dmax, id = 1.0f / dist;
      a.gpos[3 * (size_t)j + 0] += fma_(u0, sd, (dx[33] - u0 * dot) * id);
      a.gpos[3 * (size_t)j + 1] += fma_(u1, sd, (dx[34] - u1 * dot) * id);
      a.gpos[3 * (size_t)j + 2] += fma_(u2, sd, (dx[35] - u2 * dot) * id);
    }
  }
}

struct BwdLayout {
  float *X, *Dn, *Hp, *Y, *dY, *dHp, *dX;
  size_t bytes;
};

BwdLayout bwd_layout(void *base, int64_t mcap, int k, int W) {
  BwdLayout L;
  char *p = (char *)base;
  size_t off = 0;
  auto take = [&](size_t b) -> float * {
    float *r = p ? (float *)(p + off) : nullptr;
    off += (b + 255) & ~(size_t)255;
    return r;
  };
  const int64_t m = std::max<int64_t>(mcap, 1);
  const int OT = 11 * k;
  L.X = take((size_t)m * 36 * 4);
  L.Dn = take((size_t)m * 4 * 4);
  L.Hp = take((size_t)m * 3 * W * 4);
  L.Y = take((size_t)m * OT * 4);
  L.dY = take((size_t)m * OT * 4);
  L.dHp = take((size_t)m * 3 * W * 4);
  L.dX = take((size_t)m * 36 * 4);
  L.bytes = off;
  return L;
}

}  // namespace

}  // namespace octgs

using namespace octgs;

extern "C" {

size_t octgs_decode_bwd_workspace_bytes(int64_t max_anchors, int32_t k, int32_t width) {
  if (max_anchors < 0 || k < 1 || k > kMaxK || width < 1) return 0;
  return bwd_layout(nullptr, max_anchors, k, width).bytes;
}

int octgs_decode_bwd(const octgs_anchors *an, const octgs_mlp *mlp, const octgs_camera *cam,
                     const uint32_t *idx, const uint32_t *count, const float *d_gauss,
                     int64_t gauss_capacity, const octgs_anchor_grads *ga,
                     const octgs_mlp_grads *gm, void *ws, size_t ws_bytes, octgs_stream stream) {
  if (!an || !mlp || !cam || !idx || !count || !d_gauss || !ga || !gm || !ws) return OCTGS_EINVAL;
  // transition blending is an inference-time mode; training uses Eq. 7 alone
  if (cam->lod_blend) return OCTGS_EUNSUPPORTED;
  if (an->feat_dim != 32) return OCTGS_EUNSUPPORTED;
  if (an->k < 1 || an->k > kMaxK) return OCTGS_EUNSUPPORTED;
  if (mlp->width < 16 || mlp->width > 64 || mlp->width % 16) return OCTGS_EUNSUPPORTED;
  if (!an->pos || !an->feat || !an->offsets || !an->offset_scale || !an->base_scale)
    return OCTGS_EINVAL;
  if (!ga->pos || !ga->feat || !ga->offsets || !ga->offset_scale || !ga->base_scale)
    return OCTGS_EINVAL;
  for (int h = 0; h < 3; ++h)
    if (!mlp->w1[h] || !mlp->b1[h] || !mlp->w2[h] || !mlp->b2[h] || !gm->w1[h] || !gm->b1[h] ||
        !gm->w2[h] || !gm->b2[h])
      return OCTGS_EINVAL;
  if (gauss_capacity < an->k || !(an->d_max > 0.0f)) return OCTGS_EINVAL;
  const int k = an->k, W = mlp->width;
  const int64_t mcap = gauss_capacity / k;
  if (mcap > 0x7fffffff) return OCTGS_EINVAL;
  if (ws_bytes < octgs_decode_bwd_workspace_bytes(mcap, k, W)) return OCTGS_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  BwdLayout L = bwd_layout(ws, mcap, k, W);
  BwdDecodeArgs a;
  a.k = k; a.W = W; a.OT = 11 * k; a.F = 32;
  a.outs[0] = k; a.outs[1] = 3 * k; a.outs[2] = 7 * k;
  a.off[0] = 0; a.off[1] = k; a.off[2] = 4 * k;
  a.inv_dmax = 1.0f / an->d_max;
  for (int c = 0; c < 3; ++c) a.C[c] = cam->C[c];
  a.pos = an->pos; a.feat = an->feat; a.offsets = an->offsets;
  a.oscale = an->offset_scale; a.bscale = an->base_scale;
  a.idx = idx; a.count = count; a.cap_anchors = (int)mcap;
  a.dgauss = d_gauss; a.dstride = gauss_capacity;
  a.X = L.X; a.Dn = L.Dn; a.Y = L.Y; a.dY = L.dY; a.dX = L.dX;
  a.gpos = ga->pos; a.gfeat = ga->feat; a.goff = ga->offsets;
  a.gosc = ga->offset_scale; a.gbsc = ga->base_scale;
  // the per-anchor kernels give each anchor a row of 16 or 32 lanes
  const int grid = (int)std::min<int64_t>((mcap * kGatherLanes + kBlock - 1) / kBlock, 4096);
  const int grid16 = (int)std::min<int64_t>((mcap * 16 + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_bwd_gather, dim3(grid), dim3(kBlock), 0, s, a);
  const int splitk = (int)std::min<int64_t>(std::max<int64_t>(mcap / 512, 1), 64);
  hipError_t e = hipSuccess;
  // Each product below runs for the three heads in one grouped launch.
  // Forward recompute: Hp_h = X W1_h + b1_h; Y_h = relu(Hp_h) W2_h + b2_h.
  Gemm g1 = gemm_base();
  g1.groups = 3;
  g1.lda = 36; g1.ldb = W; g1.ldc = 3 * W;
  g1.M = (int)mcap; g1.K = 36; g1.dyn = count; g1.dyn_dim = 1; g1.dyn_cap = (int)mcap;
  Gemm g2 = gemm_base();
  g2.groups = 3;
  g2.lda = 3 * W; g2.reluA = 1; g2.ldc = a.OT; g2.M = (int)mcap; g2.K = W;
  g2.dyn = count; g2.dyn_dim = 1; g2.dyn_cap = (int)mcap;
  // dW2_h += relu(Hp_h)^T dY_h
  Gemm g3 = gemm_base();
  g3.groups = 3;
  g3.lda = 3 * W; g3.transA = 1; g3.reluA = 1; g3.ldb = a.OT;
  g3.M = W; g3.K = (int)mcap; g3.dyn = count; g3.dyn_dim = 2; g3.dyn_cap = (int)mcap;
  g3.accumulate = 1; g3.splitk = splitk;
  // dHp_h = (dY_h W2_h^T) * (Hp_h > 0)
  Gemm g4 = gemm_base();
  g4.groups = 3;
  g4.lda = a.OT; g4.transB = 1; g4.ldc = 3 * W; g4.ldm = 3 * W;
  g4.M = (int)mcap; g4.dyn = count; g4.dyn_dim = 1; g4.dyn_cap = (int)mcap;
  // dW1_h += X^T dHp_h
  Gemm g5 = gemm_base();
  g5.groups = 3;
  g5.lda = 36; g5.transA = 1; g5.ldb = 3 * W; g5.ldc = W; g5.M = 36; g5.K = (int)mcap;
  g5.dyn = count; g5.dyn_dim = 2; g5.dyn_cap = (int)mcap; g5.accumulate = 1; g5.splitk = splitk;
  for (int h = 0; h < 3; ++h) {
    g1.A3[h] = L.X; g1.B3[h] = mlp->w1[h]; g1.C3[h] = L.Hp + h * W; g1.bias3[h] = mlp->b1[h];
    g1.N3[h] = W;
    g2.A3[h] = L.Hp + h * W; g2.B3[h] = mlp->w2[h]; g2.ldb3[h] = a.outs[h];
    g2.C3[h] = L.Y + a.off[h]; g2.bias3[h] = mlp->b2[h]; g2.N3[h] = a.outs[h];
    g3.A3[h] = L.Hp + h * W; g3.B3[h] = L.dY + a.off[h]; g3.C3[h] = gm->w2[h];
    g3.ldc3[h] = a.outs[h]; g3.N3[h] = a.outs[h];
    g4.A3[h] = L.dY + a.off[h]; g4.B3[h] = mlp->w2[h]; g4.ldb3[h] = a.outs[h];
    g4.C3[h] = L.dHp + h * W; g4.mask3[h] = L.Hp + h * W; g4.N3[h] = W; g4.K3[h] = a.outs[h];
    g5.A3[h] = L.X; g5.B3[h] = L.dHp + h * W; g5.C3[h] = gm->w1[h]; g5.N3[h] = W;
  }
  if ((e = gemm(g1, mcap, s)) != hipSuccess) return OCTGS_EHIP;
  if ((e = gemm(g2, mcap, s)) != hipSuccess) return OCTGS_EHIP;
  hipLaunchKernelGGL(k_act_bwd, dim3(grid16), dim3(kBlock), 0, s, a);
  if ((e = gemm(g3, W, s)) != hipSuccess) return OCTGS_EHIP;
  if ((e = gemm(g4, mcap, s)) != hipSuccess) return OCTGS_EHIP;
  if ((e = gemm(g5, 36, s)) != hipSuccess) return OCTGS_EHIP;
  {
    // db2_h += column sums of dY_h; db1_h += column sums of dHp_h
    const float *Y3[3] = {L.dY + a.off[0], L.dY + a.off[1], L.dY + a.off[2]};
    float *o3[3] = {gm->b2[0], gm->b2[1], gm->b2[2]};
    if ((e = colsum3(Y3, (int64_t)a.OT, a.outs, count, (int)mcap, o3, s)) != hipSuccess)
      return OCTGS_EHIP;
    const float *H3[3] = {L.dHp, L.dHp + W, L.dHp + 2 * W};
    float *p3[3] = {gm->b1[0], gm->b1[1], gm->b1[2]};
    const int nw[3] = {W, W, W};
    if ((e = colsum3(H3, (int64_t)(3 * W), nw, count, (int)mcap, p3, s)) != hipSuccess)
      return OCTGS_EHIP;
  }
  // dX = sum over heads of dHp_h W1_h^T (accumulated head by head)
  for (int h = 0; h < 3 && e == hipSuccess; ++h) {
    Gemm g6 = gemm_base();
    g6.A = L.dHp + h * W; g6.lda = 3 * W; g6.B = mlp->w1[h]; g6.ldb = W; g6.transB = 1;
    g6.C = L.dX; g6.ldc = 36; g6.M = (int)mcap; g6.N = 36; g6.K = W;
    g6.dyn = count; g6.dyn_dim = 1; g6.dyn_cap = (int)mcap; g6.accumulate = h > 0 ? 1 : 0;
    e = gemm(g6, mcap, s);
  }
  if (e != hipSuccess) return OCTGS_EHIP;
  hipLaunchKernelGGL(k_x_bwd, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

}  // extern "C"
