// Training-step helpers: the mean-L1 image loss gradient and the Adam update
// (Octree-GS trains its scenes with image losses; the optimiser is the usual
// Adam).  Both are elementwise streams over HBM.
#include "octgs_internal.h"

namespace octgs {

namespace {

// Grid-stride over float4 groups, four groups per thread per step with all
// loads issued before any use; one atomic per block for the loss (every
// atomic on the one loss address is serialised across the XCDs, so the grid
// stays small).  The tail (n % 4 elements) and unaligned arrays take the
// scalar loop.
__device__ __forceinline__ float l1_one(float d, float scale, float &acc) {
  acc += fabsf(d);
  return d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f);
}

__global__ __launch_bounds__(kBlock) void k_l1(const float *__restrict__ img,
                                               const float *__restrict__ tgt, int64_t n,
                                               float scale, float *__restrict__ dimg,
                                               float *__restrict__ loss) {
  __shared__ float red[4];
  float acc = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool vec = (((uintptr_t)img | (uintptr_t)tgt | (uintptr_t)dimg) & 15) == 0;
  const int64_t n4 = vec ? n / 4 : 0;
  const float4 *a4 = reinterpret_cast<const float4 *>(img);
  const float4 *b4 = reinterpret_cast<const float4 *>(tgt);
  float4 *d4 = reinterpret_cast<float4 *>(dimg);
  for (int64_t i0 = tid; i0 < n4; i0 += 4 * stride) {
    float4 a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = min(i0 + u * stride, n4 - 1);
      a[u] = a4[i];
      b[u] = b4[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n4) {
        float4 d;
        d.x = l1_one(a[u].x - b[u].x, scale, acc);
        d.y = l1_one(a[u].y - b[u].y, scale, acc);
        d.z = l1_one(a[u].z - b[u].z, scale, acc);
        d.w = l1_one(a[u].w - b[u].w, scale, acc);
        d4[i] = d;
      }
    }
  }
  for (int64_t i = 4 * n4 + tid; i < n; i += stride) dimg[i] = l1_one(img[i] - tgt[i], scale, acc);
  acc = block_sum_f(acc, red);
  if (threadIdx.x == 0 && acc != 0.0f) atomicAdd(loss, acc * scale);
}

__global__ __launch_bounds__(kBlock) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                                 float *__restrict__ m, float *__restrict__ v,
                                                 int64_t n, float lr, float b1, float b2, float eps,
                                                 float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const float gi = g[i];
    const float mi = __builtin_fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = __builtin_fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

// Several parameter arrays in one launch: each block updates one chunk of
// kAdamChunk elements of one array; the block finds its array from the
// prefix counts of blocks (uniform per block, scalar selects).
constexpr int kAdamMax = 32;
constexpr int kAdamChunk = 16 * kBlock;

struct AdamMany {
  float *p[kAdamMax];
  const float *g[kAdamMax];
  float *m[kAdamMax], *v[kAdamMax];
  int64_t n[kAdamMax];
  uint32_t bstart[kAdamMax + 1];  // first block of each array
  int count;
};

__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, float lr, float b1,
                                         float b2, float eps, float c1, float c2) {
  m = __builtin_fmaf(b1, m, (1.0f - b1) * g);
  v = __builtin_fmaf(b2, v, (1.0f - b2) * g * g);
  p -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// Each block updates one kAdamChunk-element chunk of one array: four float4
// groups per thread, all of their loads issued before the first update (the
// compiler cannot reorder loads across the stores itself, the arrays may
// alias as far as it knows).  Arrays whose four pointers are not 16-byte
// aligned, and the end of an array, take the scalar loop.
__global__ __launch_bounds__(kBlock) void k_adam_many(AdamMany a, float lr, float b1, float b2,
                                                      float eps, float c1, float c2) {
  const uint32_t b = blockIdx.x;
  float *p = a.p[0], *m = a.m[0], *v = a.v[0];
  const float *g = a.g[0];
  int64_t n = a.n[0];
  uint32_t b0 = 0;
#pragma unroll
  for (int r = 1; r < kAdamMax; ++r)
    if (r < a.count && a.bstart[r] <= b) {
      p = a.p[r]; g = a.g[r]; m = a.m[r]; v = a.v[r]; n = a.n[r]; b0 = a.bstart[r];
    }
  const int64_t e0 = (int64_t)(b - b0) * kAdamChunk;
  const int64_t e1 = min(n, e0 + kAdamChunk);
  const bool vec = (((uintptr_t)p | (uintptr_t)g | (uintptr_t)m | (uintptr_t)v) & 15) == 0;
  const int t = threadIdx.x;
  int64_t done = e0;
  if (vec && e1 - e0 == kAdamChunk) {
    constexpr int U = kAdamChunk / (4 * kBlock);
    float4 pv[U], gv[U], mv[U], vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = e0 / 4 + u * kBlock + t;
      pv[u] = reinterpret_cast<const float4 *>(p)[i];
      gv[u] = reinterpret_cast<const float4 *>(g)[i];
      mv[u] = reinterpret_cast<const float4 *>(m)[i];
      vv[u] = reinterpret_cast<const float4 *>(v)[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      adam_one(pv[u].x, gv[u].x, mv[u].x, vv[u].x, lr, b1, b2, eps, c1, c2);
      adam_one(pv[u].y, gv[u].y, mv[u].y, vv[u].y, lr, b1, b2, eps, c1, c2);
      adam_one(pv[u].z, gv[u].z, mv[u].z, vv[u].z, lr, b1, b2, eps, c1, c2);
      adam_one(pv[u].w, gv[u].w, mv[u].w, vv[u].w, lr, b1, b2, eps, c1, c2);
      const int64_t i = e0 / 4 + u * kBlock + t;
      reinterpret_cast<float4 *>(p)[i] = pv[u];
      reinterpret_cast<float4 *>(m)[i] = mv[u];
      reinterpret_cast<float4 *>(v)[i] = vv[u];
    }
    done = e1;
  }
  for (int64_t e = done + t; e < e1; e += kBlock) {
    float pe = p[e], me = m[e], ve = v[e];
    adam_one(pe, g[e], me, ve, lr, b1, b2, eps, c1, c2);
    m[e] = me;
    v[e] = ve;
    p[e] = pe;
  }
}

}  // namespace

}  // namespace octgs

using namespace octgs;

extern "C" {

int octgs_l1_loss_grad(const float *img, const float *target, int64_t n, float scale, float *dimg,
                       float *loss, octgs_stream stream) {
  if (n < 0 || (n > 0 && (!img || !target || !dimg || !loss))) return OCTGS_EINVAL;
  if (n == 0) return OCTGS_OK;
  const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 512);
  hipLaunchKernelGGL(k_l1, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, img, target, n, scale,
                     dimg, loss);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, float lr,
                    float beta1, float beta2, float eps, int32_t step, octgs_stream stream) {
  if (n < 0 || step < 1 || (n > 0 && (!param || !grad || !m || !v))) return OCTGS_EINVAL;
  if (n == 0) return OCTGS_OK;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
  const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_adam, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, param, grad, m, v,
                     n, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_adam_step_many(int32_t count, float *const *params, const float *const *grads,
                         float *const *m, float *const *v, const int64_t *n, float lr,
                         float beta1, float beta2, float eps, int32_t step, octgs_stream stream) {
  if (count < 0 || step < 1 || (count > 0 && (!params || !grads || !m || !v || !n)))
    return OCTGS_EINVAL;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
  for (int base = 0; base < count; base += kAdamMax) {
    AdamMany a;
    memset(&a, 0, sizeof a);
    a.count = std::min(kAdamMax, count - base);
    int64_t blocks = 0;
    for (int q = 0; q < a.count; ++q) {
      const int i = base + q;
      if (n[i] < 0 || (n[i] > 0 && (!params[i] || !grads[i] || !m[i] || !v[i]))) return OCTGS_EINVAL;
      a.p[q] = params[i]; a.g[q] = grads[i]; a.m[q] = m[i]; a.v[q] = v[i]; a.n[q] = n[i];
      a.bstart[q] = (uint32_t)blocks;
      blocks += (n[i] + kAdamChunk - 1) / kAdamChunk;
    }
    a.bstart[a.count] = (uint32_t)blocks;
    if (blocks == 0) continue;
    if (blocks > 0x7fffffff) return OCTGS_EINVAL;
    hipLaunchKernelGGL(k_adam_many, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream, a,
                       lr, beta1, beta2, eps, c1, c2);
    if (hipGetLastError() != hipSuccess) return OCTGS_EHIP;
  }
  return OCTGS_OK;
}

}  // extern "C"
