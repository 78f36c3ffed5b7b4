// Tiled FP32 GEMM used by the skip-predictor training: 64x64 output tiles,
// K in steps of 16 staged through LDS, 4x4 outputs per thread, optional
// split-K with atomic accumulation, and an epilogue with bias add and a
// ReLU-derivative mask.  One of M or K may be a device-resident count, so
// launches need no host synchronisation.
#include "octgs_internal.h"

namespace octgs {

namespace {

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(kBlock) void k_gemm(Gemm g) {
  __shared__ float As[GK][GT + 4];
  __shared__ float Bs[GK][GT + 4];
  const int sk = blockIdx.z;
  int M = g.M, K = g.K;
  if (g.dyn) {
    const int d = (int)min(*g.dyn, (uint32_t)g.dyn_cap);
    if (g.dyn_dim == 1) M = d; else K = d;
  }
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  if (m0 >= M || n0 >= g.N) return;
  const int kchunk = (K + g.splitk - 1) / g.splitk;
  const int kb = sk * kchunk, ke = min(K, kb + kchunk);
  if (kb >= ke) return;
  const int t = threadIdx.x, tx = t % 16, ty = t / 16;
  float acc[4][4] = {};
  for (int k0 = kb; k0 < ke; k0 += GK) {
    // 64 x 16 tile of op(A) and 16 x 64 tile of op(B), zero outside
    for (int i = t; i < GT * GK; i += kBlock) {
      const int mm = i / GK, kk = i % GK;
      const int m = m0 + mm, k = k0 + kk;
      float v = 0.0f;
      if (m < M && k < ke) v = g.transA ? g.A[(int64_t)k * g.lda + m] : g.A[(int64_t)m * g.lda + k];
      if (g.reluA) v = fmaxf(v, 0.0f);
      As[kk][mm] = v;
      const int nn = i % GT, kk2 = i / GT;
      const int n = n0 + nn, k2 = k0 + kk2;
      float w = 0.0f;
      if (n < g.N && k2 < ke) w = g.transB ? g.B[(int64_t)n * g.ldb + k2] : g.B[(int64_t)k2 * g.ldb + n];
      Bs[kk2][nn] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma_(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty * 4 + i;
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + tx * 4 + j;
      if (n >= g.N) continue;
      float v = acc[i][j];
      if (g.bias) v += g.bias[n];
      if (g.mask) v = g.mask[(int64_t)m * g.ldm + n] > 0.0f ? v : 0.0f;
      float *c = g.C + (int64_t)m * g.ldc + n;
      if (g.accumulate) {
        if (g.splitk > 1) atomicAdd(c, v); else *c += v;
      } else {
        *c = v;
      }
    }
  }
}

// column sums of Y[M][N] (row stride ld) added to out; rows strided over blocks
__global__ __launch_bounds__(kBlock) void k_colsum(const float *Y, int64_t ld, int N,
                                                   const uint32_t *dyn, int cap, float *out) {
  const int M = dyn ? (int)min(*dyn, (uint32_t)cap) : cap;
  const int n = threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int m = blockIdx.x; m < M; m += gridDim.x) s += Y[(int64_t)m * ld + n];
  if (s != 0.0f) atomicAdd(out + n, s);
}

__global__ void k_fill(float *p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

hipError_t colsum(const float *Y, int64_t ld, int N, const uint32_t *dyn, int cap, float *out,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3(256), dim3(kBlock), 0, s, Y, ld, N, dyn, cap, out);
  return hipGetLastError();
}

hipError_t fill(float *p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t gemm(const Gemm &g0, int64_t m_cap, hipStream_t s) {
  const int64_t mt = (std::max<int64_t>(m_cap, 1) + GT - 1) / GT;
  const int nt = (g0.N + GT - 1) / GT;
  hipLaunchKernelGGL(k_gemm, dim3(nt, (unsigned)mt, g0.splitk), dim3(kBlock), 0, s, g0);
  return hipGetLastError();
}

Gemm gemm_base() {
  Gemm g;
  memset(&g, 0, sizeof g);
  g.splitk = 1;
  return g;
}

}  // namespace octgs
