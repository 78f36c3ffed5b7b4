// Tiled FP32 GEMM used by the backward passes and the skip-predictor
// training: 64x64 output tiles, K in steps of 16 staged through LDS, 4x4
// outputs per thread, optional split-K with atomic accumulation, and an
// epilogue with bias add and a ReLU-derivative mask.  One of M or K may be a
// device-resident count, so launches need no host synchronisation.
#include "octgs_internal.h"

namespace octgs {

namespace {

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(kBlock) void k_gemm(Gemm g) {
  __shared__ float As[GK][GT + 4];
  __shared__ float Bs[GK][GT + 4];
  const int grp = blockIdx.z / g.splitk, sk = blockIdx.z % g.splitk;
  if (g.groups > 1) {
    g.A = g.A3[grp]; g.B = g.B3[grp]; g.C = g.C3[grp];
    g.bias = g.bias3[grp]; g.mask = g.mask3[grp]; g.N = g.N3[grp];
    if (g.K3[grp]) g.K = g.K3[grp];
    if (g.ldb3[grp]) g.ldb = g.ldb3[grp];
    if (g.ldc3[grp]) g.ldc = g.ldc3[grp];
  }
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

struct Colsum3 {
  const float *Y[3];
  float *out[3];
  int N[3];
};

// blockIdx.y selects the column set; rows are strided over blockIdx.x
__global__ __launch_bounds__(kBlock) void k_colsum(Colsum3 c, int64_t ld, const uint32_t *dyn,
                                                   int cap) {
  const int M = dyn ? (int)min(*dyn, (uint32_t)cap) : cap;
  const int gsel = blockIdx.y, n = threadIdx.x;
  if (n >= c.N[gsel]) return;
  const float *Y = c.Y[gsel];
  float s = 0.0f;
  for (int m = blockIdx.x; m < M; m += gridDim.x) s += Y[(int64_t)m * ld + n];
  if (s != 0.0f) atomicAdd(c.out[gsel] + n, s);
}

__global__ void k_fill(float *p, int64_t n, float v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

hipError_t colsum(const float *Y, int64_t ld, int N, const uint32_t *dyn, int cap, float *out,
                  hipStream_t s) {
  Colsum3 c;
  memset(&c, 0, sizeof c);
  c.Y[0] = Y; c.out[0] = out; c.N[0] = N;
  hipLaunchKernelGGL(k_colsum, dim3(256, 1), dim3(kBlock), 0, s, c, ld, dyn, cap);
  return hipGetLastError();
}

hipError_t colsum3(const float *const Y3[3], int64_t ld, const int N3[3], const uint32_t *dyn,
                   int cap, float *const out3[3], hipStream_t s) {
  Colsum3 c;
  for (int i = 0; i < 3; ++i) {
    c.Y[i] = Y3[i]; c.out[i] = out3[i]; c.N[i] = N3[i];
  }
  hipLaunchKernelGGL(k_colsum, dim3(256, 3), dim3(kBlock), 0, s, c, ld, dyn, cap);
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
  int nmax = g0.N;
  if (g0.groups > 1)
    for (int i = 0; i < g0.groups; ++i) nmax = std::max(nmax, g0.N3[i]);
  const int nt = (nmax + GT - 1) / GT;
  const int groups = std::max(g0.groups, 1);
  hipLaunchKernelGGL(k_gemm, dim3(nt, (unsigned)mt, g0.splitk * groups), dim3(kBlock), 0, s, g0);
  return hipGetLastError();
}

Gemm gemm_base() {
  Gemm g;
  memset(&g, 0, sizeof g);
  g.splitk = 1;
  g.groups = 1;
  return g;
}

}  // namespace octgs
