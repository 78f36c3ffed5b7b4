// Training losses of the framework (Sec. V, implementation details): the
// photometric loss w_l1 * L1 + w_ssim * (1 - SSIM) of the 3D-GS model
// (0.8 / 0.2) and the volume regularisation sum_i Prod(s_i) of the
// Scaffold-GS model (weight 0.01).
//
// SSIM (Wang et al. 2004, the standard form the paper refers to): an 11 x 11
// Gaussian window (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, windowed statistics
// as a same-size correlation with zeros outside the image, per channel
// image, averaged over all images and pixels.  Its gradient needs the window
// correlation twice: once for the statistics, once (the adjoint; the window
// is symmetric) for the three per-pixel derivative maps
//   dS/dmu_x = S (2 mu_y / A1 - 2 mu_y / A2 - 2 mu_x / B1 + 2 mu_x / B2),
//   dS/dE[x^2] = -S / B2,  dS/dE[xy] = 2 S / A2,
// with A1 = 2 mu_x mu_y + C1, A2 = 2 s_xy + C2, B1 = mu_x^2 + mu_y^2 + C1,
// B2 = s_xx + s_yy + C2, so dS/dx = w * m0 + 2 x (w * m1) + y (w * m2).
//
// Two tiled passes over 64 x 16 output tiles, one block per tile and
// channel image.  Each stages its input with a 5-pixel halo in LDS and runs
// the separable window as a horizontal then a vertical sweep, each thread
// producing four adjacent outputs from one register window (14 taps loaded
// for 4 x 11 products).  Pass 1 writes the three derivative maps (scaled by
// -w_ssim / n) to the workspace; pass 2 correlates them, adds the L1 term
// and writes the image gradient.  Each block leaves one partial loss sum; a
// final block adds them in double, in a fixed order.
#include "octgs_internal.h"

namespace octgs {

namespace {

constexpr int kSW = 64, kSH = 16, kR = 5, kTaps = 2 * kR + 1;
constexpr int kRW = kSW + 2 * kR, kRH = kSH + 2 * kR;  // 74 x 26 staged region
constexpr float kC1 = 0.0001f, kC2 = 0.0009f;

__device__ __forceinline__ int64_t block_index() {
  return ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}

int64_t ssim_blocks(int64_t n_images, int32_t height, int32_t width) {
  return (int64_t)((width + kSW - 1) / kSW) * ((height + kSH - 1) / kSH) * n_images;
}

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

struct SsimArgs {
  const float *x, *y;
  float *m0, *m1, *m2;  // derivative maps (workspace)
  float *part;          // per-block loss partial sums: [2][blocks] (workspace)
  float *dimg, *loss;
  int H, W;
  float w_l1, w_ssim, inv_n;
  float g[kTaps];
};

// Stage `nmaps` planes of the (kRH x kRW) region around the block's tile
// (zeros outside the image).
template <int NM>
__device__ __forceinline__ void stage(const float *const *src, int64_t base, int H, int W,
                                      float (*dst)[kRH][kRW]) {
  const int x0 = blockIdx.x * kSW - kR, y0 = blockIdx.y * kSH - kR;
  for (int i = threadIdx.x; i < kRH * kRW; i += kBlock) {
    const int r = i / kRW, c = i - r * kRW;
    const int gy = y0 + r, gx = x0 + c;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const int64_t o = base + (int64_t)(in ? gy : 0) * W + (in ? gx : 0);
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      const float v = src[m][o];
      dst[m][r][c] = in ? v : 0.0f;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_ssim_fwd(SsimArgs a) {
  __shared__ float in[2][kRH][kRW];
  __shared__ float hs[5][kRH][kSW];
  __shared__ float red[4];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.z * a.H * a.W;
  {
    const float *src[2] = {a.x, a.y};
    stage<2>(src, base, a.H, a.W, in);
  }
  __syncthreads();
  // horizontal sweep: rows of the region, 4 outputs per task
  for (int task = t; task < kRH * (kSW / 4); task += kBlock) {
    const int r = task / (kSW / 4), j0 = (task % (kSW / 4)) * 4;
    float xv[kTaps + 3], yv[kTaps + 3];
#pragma unroll
    for (int q = 0; q < kTaps + 3; ++q) {
      xv[q] = in[0][r][j0 + q];
      yv[q] = in[1][r][j0 + q];
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f, s4 = 0.0f;
#pragma unroll
      for (int q = 0; q < kTaps; ++q) {
        const float X = xv[o + q], Y = yv[o + q];
        const float gX = a.g[q] * X, gY = a.g[q] * Y;
        s0 += gX;
        s1 += gY;
        s2 = fma_(gX, X, s2);
        s3 = fma_(gY, Y, s3);
        s4 = fma_(gX, Y, s4);
      }
      hs[0][r][j0 + o] = s0; hs[1][r][j0 + o] = s1; hs[2][r][j0 + o] = s2;
      hs[3][r][j0 + o] = s3; hs[4][r][j0 + o] = s4;
    }
  }
  __syncthreads();
  // vertical sweep: 4 rows per thread at one column; SSIM and its partials
  const int j = t % kSW, r0 = (t / kSW) * 4;
  float st[5][4];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    float v[kTaps + 3];
#pragma unroll
    for (int q = 0; q < kTaps + 3; ++q) v[q] = hs[k][r0 + q][j];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < kTaps; ++q) s = fma_(a.g[q], v[o + q], s);
      st[k][o] = s;
    }
  }
  const int gx = blockIdx.x * kSW + j;
  const float coef = -a.w_ssim * a.inv_n;
  float acc = 0.0f;
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    const int gy = blockIdx.y * kSH + r0 + o;
    if (gx < a.W && gy < a.H) {
      const float mx = st[0][o], my = st[1][o];
      const float sxx = st[2][o] - mx * mx, syy = st[3][o] - my * my, sxy = st[4][o] - mx * my;
      const float A1 = fma_(2.0f * mx, my, kC1), A2 = fma_(2.0f, sxy, kC2);
      const float B1 = fma_(mx, mx, fma_(my, my, kC1)), B2 = sxx + syy + kC2;
      const float iA1 = 1.0f / A1, iA2 = 1.0f / A2, iB1 = 1.0f / B1, iB2 = 1.0f / B2;
      const float S = A1 * A2 * iB1 * iB2;
      acc += S;
      const int64_t o_ = base + (int64_t)gy * a.W + gx;
      a.m0[o_] = coef * S * 2.0f * (my * (iA1 - iA2) + mx * (iB2 - iB1));
      a.m1[o_] = coef * (-S * iB2);
      a.m2[o_] = coef * (2.0f * S * iA2);
    }
  }
  acc = block_sum_f(acc, red);
  if (t == 0) a.part[block_index()] = coef * acc;
}

__global__ __launch_bounds__(kBlock) void k_ssim_bwd(SsimArgs a) {
  __shared__ float in[3][kRH][kRW];
  __shared__ float hs[3][kRH][kSW];
  __shared__ float red[4];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.z * a.H * a.W;
  {
    const float *src[3] = {a.m0, a.m1, a.m2};
    stage<3>(src, base, a.H, a.W, in);
  }
  __syncthreads();
  for (int task = t; task < kRH * (kSW / 4); task += kBlock) {
    const int r = task / (kSW / 4), j0 = (task % (kSW / 4)) * 4;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      float v[kTaps + 3];
#pragma unroll
      for (int q = 0; q < kTaps + 3; ++q) v[q] = in[m][r][j0 + q];
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        float s = 0.0f;
#pragma unroll
        for (int q = 0; q < kTaps; ++q) s = fma_(a.g[q], v[o + q], s);
        hs[m][r][j0 + o] = s;
      }
    }
  }
  __syncthreads();
  const int j = t % kSW, r0 = (t / kSW) * 4;
  float cv[3][4];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    float v[kTaps + 3];
#pragma unroll
    for (int q = 0; q < kTaps + 3; ++q) v[q] = hs[m][r0 + q][j];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float s = 0.0f;
#pragma unroll
      for (int q = 0; q < kTaps; ++q) s = fma_(a.g[q], v[o + q], s);
      cv[m][o] = s;
    }
  }
  const int gx = blockIdx.x * kSW + j;
  const float l1 = a.w_l1 * a.inv_n;
  float acc = 0.0f;
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    const int gy = blockIdx.y * kSH + r0 + o;
    if (gx < a.W && gy < a.H) {
      const int64_t o_ = base + (int64_t)gy * a.W + gx;
      const float X = a.x[o_], Y = a.y[o_];
      const float d = X - Y;
      const float sg = d > 0.0f ? l1 : (d < 0.0f ? -l1 : 0.0f);
      a.dimg[o_] = fma_(2.0f * X, cv[1][o], fma_(Y, cv[2][o], cv[0][o])) + sg;
      acc += fabsf(d);
    }
  }
  acc = block_sum_f(acc, red);
  if (t == 0) a.part[(int64_t)gridDim.x * gridDim.y * gridDim.z + block_index()] = l1 * acc;
}

// One block: *loss += w_ssim + the per-block partial sums, added in double
// in a fixed order (the loss is the same bit for bit on every run).
__global__ __launch_bounds__(kBlock) void k_loss_finish(const float *__restrict__ part, int64_t n,
                                                        float base, float *__restrict__ loss) {
  __shared__ double red[kBlock];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) s += (double)part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)((double)*loss + (double)base + red[0]);
}

// L1 only (w_ssim = 0): elementwise, four independent elements per step.
__global__ __launch_bounds__(kBlock) void k_l1_only(const float *__restrict__ x,
                                                    const float *__restrict__ y, int64_t n,
                                                    float scale, float *__restrict__ dimg,
                                                    float *__restrict__ loss) {
  __shared__ float red[4];
  float acc = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x; i0 < n; i0 += 4 * stride) {
    float d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = min(i0 + u * stride, n - 1);
      d[u] = x[i] - y[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < n) {
        dimg[i] = d[u] > 0.0f ? scale : (d[u] < 0.0f ? -scale : 0.0f);
        acc += fabsf(d[u]);
      }
    }
  }
  acc = block_sum_f(acc, red);
  if (threadIdx.x == 0 && acc != 0.0f) atomicAdd(loss, acc * scale);
}

// Volume regularisation over the rendered slots (opacity > 0).
__global__ __launch_bounds__(kBlock) void k_volume(const float *__restrict__ g, int64_t cap,
                                                   const uint32_t *__restrict__ count, float w,
                                                   float *__restrict__ dg, float *__restrict__ loss) {
  __shared__ float red[4];
  const int64_t n = min((int64_t)*count, cap);
  float acc = 0.0f;
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * kBlock) {
    const float op = g[10 * cap + s];
    const float s0 = g[3 * cap + s], s1 = g[4 * cap + s], s2 = g[5 * cap + s];
    if (op > 0.0f) {
      acc = fma_(s0 * s1, s2, acc);
      dg[3 * cap + s] += w * (s1 * s2);
      dg[4 * cap + s] += w * (s0 * s2);
      dg[5 * cap + s] += w * (s0 * s1);
    }
  }
  acc = block_sum_f(acc, red);
  if (threadIdx.x == 0 && acc != 0.0f) atomicAdd(loss, w * acc);
}

}  // namespace

}  // namespace octgs

using namespace octgs;

extern "C" {

size_t octgs_photometric_workspace_bytes(int64_t n_images, int32_t height, int32_t width) {
  if (n_images < 0 || height < 0 || width < 0) return 0;
  return (size_t)(3 * n_images * (int64_t)height * width +
                  2 * ssim_blocks(n_images, height, width)) * sizeof(float) + 256;
}

int octgs_photometric_loss_grad(const float *img, const float *target, int64_t n_images,
                                int32_t height, int32_t width, float w_l1, float w_ssim,
                                float *dimg, float *loss, void *ws, size_t ws_bytes,
                                octgs_stream stream) {
  if (n_images < 0 || height < 0 || width < 0) return OCTGS_EINVAL;
  const int64_t n = n_images * (int64_t)height * width;
  if (n == 0) return OCTGS_OK;
  if (!img || !target || !dimg || !loss) return OCTGS_EINVAL;
  if (n_images > 65535 || !(w_l1 >= 0.0f) || !(w_ssim >= 0.0f)) return OCTGS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (w_ssim == 0.0f) {
    const int grid = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 512);
    hipLaunchKernelGGL(k_l1_only, dim3(grid), dim3(kBlock), 0, s, img, target, n,
                       (float)(w_l1 / (double)n), dimg, loss);
    return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
  }
  if (!ws) return OCTGS_EINVAL;
  if (ws_bytes < octgs_photometric_workspace_bytes(n_images, height, width)) return OCTGS_ENOSPC;
  SsimArgs a;
  a.x = img; a.y = target;
  a.m0 = (float *)ws; a.m1 = a.m0 + n; a.m2 = a.m1 + n; a.part = a.m2 + n;
  a.dimg = dimg; a.loss = loss;
  a.H = height; a.W = width;
  a.w_l1 = w_l1; a.w_ssim = w_ssim; a.inv_n = (float)(1.0 / (double)n);
  double gs[kTaps], sum = 0.0;
  for (int q = 0; q < kTaps; ++q) {
    const double d = q - kR;
    gs[q] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += gs[q];
  }
  for (int q = 0; q < kTaps; ++q) a.g[q] = (float)(gs[q] / sum);
  const dim3 grid((width + kSW - 1) / kSW, (height + kSH - 1) / kSH, (unsigned)n_images);
  hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(kBlock), 0, s, a);
  hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(kBlock), 0, s, a.part,
                     2 * ssim_blocks(n_images, height, width), w_ssim, loss);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_volume_loss_grad(const octgs_gaussians *g, float weight, float *d_gauss, float *loss,
                           octgs_stream stream) {
  if (!g || !g->data || !g->count || g->capacity < 0 || !d_gauss || !loss) return OCTGS_EINVAL;
  if (g->capacity == 0) return OCTGS_OK;
  const int grid = (int)std::min<int64_t>((g->capacity + kBlock - 1) / kBlock, 512);
  hipLaunchKernelGGL(k_volume, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, g->data,
                     g->capacity, g->count, weight, d_gauss, loss);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

}  // extern "C"
