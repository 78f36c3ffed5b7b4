// Explicit 3D Gaussians on the octree anchors: the 3D-GS instance of the
// framework (Sec. V, "Our-3D-GS").  Selection is Eq. 7 unchanged; decode
// becomes a gather of stored attributes, their activations (exp scale,
// normalised rotation, sigmoid opacity) and a view-dependent colour from
// spherical-harmonic coefficients (Sec. III-A), written in the same planar
// Gaussian record the rasterizer reads.
//
// Layout and traffic.  The SH block of a Gaussian ((D+1)^2 x 3 values, 192 B
// in FP32 at degree 3) dominates the bytes.  Each block of 256 threads owns
// consecutive output slots; the slots of one listed anchor are k
// consecutive Gaussians in memory, so the block first copies all its SH rows
// into LDS with consecutive lanes reading consecutive 16-byte words (whole
// cache lines per instruction), then each thread evaluates its own row from
// LDS (row pitch padded to an odd number of 16-byte words: conflict-free).
// Blocks hold 128 slots.
// A thread-per-slot read of 192-byte rows straight from memory would touch
// 64 lines per instruction and re-fetch them from L2 as L1 thrashes.
//
// Real SH basis, degree <= 3, on the unit view direction (x, y, z), index
// l^2 + l + m, Condon-Shortley phase kept (the 3D-GS colour convention):
//   l=0: 1/(2 sqrt(pi))
//   l=1: -C1 y, C1 z, -C1 x                        C1 = sqrt(3/(4 pi))
//   l=2: a xy, -a yz, b (2z^2 - x^2 - y^2), -a xz, c (x^2 - y^2)
//        a = sqrt(15/pi)/2, b = sqrt(5/pi)/4, c = sqrt(15/pi)/4
//   l=3: -d y(3x^2 - y^2), e xyz, -f y(4z^2 - x^2 - y^2),
//        g z(2z^2 - 3x^2 - 3y^2), -f x(4z^2 - x^2 - y^2), h z(x^2 - y^2),
//        -d x(x^2 - 3y^2)
//        d = sqrt(35/(2 pi))/4, e = sqrt(105/pi)/2, f = sqrt(21/(2 pi))/4,
//        g = sqrt(7/pi)/4, h = sqrt(105/pi)/4
// colour = max(0, sum_lm sh_lm Y_lm + 0.5).
#include "octgs_internal.h"

namespace octgs {

namespace {

constexpr float kC0 = 2.820947918e-01f, kC1 = 4.886025119e-01f;
constexpr float kA = 1.092548431e+00f, kB = 3.153915653e-01f, kCc = 5.462742153e-01f;
constexpr float kD = 5.900435899e-01f, kE = 2.890611443e+00f, kF = 4.570457995e-01f;
constexpr float kG = 3.731763326e-01f, kH = 1.445305721e+00f;

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Gaussians (slots) per block and per iteration, one per thread.  128-slot
// blocks keep the LDS of a block at ~27 KB (degree 3, FP32), so five blocks
// are resident per CU and their loads overlap.
constexpr int kExT = 128;

template <int D>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float *Y) {
  Y[0] = kC0;
  if constexpr (D >= 1) {
    Y[1] = -kC1 * y; Y[2] = kC1 * z; Y[3] = -kC1 * x;
  }
  if constexpr (D >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = kA * x * y;
    Y[5] = -kA * y * z;
    Y[6] = kB * (2.0f * zz - xx - yy);
    Y[7] = -kA * x * z;
    Y[8] = kCc * (xx - yy);
    if constexpr (D >= 3) {
      Y[9] = -kD * y * (3.0f * xx - yy);
      Y[10] = kE * x * y * z;
      Y[11] = -kF * y * (4.0f * zz - xx - yy);
      Y[12] = kG * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
      Y[13] = -kF * x * (4.0f * zz - xx - yy);
      Y[14] = kH * z * (xx - yy);
      Y[15] = -kD * x * (xx - 3.0f * yy);
    }
  }
}

// sum_l w_l grad Y_l of the polynomial forms above, as functions of free
// (x, y, z); the caller projects out the radial part.
template <int D>
__device__ __forceinline__ void sh_grad_dot(float x, float y, float z, const float *w, float &gx,
                                            float &gy, float &gz) {
  gx = 0.0f; gy = 0.0f; gz = 0.0f;
  if constexpr (D >= 1) {
    gx = -kC1 * w[3]; gy = -kC1 * w[1]; gz = kC1 * w[2];
  }
  if constexpr (D >= 2) {
    const float xx = x * x, yy = y * y, zz = z * z;
    gx += kA * (y * w[4] - z * w[7]) + 2.0f * x * (kCc * w[8] - kB * w[6]);
    gy += kA * (x * w[4] - z * w[5]) - 2.0f * y * (kB * w[6] + kCc * w[8]);
    gz += 4.0f * kB * z * w[6] - kA * (y * w[5] + x * w[7]);
    if constexpr (D >= 3) {
      gx += -6.0f * kD * x * y * w[9] + kE * y * z * w[10] + 2.0f * kF * x * y * w[11] -
            6.0f * kG * x * z * w[12] - kF * (4.0f * zz - 3.0f * xx - yy) * w[13] +
            2.0f * kH * x * z * w[14] - 3.0f * kD * (xx - yy) * w[15];
      gy += -3.0f * kD * (xx - yy) * w[9] + kE * x * z * w[10] -
            kF * (4.0f * zz - xx - 3.0f * yy) * w[11] - 6.0f * kG * y * z * w[12] +
            2.0f * kF * x * y * w[13] - 2.0f * kH * y * z * w[14] + 6.0f * kD * x * y * w[15];
      gz += kE * x * y * w[10] - 8.0f * kF * y * z * w[11] +
            kG * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12] - 8.0f * kF * x * z * w[13] +
            kH * (xx - yy) * w[14];
    }
  }
}

template <int B> struct UnitT;
template <> struct UnitT<16> { using T = uint4; };
template <> struct UnitT<8> { using T = uint2; };
template <> struct UnitT<4> { using T = uint32_t; };

// Per-slot SH row: NV values of ES bytes, copied in units of UB bytes.
template <int D, bool BF16>
struct ShRow {
  static constexpr int NC = (D + 1) * (D + 1);
  static constexpr int NV = 3 * NC;
  static constexpr int BYTES = NV * (BF16 ? 2 : 4);
  static constexpr int UB = BYTES % 16 == 0 ? 16 : BYTES % 8 == 0 ? 8 : 4;
  static constexpr int CH = BYTES / UB;           // units per row
  static constexpr int PITCH = CH % 2 ? CH : CH + 1;  // odd pitch: conflict-free rows
  static constexpr int WORDS = BYTES / 4;
  using U = typename UnitT<UB>::T;
  static_assert(BYTES % 4 == 0, "SH row must be a whole number of 32-bit words");
};

struct ExArgs {
  int k, cap_anchors, blend, n_levels;
  float C[3];
  float d_max, s;
  const float *pos;
  const uint8_t *level;
  const float *lod_bias;
  const float *mean, *log_scale, *rot, *opac;
  const void *sh;
  const uint32_t *idx, *count;
  float *out;
  int64_t cap;
  uint32_t *out_count;
  uint32_t *status;  // nullable: OCTGS_STATUS_TRUNCATED when the listed anchors exceed the capacity
  // backward
  const float *dg;
  int64_t dstride;
  float *g_mean, *g_ls, *g_rot, *g_op, *g_sh;
};

// Copies the SH rows of the block's slots into LDS.  gidx[t] = global
// Gaussian index of local slot t (valid for t < nsl).  Unit q of the block
// maps to (slot q / CH, word q % CH): consecutive lanes read consecutive
// units of one anchor's contiguous rows.
template <int D, bool BF16>
__device__ __forceinline__ void stage_rows(const void *src, const int64_t *gidx, int nsl,
                                           typename ShRow<D, BF16>::U *rows) {
  using R = ShRow<D, BF16>;
  using U = typename R::U;
  const U *g = (const U *)src;
  const int t = threadIdx.x;
  U v[R::CH];
#pragma unroll
  for (int r = 0; r < R::CH; ++r) {
    const int q = t + r * kExT;
    const int ls = q / R::CH, part = q - ls * R::CH;
    const int lsc = ls < nsl ? ls : 0;
    v[r] = g[gidx[lsc] * R::CH + part];
  }
#pragma unroll
  for (int r = 0; r < R::CH; ++r) {
    const int q = t + r * kExT;
    const int ls = q / R::CH, part = q - ls * R::CH;
    if (ls < nsl) rows[ls * R::PITCH + part] = v[r];
  }
}

template <int D, bool BF16>
__device__ __forceinline__ void load_row(const typename ShRow<D, BF16>::U *rows, int t,
                                         float *c) {
  using R = ShRow<D, BF16>;
  uint32_t w[R::WORDS];
#pragma unroll
  for (int u = 0; u < R::CH; ++u) {
    const typename R::U x = rows[t * R::PITCH + u];
    memcpy(&w[u * (R::UB / 4)], &x, R::UB);
  }
#pragma unroll
  for (int v = 0; v < R::NV; ++v) {
    if constexpr (BF16) c[v] = __uint_as_float((v & 1 ? w[v >> 1] >> 16 : w[v >> 1] & 0xffffu) << 16);
    else c[v] = __uint_as_float(w[v]);
  }
}

template <int D, bool BF16>
struct ExLds {
  typename ShRow<D, BF16>::U rows[kExT * ShRow<D, BF16>::PITCH];
  int64_t gidx[kExT];
};

template <int D, bool BF16>
__global__ __launch_bounds__(kExT) void k_decode_explicit(ExArgs a) {
  using R = ShRow<D, BF16>;
  __shared__ ExLds<D, BF16> sm;
  const int t = threadIdx.x, k = a.k;
  const uint32_t m_total = min(*a.count, (uint32_t)a.cap_anchors);
  const int64_t total = (int64_t)m_total * k;
  if (blockIdx.x == 0 && t == 0) {
    *a.out_count = (uint32_t)total;
    if (a.status && *a.count > (uint32_t)a.cap_anchors) atomicOr(a.status, OCTGS_STATUS_TRUNCATED);
  }
  for (int64_t s0 = (int64_t)blockIdx.x * kExT; s0 < total; s0 += (int64_t)gridDim.x * kExT) {
    const int nsl = (int)min<int64_t>(kExT, total - s0);
    const int64_t s = s0 + min(t, nsl - 1);
    const uint32_t p = (uint32_t)(s / k);
    const int i = (int)(s - (int64_t)p * k);
    const uint32_t j = a.idx[p];
    const int64_t gi = (int64_t)j * k + i;
    sm.gidx[t] = gi;
    // per-slot attributes, issued before the SH copy so both are in flight
    const float mx = a.mean[3 * gi], my = a.mean[3 * gi + 1], mz = a.mean[3 * gi + 2];
    const float l0 = a.log_scale[3 * gi], l1 = a.log_scale[3 * gi + 1], l2 = a.log_scale[3 * gi + 2];
    const float4 q = *(const float4 *)(a.rot + 4 * gi);
    const float lo = a.opac[gi];
    float fac = 1.0f;
    if (a.blend) {
      // fractional level L* = clamp(log2(d_max / (d s)) + Delta L, 0, K - 1)
      const float d0 = a.pos[3 * (size_t)j] - a.C[0];
      const float d1 = a.pos[3 * (size_t)j + 1] - a.C[1];
      const float d2 = a.pos[3 * (size_t)j + 2] - a.C[2];
      const float dist = sqrtf(fma_(d0, d0, fma_(d1, d1, d2 * d2)));
      const float ls = fminf(fmaxf(log2f(a.d_max / (dist * a.s)) + a.lod_bias[j], 0.0f),
                             (float)(a.n_levels - 1));
      fac = fminf(fmaxf(ls - (float)a.level[j] + 1.0f, 0.0f), 1.0f);
    }
    __syncthreads();
    stage_rows<D, BF16>(a.sh, sm.gidx, nsl, sm.rows);
    __syncthreads();
    if (t < nsl) {
      float c[R::NV];
      load_row<D, BF16>(sm.rows, t, c);
      const float vx = mx - a.C[0], vy = my - a.C[1], vz = mz - a.C[2];
      const float inv = 1.0f / sqrtf(fma_(vx, vx, fma_(vy, vy, vz * vz)));
      float Y[R::NC];
      sh_basis<D>(vx * inv, vy * inv, vz * inv, Y);
      float col[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.5f;
#pragma unroll
        for (int l = 0; l < R::NC; ++l) acc = fma_(Y[l], c[3 * l + ch], acc);
        col[ch] = fmaxf(acc, 0.0f);
      }
      const float n2 = fma_(q.x, q.x, fma_(q.y, q.y, fma_(q.z, q.z, q.w * q.w)));
      float nw = 1.0f, nx = 0.0f, ny = 0.0f, nz = 0.0f;
      if (n2 > 0.0f) {
        const float r = 1.0f / sqrtf(n2);
        nw = q.x * r; nx = q.y * r; ny = q.z * r; nz = q.w * r;
      }
      const int64_t cap = a.cap, o = s0 + t;
      float *out = a.out;
      out[o] = mx; out[cap + o] = my; out[2 * cap + o] = mz;
      out[3 * cap + o] = expf(l0); out[4 * cap + o] = expf(l1); out[5 * cap + o] = expf(l2);
      out[6 * cap + o] = nw; out[7 * cap + o] = nx; out[8 * cap + o] = ny; out[9 * cap + o] = nz;
      out[10 * cap + o] = fac / (1.0f + expf(-lo));
      out[11 * cap + o] = col[0]; out[12 * cap + o] = col[1]; out[13 * cap + o] = col[2];
    }
    __syncthreads();
  }
}

// Backward of the explicit decode (FP32 coefficients).  The SH gradient rows
// go back through LDS so the accumulation into the [slot][NV] array is one
// coalesced read-modify-write per 16-byte word.
template <int D>
__global__ __launch_bounds__(kExT) void k_decode_explicit_bwd(ExArgs a) {
  using R = ShRow<D, false>;
  __shared__ ExLds<D, false> sm;
  const int t = threadIdx.x, k = a.k;
  const uint32_t m_total = min(*a.count, (uint32_t)a.cap_anchors);
  const int64_t total = (int64_t)m_total * k;
  for (int64_t s0 = (int64_t)blockIdx.x * kExT; s0 < total; s0 += (int64_t)gridDim.x * kExT) {
    const int nsl = (int)min<int64_t>(kExT, total - s0);
    const int64_t s = s0 + min(t, nsl - 1);
    const uint32_t p = (uint32_t)(s / k);
    const int i = (int)(s - (int64_t)p * k);
    const int64_t gi = (int64_t)a.idx[p] * k + i;
    sm.gidx[t] = gi;
    const float mx = a.mean[3 * gi], my = a.mean[3 * gi + 1], mz = a.mean[3 * gi + 2];
    const float l0 = a.log_scale[3 * gi], l1 = a.log_scale[3 * gi + 1], l2 = a.log_scale[3 * gi + 2];
    const float4 q = *(const float4 *)(a.rot + 4 * gi);
    const float lo = a.opac[gi];
    float dg[kGaussFields];
#pragma unroll
    for (int f = 0; f < kGaussFields; ++f) dg[f] = a.dg[f * a.dstride + s];
    __syncthreads();
    stage_rows<D, false>(a.sh, sm.gidx, nsl, sm.rows);
    __syncthreads();
    if (t < nsl) {
      float c[R::NV];
      load_row<D, false>(sm.rows, t, c);
      const float vx = mx - a.C[0], vy = my - a.C[1], vz = mz - a.C[2];
      const float inv = 1.0f / sqrtf(fma_(vx, vx, fma_(vy, vy, vz * vz)));
      const float x = vx * inv, y = vy * inv, z = vz * inv;
      float Y[R::NC];
      sh_basis<D>(x, y, z, Y);
      float g[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float acc = 0.5f;
#pragma unroll
        for (int l = 0; l < R::NC; ++l) acc = fma_(Y[l], c[3 * l + ch], acc);
        g[ch] = acc > 0.0f ? dg[11 + ch] : 0.0f;
      }
      // dL/dcoefficient = Y_l g_c, written over this thread's own LDS row
      float w[R::NC];
      float *row = (float *)&sm.rows[t * R::PITCH];
#pragma unroll
      for (int l = 0; l < R::NC; ++l) {
        w[l] = fma_(g[0], c[3 * l], fma_(g[1], c[3 * l + 1], g[2] * c[3 * l + 2]));
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) row[3 * l + ch] = Y[l] * g[ch];
      }
      // direction: d = v / |v|, dL/dv = (I - d d^T) dL/dd / |v|
      float gx, gy, gz;
      sh_grad_dot<D>(x, y, z, w, gx, gy, gz);
      const float rad = fma_(x, gx, fma_(y, gy, z * gz));
      float *gm = a.g_mean + 3 * gi;
      gm[0] += dg[0] + (gx - rad * x) * inv;
      gm[1] += dg[1] + (gy - rad * y) * inv;
      gm[2] += dg[2] + (gz - rad * z) * inv;
      float *gl = a.g_ls + 3 * gi;
      gl[0] += dg[3] * expf(l0); gl[1] += dg[4] * expf(l1); gl[2] += dg[5] * expf(l2);
      const float n2 = fma_(q.x, q.x, fma_(q.y, q.y, fma_(q.z, q.z, q.w * q.w)));
      if (n2 > 0.0f) {
        const float r = 1.0f / sqrtf(n2);
        const float qw = q.x * r, qx = q.y * r, qy = q.z * r, qz = q.w * r;
        const float dot = fma_(qw, dg[6], fma_(qx, dg[7], fma_(qy, dg[8], qz * dg[9])));
        float4 *gr = (float4 *)(a.g_rot + 4 * gi);
        float4 o = *gr;
        o.x += (dg[6] - qw * dot) * r; o.y += (dg[7] - qx * dot) * r;
        o.z += (dg[8] - qy * dot) * r; o.w += (dg[9] - qz * dot) * r;
        *gr = o;
      }
      const float sg = 1.0f / (1.0f + expf(-lo));
      a.g_op[gi] += dg[10] * sg * (1.0f - sg);
    }
    __syncthreads();
    // coalesced accumulation of the staged coefficient gradients
    {
      using U = typename R::U;
      U *gsh = (U *)a.g_sh;
#pragma unroll
      for (int r = 0; r < R::CH; ++r) {
        const int qq = t + r * kExT;
        const int ls = qq / R::CH, part = qq - ls * R::CH;
        if (ls < nsl) {
          U *dst = gsh + sm.gidx[ls] * R::CH + part;
          U v = *dst;
          const U d = sm.rows[ls * R::PITCH + part];
          float *fv = (float *)&v;
          const float *fd = (const float *)&d;
#pragma unroll
          for (int e = 0; e < R::UB / 4; ++e) fv[e] += fd[e];
          *dst = v;
        }
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_prepare_explicit(int64_t n, int k, float d_max,
                                                             const uint8_t *__restrict__ level,
                                                             const float *__restrict__ bias,
                                                             const float *__restrict__ pos,
                                                             const float *__restrict__ mean,
                                                             const float *__restrict__ lsc,
                                                             float *__restrict__ thr2,
                                                             float *__restrict__ rho) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  const int L = level[j];
  if (L == 0) {
    thr2[j] = __builtin_inff();
  } else {
    const double tt = (double)d_max * exp2((double)bias[j] - (double)L);
    thr2[j] = (float)(tt * tt);
  }
  const float p0 = pos[3 * j], p1 = pos[3 * j + 1], p2 = pos[3 * j + 2];
  float m = 0.0f, lmax = -__builtin_inff();
  for (int i = 0; i < k; ++i) {
    const int64_t g = j * k + i;
    const float a = mean[3 * g] - p0, b = mean[3 * g + 1] - p1, c = mean[3 * g + 2] - p2;
    m = fmaxf(m, sqrtf(fma_(a, a, fma_(b, b, c * c))));
    lmax = fmaxf(lmax, fmaxf(fmaxf(lsc[3 * g], lsc[3 * g + 1]), lsc[3 * g + 2]));
  }
  const float smax = (float)exp((double)lmax);
  rho[j] = fma_(3.0f, smax, m);
}

__global__ void k_zero_count_ex(uint32_t *p) { *p = 0u; }

template <bool BF16>
void launch_decode(int D, int grid, hipStream_t s, const ExArgs &a) {
  switch (D) {
    case 0: if constexpr (!BF16) hipLaunchKernelGGL((k_decode_explicit<0, false>), dim3(grid), dim3(kExT), 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_decode_explicit<1, BF16>), dim3(grid), dim3(kExT), 0, s, a); break;
    case 2: if constexpr (!BF16) hipLaunchKernelGGL((k_decode_explicit<2, false>), dim3(grid), dim3(kExT), 0, s, a); break;
    default: hipLaunchKernelGGL((k_decode_explicit<3, BF16>), dim3(grid), dim3(kExT), 0, s, a); break;
  }
}

int fill_common(const octgs_anchors *an, const octgs_explicit *e, const octgs_camera *cam,
                const uint32_t *idx, const uint32_t *count, int64_t gauss_capacity, ExArgs &a) {
  if (!an || !e || !cam || !idx || !count) return OCTGS_EINVAL;
  if (an->k < 1 || an->k > kMaxK) return OCTGS_EUNSUPPORTED;
  if (e->sh_degree < 0 || e->sh_degree > 3) return OCTGS_EUNSUPPORTED;
  if (gauss_capacity < 0 || gauss_capacity / an->k > 0x7fffffff) return OCTGS_EINVAL;
  memset(&a, 0, sizeof a);
  a.k = an->k;
  a.cap_anchors = (int)(gauss_capacity / an->k);
  for (int c = 0; c < 3; ++c) a.C[c] = cam->C[c];
  a.pos = an->pos; a.level = an->level; a.lod_bias = an->lod_bias;
  a.n_levels = an->n_levels; a.d_max = an->d_max; a.s = sqrtf(cam->lod_scale2);
  a.mean = e->mean; a.log_scale = e->log_scale; a.rot = e->rot; a.opac = e->opacity;
  a.idx = idx; a.count = count;
  return OCTGS_OK;
}

int grid_for(int64_t gauss_capacity) {
  // 256 slots per block and iteration; LDS holds two FP32 degree-3 blocks
  // per CU, so a few resident rounds over 256 CUs is enough to stream
  return (int)std::max<int64_t>(1, std::min<int64_t>((gauss_capacity + kExT - 1) / kExT, 4096));
}

}  // namespace

}  // namespace octgs

using namespace octgs;

extern "C" {

int octgs_prepare_explicit(const octgs_anchors *a, const octgs_explicit *e, float *thr2,
                           float *bound_r, uint16_t *sh_bf16, octgs_stream stream) {
  if (!a || !e) return OCTGS_EINVAL;
  if (a->n < 0 || a->n >= (int64_t(1) << 31)) return OCTGS_EINVAL;
  if (a->k < 1 || a->k > kMaxK) return OCTGS_EUNSUPPORTED;
  if (a->n == 0) return OCTGS_OK;
  if (!thr2 || !bound_r || !a->level || !a->lod_bias || !a->pos || !e->mean || !e->log_scale)
    return OCTGS_EINVAL;
  if (!(a->d_max > 0.0f)) return OCTGS_EINVAL;
  if (sh_bf16 && (!e->sh || e->sh_degree < 0 || e->sh_degree > 3)) return OCTGS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int grid = (int)((a->n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_prepare_explicit, dim3(grid), dim3(kBlock), 0, s, a->n,
                     a->k, a->d_max, a->level, a->lod_bias, a->pos, e->mean, e->log_scale, thr2,
                     bound_r);
  const int64_t nsh = a->n * a->k * (int64_t)(e->sh_degree + 1) * (e->sh_degree + 1) * 3;
  if (sh_bf16 && launch_round_bf16(e->sh, sh_bf16, nsh, s) != hipSuccess) return OCTGS_EHIP;
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_decode_explicit(const octgs_anchors *an, const octgs_explicit *e,
                          const octgs_camera *cam, const uint32_t *idx, const uint32_t *count,
                          int precision, const octgs_gaussians *out, octgs_stream stream) {
  if (!out || !out->data || !out->count || out->capacity < 0) return OCTGS_EINVAL;
  if (precision != OCTGS_FP32 && precision != OCTGS_BF16) return OCTGS_EINVAL;
  ExArgs a{};
  const int st = fill_common(an, e, cam, idx, count, out->capacity, a);
  if (st != OCTGS_OK) return st;
  const bool bf16 = precision == OCTGS_BF16;
  if (bf16 && e->sh_degree != 1 && e->sh_degree != 3) return OCTGS_EUNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  if (an->n == 0) {
    hipLaunchKernelGGL(k_zero_count_ex, dim3(1), dim3(1), 0, s, out->count);
    return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
  }
  const void *sh = bf16 ? (const void *)e->sh_bf16 : (const void *)e->sh;
  if (!e->mean || !e->log_scale || !e->rot || !e->opacity || !sh) return OCTGS_EINVAL;
  if (((uintptr_t)e->rot | (uintptr_t)sh) & 15) return OCTGS_EINVAL;
  a.blend = cam->lod_blend ? 1 : 0;
  if (a.blend && (!an->pos || !an->level || !an->lod_bias || an->n_levels < 1 ||
                  !(cam->lod_scale2 > 0.0f) || !(an->d_max > 0.0f)))
    return OCTGS_EINVAL;
  a.sh = sh;
  a.out = out->data; a.cap = out->capacity; a.out_count = out->count; a.status = out->status;
  const int grid = grid_for(out->capacity);
  if (bf16) launch_decode<true>(e->sh_degree, grid, s, a);
  else launch_decode<false>(e->sh_degree, grid, s, a);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_decode_explicit_bwd(const octgs_anchors *an, const octgs_explicit *e,
                              const octgs_camera *cam, const uint32_t *idx,
                              const uint32_t *count, const float *d_gauss,
                              int64_t gauss_capacity, const octgs_explicit_grads *g,
                              octgs_stream stream) {
  if (!d_gauss || !g) return OCTGS_EINVAL;
  ExArgs a{};
  const int st = fill_common(an, e, cam, idx, count, gauss_capacity, a);
  if (st != OCTGS_OK) return st;
  if (cam->lod_blend) return OCTGS_EUNSUPPORTED;
  if (an->n == 0 || gauss_capacity < an->k) return OCTGS_OK;
  if (!e->mean || !e->log_scale || !e->rot || !e->opacity || !e->sh) return OCTGS_EINVAL;
  if (!g->mean || !g->log_scale || !g->rot || !g->opacity || !g->sh) return OCTGS_EINVAL;
  if (((uintptr_t)e->rot | (uintptr_t)e->sh | (uintptr_t)g->rot | (uintptr_t)g->sh) & 15)
    return OCTGS_EINVAL;
  a.sh = e->sh;
  a.dg = d_gauss; a.dstride = gauss_capacity;
  a.g_mean = g->mean; a.g_ls = g->log_scale; a.g_rot = g->rot; a.g_op = g->opacity;
  a.g_sh = g->sh;
  const int grid = grid_for(gauss_capacity);
  hipStream_t s = (hipStream_t)stream;
  switch (e->sh_degree) {
    case 0: hipLaunchKernelGGL(k_decode_explicit_bwd<0>, dim3(grid), dim3(kExT), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_decode_explicit_bwd<1>, dim3(grid), dim3(kExT), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_decode_explicit_bwd<2>, dim3(grid), dim3(kExT), 0, s, a); break;
    default: hipLaunchKernelGGL(k_decode_explicit_bwd<3>, dim3(grid), dim3(kExT), 0, s, a); break;
  }
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

}  // extern "C"
