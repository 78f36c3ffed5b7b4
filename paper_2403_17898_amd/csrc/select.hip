// Anchor selection (Octree-GS Sec. IV-A, "Anchor Selection", Eq. 7) and its
// per-scene preparation.
//
// Eq. 7 picks, per view, every anchor whose level L satisfies
// L <= floor(clamp(log2(d_max / (d s)) + Delta L, 0, K - 1)).  For an integer
// level in [0, K-1] that is: level 0 always, otherwise d^2 s^2 <= thr2 with
// thr2 = (d_max 2^(Delta L - L))^2, a per-anchor constant computed once per
// scene.  The per-view test is then one squared distance and one compare,
// with no transcendental, so the scan over all anchors is a pure HBM stream.
//
// Decisions are taken in FP32 with an explicit operation order (explicit
// fmaf, no contraction - the library is built with -ffp-contract=off):
//   d = p - C;  dd = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));  lod = dd * s2 <= thr2
//   (xc, yc, zc) rows fmaf(R0, d0, fmaf(R1, d1, R2 * d2))
//   visibility, conservative for a render with the given raster parameters
//   (a sphere is culled only if none of the Gaussians inside it can reach a
//   pixel centre of the image under the dilated EWA projection):
//   pad = 3 sqrtf(dilation); side-plane slopes tl = (cx + pad) / fx,
//   tr = ((W - cx) + pad) / fx, tt = (cy + pad) / fy, tb = ((H - cy) + pad) / fy;
//   the projection's Jacobian clamp lx = jac_clamp ((0.5 W) / fx), ly alike;
//   per side m = sqrtf(fmaf(t, t, 1)) + fabsf(l - t) (plane-normal length plus
//   the largest slope change of the clamped Jacobian across the Gaussian);
//   visible = zc + rho >= z_near and, per side, +-x (or +-y) <= fmaf(t, zc, rho * m)
#include "octgs_internal.h"

#include <mutex>

namespace octgs {

namespace {

// Thresholds and bound radii, one thread per anchor.  The offset rows (3k
// floats per anchor) are staged through LDS: the block's rows are one
// contiguous span, read with coalesced loads, then each thread reduces its
// own row.
__global__ __launch_bounds__(kBlock) void k_prepare(int64_t n, int k, float d_max,
                                                    const uint8_t *__restrict__ level,
                                                    const float *__restrict__ bias,
                                                    const float *__restrict__ offsets,
                                                    const float *__restrict__ oscale,
                                                    const float *__restrict__ bscale,
                                                    float *__restrict__ thr2,
                                                    float *__restrict__ rho) {
  __shared__ alignas(16) float rows[kBlock * 3 * kMaxK];
  const int rl = 3 * k;
  const int64_t j0 = (int64_t)blockIdx.x * kBlock;
  const int na = (int)min<int64_t>(kBlock, n - j0);
  const float *src = offsets + (size_t)j0 * rl;
  const int nf = na * rl;
  // the span starts 1024 rl bytes into the array, so it is 16-byte aligned
  // whenever the array is; all loads are issued before the first store
  const int nv = (((uintptr_t)offsets & 15) == 0) ? nf >> 2 : 0;
  constexpr int kV = 3 * kMaxK / 4;  // float4s per thread at most (12)
  float4 v[kV];
#pragma unroll
  for (int u = 0; u < kV; ++u) {
    const int i = threadIdx.x + u * kBlock;
    v[u] = i < nv ? ((const float4 *)src)[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
#pragma unroll
  for (int u = 0; u < kV; ++u) {
    const int i = threadIdx.x + u * kBlock;
    if (i < nv) ((float4 *)rows)[i] = v[u];
  }
  for (int e = 4 * nv + threadIdx.x; e < nf; e += kBlock) rows[e] = src[e];
  __syncthreads();
  const int64_t j = j0 + threadIdx.x;
  if (j >= n) return;
  const int L = level[j];
  if (L == 0) {
    thr2[j] = __builtin_inff();
  } else {
    double t = (double)d_max * exp2((double)bias[j] - (double)L);
    thr2[j] = (float)(t * t);
  }
  const float l0 = oscale[3 * j], l1 = oscale[3 * j + 1], l2 = oscale[3 * j + 2];
  float m = 0.0f;
  const float *o = rows + threadIdx.x * rl;
  for (int i = 0; i < k; ++i) {
    float a = o[3 * i] * l0, b = o[3 * i + 1] * l1, c = o[3 * i + 2] * l2;
    float nn = sqrtf(__builtin_fmaf(a, a, __builtin_fmaf(b, b, c * c)));
    m = fmaxf(m, nn);
  }
  const float bmax = fmaxf(fmaxf(bscale[3 * j], bscale[3 * j + 1]), bscale[3 * j + 2]);
  rho[j] = __builtin_fmaf(3.0f, bmax, m);
}

// BF16 copy of an FP32 array, four elements per thread (8-byte stores).
__global__ __launch_bounds__(kBlock) void k_round_bf16(const float *__restrict__ src,
                                                       uint16_t *__restrict__ dst, int64_t count) {
  const int64_t i = 4 * ((int64_t)blockIdx.x * kBlock + threadIdx.x);
  if (i + 4 <= count && ((((uintptr_t)src) | ((uintptr_t)dst)) & 15) == 0) {
    const float4 v = *(const float4 *)(src + i);
    ushort4 o;
    o.x = f2bf(v.x); o.y = f2bf(v.y); o.z = f2bf(v.z); o.w = f2bf(v.w);
    *(ushort4 *)(dst + i) = o;
  } else {
    for (int64_t j = i; j < min(i + 4, count); ++j) dst[j] = f2bf(src[j]);
  }
}

struct Frustum {
  float tl, tr, tt, tb, ml, mr, mt, mb;
};

__device__ __forceinline__ Frustum frustum(const octgs_camera &c, float dilation, float jac_clamp) {
  Frustum f;
  const float pad = 3.0f * sqrtf(dilation);
  f.tl = (c.cx + pad) / c.fx;
  f.tr = (((float)c.width - c.cx) + pad) / c.fx;
  f.tt = (c.cy + pad) / c.fy;
  f.tb = (((float)c.height - c.cy) + pad) / c.fy;
  const float lx = jac_clamp * ((0.5f * (float)c.width) / c.fx);
  const float ly = jac_clamp * ((0.5f * (float)c.height) / c.fy);
  f.ml = sqrtf(__builtin_fmaf(f.tl, f.tl, 1.0f)) + fabsf(lx - f.tl);
  f.mr = sqrtf(__builtin_fmaf(f.tr, f.tr, 1.0f)) + fabsf(lx - f.tr);
  f.mt = sqrtf(__builtin_fmaf(f.tt, f.tt, 1.0f)) + fabsf(ly - f.tt);
  f.mb = sqrtf(__builtin_fmaf(f.tb, f.tb, 1.0f)) + fabsf(ly - f.tb);
  return f;
}

__device__ __forceinline__ bool anchor_selected(const octgs_camera &c, const Frustum &f, float px,
                                                float py, float pz, float thr2, float rho) {
  const float d0 = px - c.C[0], d1 = py - c.C[1], d2 = pz - c.C[2];
  const float dd = __builtin_fmaf(d0, d0, __builtin_fmaf(d1, d1, d2 * d2));
  if (!(dd * c.lod_scale2 <= thr2)) return false;
  const float xc = __builtin_fmaf(c.R[0], d0, __builtin_fmaf(c.R[1], d1, c.R[2] * d2));
  const float yc = __builtin_fmaf(c.R[3], d0, __builtin_fmaf(c.R[4], d1, c.R[5] * d2));
  const float zc = __builtin_fmaf(c.R[6], d0, __builtin_fmaf(c.R[7], d1, c.R[8] * d2));
  if (!(zc + rho >= c.z_near)) return false;
  if (!(xc <= __builtin_fmaf(f.tr, zc, rho * f.mr))) return false;
  if (!(-xc <= __builtin_fmaf(f.tl, zc, rho * f.ml))) return false;
  if (!(yc <= __builtin_fmaf(f.tb, zc, rho * f.mb))) return false;
  if (!(-yc <= __builtin_fmaf(f.tt, zc, rho * f.mt))) return false;
  return true;
}

// Pass 1: block b tests anchors [b*1024, (b+1)*1024) with coalesced loads,
// stores one 64-bit ballot per 64 consecutive anchors and the block count.
__global__ __launch_bounds__(kBlock) void k_select_mark(int64_t n, octgs_camera cam,
                                                        float dilation, float jac_clamp,
                                                        const float *__restrict__ pos,
                                                        const float *__restrict__ thr2,
                                                        const float *__restrict__ rho,
                                                        uint64_t *__restrict__ masks,
                                                        uint32_t *__restrict__ blk_cnt) {
  __shared__ uint32_t wsum[4];
  const Frustum f = frustum(cam, dilation, jac_clamp);
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  uint32_t cnt = 0;
  // the four anchors' inputs are loaded up front (clamped index, n >= 1),
  // so all the loads are in flight together
  float in[kChunkPerThread][5];
#pragma unroll
  for (int i = 0; i < kChunkPerThread; ++i) {
    const int64_t j = min(base + i * kBlock + t, n - 1);
    in[i][0] = pos[3 * j]; in[i][1] = pos[3 * j + 1]; in[i][2] = pos[3 * j + 2];
    in[i][3] = thr2[j]; in[i][4] = rho[j];
  }
  if (cam.lod_blend) {
    // transition blending also takes level L_hat + 1 (L <= L* + 1): the
    // threshold of level L - 1, which is 4 thr2 (exact)
#pragma unroll
    for (int i = 0; i < kChunkPerThread; ++i) in[i][3] = 4.0f * in[i][3];
  }
#pragma unroll
  for (int i = 0; i < kChunkPerThread; ++i) {
    const int64_t j = base + i * kBlock + t;
    const bool sel = j < n && anchor_selected(cam, f, in[i][0], in[i][1], in[i][2], in[i][3], in[i][4]);
    const uint64_t m = ballot(sel);
    if (l == 0 && base + i * kBlock + w * kWave < n) masks[(base + i * kBlock + w * kWave) >> 6] = m;
    cnt += (uint32_t)__popcll(m);
  }
  if (l == 0) wsum[w] = cnt;
  __syncthreads();
  if (t == 0) blk_cnt[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Pass 2: block b adds up the counts of blocks < b, scans its 16 ballots and
// writes the selected indices in ascending order.
__global__ __launch_bounds__(kBlock) void k_select_scatter(int64_t n,
                                                           const uint64_t *__restrict__ masks,
                                                           const uint32_t *__restrict__ blk_cnt,
                                                           uint32_t *__restrict__ sel_idx,
                                                           uint32_t *__restrict__ sel_count) {
  __shared__ uint32_t red[4];
  __shared__ uint32_t gpre[64];
  __shared__ uint64_t gmask[64];
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const int b = blockIdx.x;
  uint32_t s = 0;
  s = partial_sum_prefix(blk_cnt, b);
  s = wave_sum(s);
  if (l == 0) red[w] = s;
  const int64_t base = (int64_t)b * kChunk;
  const int ngroups = (int)min<int64_t>(kGroups, (n - base + 63) / 64);
  if (w == 0) {
    uint64_t m = l < ngroups ? masks[(base >> 6) + l] : 0ull;
    uint32_t c = (uint32_t)__popcll(m);
    uint32_t inc = wave_incl_scan(c);
    gpre[l] = inc - c;
    gmask[l] = m;
  }
  __syncthreads();
  const uint32_t prefix = red[0] + red[1] + red[2] + red[3];
  // group g covers anchors base + 64 g + lane; the four waves take groups round-robin
  for (int g = w; g < ngroups; g += 4) {
    const uint64_t m = gmask[g];
    if ((m >> l) & 1ull) {
      const uint32_t pos = prefix + gpre[g] + (uint32_t)__popcll(m & lanemask_lt());
      sel_idx[pos] = (uint32_t)(base + 64 * g + l);
    }
  }
  if (b == (int)gridDim.x - 1 && t == 0) {
    const uint64_t last = gmask[ngroups - 1];
    *sel_count = prefix + gpre[ngroups - 1] + (uint32_t)__popcll(last);
  }
}

__global__ void k_zero_u32(uint32_t *p) { *p = 0u; }

// Workspace of the two selection passes for n anchors: one 64-bit ballot per
// 64 anchors, then one count per 1024-anchor block (256-byte aligned).
constexpr size_t select_ws_bytes(int64_t n) {
  return (size_t)(((n + kChunk - 1) / kChunk) * (kChunk / 64) * 8 +
                  ((((n + kChunk - 1) / kChunk) * 4 + 255) / 256) * 256 + 256);
}

// Selection without a workspace argument: its ballots and block counts live
// in this file-scope array, sized for at most kScratchMaxAnchors anchors.
// Each GPU the library runs on holds its own copy until the process ends.
constexpr int64_t kScratchMaxAnchors = OCTGS_SELECT_NOALLOC_MAX_ANCHORS;
static_assert(kScratchMaxAnchors < (int64_t(1) << 31), "anchor indices are 32-bit");
constexpr size_t kScratchBytes = select_ws_bytes(kScratchMaxAnchors);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device ordinal, looked up once per device
// with that device current (the host-side name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_address(hipStream_t s, void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return OCTGS_EHIP;
  if (s) {
    int sdev = -1;
    if (hipStreamGetDevice(s, &sdev) != hipSuccess) return OCTGS_EHIP;
    if (sdev != dev) return OCTGS_EINVAL;  // the stream must be on the current device
  }
  if (dev < 0 || dev >= kMaxDevices) return OCTGS_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OCTGS_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return OCTGS_OK;
}

// The two selection passes with the workspace at `ws` (>= select_ws_bytes(n)).
int launch_select(const octgs_anchors *a, const octgs_camera *cam, const octgs_raster_params *p,
                  uint32_t *sel_idx, uint32_t *sel_count, void *ws, hipStream_t s) {
  const int64_t nblk = (a->n + kChunk - 1) / kChunk;
  uint64_t *masks = (uint64_t *)ws;
  uint32_t *blk = (uint32_t *)((char *)ws + nblk * (kChunk / 64) * 8);
  hipLaunchKernelGGL(k_select_mark, dim3((unsigned)nblk), dim3(kBlock), 0, s, a->n, *cam,
                     p->dilation, p->jac_clamp, a->pos, a->thr2, a->bound_r, masks, blk);
  hipLaunchKernelGGL(k_select_scatter, dim3((unsigned)nblk), dim3(kBlock), 0, s, a->n, masks,
                     blk, sel_idx, sel_count);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

// Host-side checks shared by both selection entry points.
int check_select_args(const octgs_anchors *a, const octgs_camera *cam, const octgs_raster_params *p,
                      const uint32_t *sel_idx, const uint32_t *sel_count) {
  if (!a || !cam || !p || !sel_idx || !sel_count) return OCTGS_EINVAL;
  if (a->n < 0 || a->n >= (int64_t(1) << 31)) return OCTGS_EINVAL;
  if (cam->width <= 0 || cam->height <= 0 || !(cam->fx > 0.0f) || !(cam->fy > 0.0f))
    return OCTGS_EINVAL;
  // z_near > 0 keeps every listed depth positive (the depth keys are float bits)
  if (!(cam->z_near > 0.0f)) return OCTGS_EINVAL;
  if (!(p->dilation >= 0.0f) || !(p->jac_clamp > 0.0f)) return OCTGS_EINVAL;
  if (a->n > 0 && (!a->pos || !a->thr2 || !a->bound_r)) return OCTGS_EINVAL;
  return OCTGS_OK;
}

}  // namespace

hipError_t launch_round_bf16(const float *src, uint16_t *dst, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t threads = (count + 3) / 4;
  hipLaunchKernelGGL(k_round_bf16, dim3((unsigned)((threads + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, src, dst, count);
  return hipGetLastError();
}

}  // namespace octgs

using namespace octgs;

extern "C" {

int octgs_prepare_anchors(const octgs_anchors *a, float *thr2, float *bound_r,
                          uint16_t *feat_bf16, octgs_stream stream) {
  if (!a) return OCTGS_EINVAL;
  if (a->n < 0 || a->n >= (int64_t(1) << 31)) return OCTGS_EINVAL;
  if (a->k < 1 || a->k > kMaxK) return OCTGS_EUNSUPPORTED;
  if (a->n == 0) return OCTGS_OK;
  if (!thr2 || !bound_r) return OCTGS_EINVAL;
  if (!a->level || !a->lod_bias || !a->offsets || !a->offset_scale || !a->base_scale)
    return OCTGS_EINVAL;
  if (!(a->d_max > 0.0f)) return OCTGS_EINVAL;
  if (feat_bf16 && (!a->feat || a->feat_dim < 1)) return OCTGS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int grid = (int)((a->n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_prepare, dim3(grid), dim3(kBlock), 0, s, a->n, a->k,
                     a->d_max, a->level, a->lod_bias, a->offsets, a->offset_scale,
                     a->base_scale, thr2, bound_r);
  if (feat_bf16 && launch_round_bf16(a->feat, feat_bf16, a->n * a->feat_dim, s) != hipSuccess)
    return OCTGS_EHIP;
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

size_t octgs_select_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  return select_ws_bytes(n);
}

int octgs_select_lod(const octgs_anchors *a, const octgs_camera *cam, const octgs_raster_params *p,
                     uint32_t *sel_idx, uint32_t *sel_count, void *ws, size_t ws_bytes,
                     octgs_stream stream) {
  const int st = check_select_args(a, cam, p, sel_idx, sel_count);
  if (st != OCTGS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (a->n == 0) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, sel_count);
    return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
  }
  if (!ws) return OCTGS_EINVAL;
  if (ws_bytes < octgs_select_workspace_bytes(a->n)) return OCTGS_ENOSPC;
  return launch_select(a, cam, p, sel_idx, sel_count, ws, s);
}

int octgs_select_lod_noalloc(const octgs_anchors *a, const octgs_camera *cam,
                             const octgs_raster_params *p, uint32_t *sel_idx,
                             uint32_t *sel_count, octgs_stream stream) {
  const int st = check_select_args(a, cam, p, sel_idx, sel_count);
  if (st != OCTGS_OK) return st;
  if (a->n > kScratchMaxAnchors) return OCTGS_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  if (a->n == 0) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, sel_count);
    return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
  }
  void *ws = nullptr;
  const int sa = scratch_address(s, &ws);
  if (sa != OCTGS_OK) return sa;
  // every scratch word the two passes read is written by the first pass of
  // the same call, so nothing needs clearing
  return launch_select(a, cam, p, sel_idx, sel_count, ws, s);
}

}  // extern "C"
