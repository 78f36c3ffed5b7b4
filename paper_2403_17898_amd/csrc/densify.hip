// Densification statistics and decisions of the adaptive anchor control
// (Sec. IV-B, "Anchor Growing" and "Anchor Pruning").
//
// Accumulation runs once per training view, after octgs_rasterize_bwd: the
// backward leaves dL/d(projected centre) per slot (pixel units) and the
// visibility bit of every slot in the rasterizer workspace.  Each slot of a
// listed anchor maps to its global Gaussian id (anchor * k + i); within one
// view each id occurs once, so the sums are plain read-modify-writes in view
// order (no atomics, the same values on every run).
//
// The decisions every T iterations are taken in FP32 in a fixed order, with
// the per-level thresholds tau_g 2^(beta L) rounded once from double on the
// host:
//   grad_g = sum / count (0 if never visible)
//   grow at L if grad_g > tau_L; at L + 1 if also grad_g > tau_(L+1), L + 1 < K
//   grad_v = (sum of grad_g over visible Gaussians in index order) / their number
//   Delta L += epsilon if grad_v > tau_L / 4
//   prune if count_views / n_views < tau_v, or selected and
//         opacity_sum / (k count_views) < tau_opacity.
#include "octgs_internal.h"

namespace octgs {

namespace {

constexpr int kMaxLevels = 64;

struct AccArgs {
  const float *g;           // decoded Gaussians, planar [14][cap]
  int64_t cap;
  const uint32_t *n_slots;  // rasterizer header word 0: slots it read
  const uint64_t *vis;      // visibility bits per slot
  const float *dproj;       // [cap][9] d(mx, my, ...) per slot
  const uint32_t *idx, *count;
  int k, cap_anchors;
  float half_w, half_h;
  float *grad_sum, *opacity_sum;
  uint32_t *grad_count, *view_count;
};

__global__ __launch_bounds__(kBlock) void k_densify_accumulate(AccArgs a) {
  const uint32_t m = min(*a.count, (uint32_t)a.cap_anchors);
  const int64_t n = min((int64_t)*a.n_slots, (int64_t)m * a.k);
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * kBlock) {
    const uint32_t p = (uint32_t)(s / a.k);
    const int i = (int)(s - (int64_t)p * a.k);
    const uint32_t j = a.idx[p];
    const int64_t gid = (int64_t)j * a.k + i;
    if ((a.vis[s >> 6] >> (s & 63)) & 1ull) {
      const float gx = a.dproj[9 * s] * a.half_w, gy = a.dproj[9 * s + 1] * a.half_h;
      a.grad_sum[gid] += sqrtf(__builtin_fmaf(gx, gx, gy * gy));
      a.grad_count[gid] += 1u;
    }
    if (i == 0) {
      float o = 0.0f;
      for (int q = 0; q < a.k; ++q) o += fmaxf(a.g[10 * a.cap + s + q], 0.0f);
      a.opacity_sum[j] += o;
      a.view_count[j] += 1u;
    }
  }
}

struct DecArgs {
  int64_t n;
  int k, n_levels, n_views;
  float thr[kMaxLevels + 1];
  float epsilon, tau_opacity, tau_v;
  const uint8_t *level;
  const float *grad_sum, *opacity_sum;
  const uint32_t *grad_count, *view_count;
  float *lod_bias;
  int8_t *grow;
  uint8_t *prune;
  uint32_t *counts;  // grow, promote, bias updates, prune
};

__global__ void k_zero4(uint32_t *c) {
  if (threadIdx.x < 4) c[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_densify_decide(DecArgs a) {
  __shared__ uint32_t red[4][kBlock / kWave];
  uint32_t c_grow = 0, c_prom = 0, c_bias = 0, c_prune = 0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < a.n;
       j += (int64_t)gridDim.x * kBlock) {
    const int L = a.level[j];
    const float tl = a.thr[L], tn = a.thr[min(L + 1, a.n_levels)];
    const bool can_promote = L + 1 < a.n_levels;
    float sv = 0.0f;
    uint32_t nv = 0;
    for (int i = 0; i < a.k; ++i) {
      const int64_t g = j * a.k + i;
      const uint32_t c = a.grad_count[g];
      const float grad = c > 0u ? a.grad_sum[g] / (float)c : 0.0f;
      int8_t out = -1;
      if (grad > tl) {
        const bool up = can_promote && grad > tn;
        out = (int8_t)(up ? L + 1 : L);
        ++c_grow;
        c_prom += up ? 1u : 0u;
      }
      a.grow[g] = out;
      if (c > 0u) {
        sv += grad;
        ++nv;
      }
    }
    const float gv = nv > 0u ? sv / (float)nv : 0.0f;
    if (gv > tl * 0.25f) {
      a.lod_bias[j] = a.lod_bias[j] + a.epsilon;
      ++c_bias;
    }
    const uint32_t vc = a.view_count[j];
    const float freq = (float)vc / (float)a.n_views;
    const bool low_op = vc > 0u && a.opacity_sum[j] / ((float)a.k * (float)vc) < a.tau_opacity;
    const bool pr = freq < a.tau_v || low_op;
    a.prune[j] = pr ? 1 : 0;
    c_prune += pr ? 1u : 0u;
  }
  const int w = threadIdx.x / kWave;
  c_grow = wave_sum(c_grow); c_prom = wave_sum(c_prom);
  c_bias = wave_sum(c_bias); c_prune = wave_sum(c_prune);
  if (__lane_id() == 0) {
    red[0][w] = c_grow; red[1][w] = c_prom; red[2][w] = c_bias; red[3][w] = c_prune;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    uint32_t s = 0;
    for (int i = 0; i < kBlock / kWave; ++i) s += red[threadIdx.x][i];
    if (s) atomicAdd(a.counts + threadIdx.x, s);
  }
}

}  // namespace

}  // namespace octgs

using namespace octgs;

extern "C" {

int octgs_densify_accumulate(const octgs_gaussians *g, const octgs_camera *cam,
                             int64_t pair_capacity, const void *raster_ws, size_t ws_bytes,
                             const uint32_t *idx, const uint32_t *count, int32_t k,
                             const octgs_densify_stats *st, octgs_stream stream) {
  if (!g || !cam || !raster_ws || !idx || !count || !st) return OCTGS_EINVAL;
  if (!g->data || !g->count || g->capacity < 0 || g->capacity >= (int64_t(1) << 31))
    return OCTGS_EINVAL;
  if (k < 1 || k > kMaxK) return OCTGS_EUNSUPPORTED;
  if (pair_capacity < 0 || pair_capacity >= (int64_t(1) << 30)) return OCTGS_EINVAL;
  if (cam->width <= 0 || cam->height <= 0) return OCTGS_EINVAL;
  if (!st->grad_sum || !st->grad_count || !st->opacity_sum || !st->view_count)
    return OCTGS_EINVAL;
  if (ws_bytes < octgs_raster_workspace_bytes(g->capacity, pair_capacity, cam->width, cam->height))
    return OCTGS_ENOSPC;
  if (g->capacity == 0) return OCTGS_OK;
  RasterWs ws = raster_layout(const_cast<void *>(raster_ws), g->capacity, pair_capacity,
                              cam->width, cam->height);
  AccArgs a;
  a.g = g->data; a.cap = g->capacity;
  a.n_slots = &ws.hdr->n_slots;
  a.vis = ws.vis_mask; a.dproj = ws.dproj;
  a.idx = idx; a.count = count;
  a.k = k; a.cap_anchors = (int)(g->capacity / k);
  a.half_w = 0.5f * (float)cam->width; a.half_h = 0.5f * (float)cam->height;
  a.grad_sum = st->grad_sum; a.grad_count = st->grad_count;
  a.opacity_sum = st->opacity_sum; a.view_count = st->view_count;
  const int grid = (int)std::min<int64_t>((g->capacity + kBlock - 1) / kBlock, 2048);
  hipLaunchKernelGGL(k_densify_accumulate, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_densify_decide(const octgs_anchors *an, const octgs_densify_stats *st,
                         const octgs_densify_params *p, float *lod_bias, int8_t *grow_level,
                         uint8_t *prune, uint32_t *counts, octgs_stream stream) {
  if (!an || !st || !p || !counts) return OCTGS_EINVAL;
  if (an->n < 0 || an->n >= (int64_t(1) << 31)) return OCTGS_EINVAL;
  if (an->k < 1 || an->k > kMaxK) return OCTGS_EUNSUPPORTED;
  if (an->n_levels < 1 || an->n_levels > kMaxLevels || p->n_views < 1) return OCTGS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero4, dim3(1), dim3(64), 0, s, counts);
  if (an->n == 0) return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
  if (!an->level || !lod_bias || !grow_level || !prune || !st->grad_sum || !st->grad_count ||
      !st->opacity_sum || !st->view_count)
    return OCTGS_EINVAL;
  DecArgs a;
  a.n = an->n; a.k = an->k; a.n_levels = an->n_levels; a.n_views = p->n_views;
  for (int L = 0; L <= kMaxLevels; ++L)
    a.thr[L] = L <= an->n_levels
                   ? (float)((double)p->tau_g * std::exp2((double)p->beta * (double)L))
                   : 0.0f;
  a.epsilon = p->epsilon; a.tau_opacity = p->tau_opacity; a.tau_v = p->tau_v;
  a.level = an->level;
  a.grad_sum = st->grad_sum; a.grad_count = st->grad_count;
  a.opacity_sum = st->opacity_sum; a.view_count = st->view_count;
  a.lod_bias = lod_bias; a.grow = grow_level; a.prune = prune; a.counts = counts;
  const int grid = (int)std::min<int64_t>((an->n + kBlock - 1) / kBlock, 1024);
  hipLaunchKernelGGL(k_densify_decide, dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

}  // extern "C"
