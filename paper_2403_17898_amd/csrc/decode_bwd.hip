// Backward pass of the neural-Gaussian decode (Octree-GS Sec. III-B, Eq. 3
// and Eq. 4): from the gradients of the decoded Gaussian attributes to the
// gradients of the anchor features, positions, offsets, scalings and of the
// three MLP heads' weights and biases.  FP32 throughout.
//
// One fused kernel.  A persistent block of two wave groups (4 waves each)
// stages every weight in LDS once, then walks pairs of tiles of 16 listed
// anchors, one tile per group, the groups in step at the block's barriers so
// that each hides the other's memory and LDS latency; per tile, every
// product runs on v_mfma_f32_16x16x4_f32 out of LDS:
//   Hp = X W1 + b1            forward recompute (per head: 36 -> W)
//   Y  = relu(Hp) W2 + b2     forward recompute (per head: W -> k, 3k, 7k)
//   dY                        activation derivatives; one 16-lane row per
//                             anchor, lane i for Gaussian i, which also sums
//                             the anchor-array gradients (Eq. 3) in the row
//   dHp = (dY W2^T) * [Hp > 0]
//   dX = dHp W1^T             -> feature and position gradients
//   dW2 += relu(Hp)^T dY, dW1 += X^T dHp, db += column sums
// The weight-gradient sums stay in MFMA accumulators across all of the
// block's tiles; the second group hands its sums to the first through LDS
// (added in group order), and each block writes them once to its row of a
// workspace.  Each listed anchor's gradients go to its own row of the
// workspace too.  A second pair of kernels (the apply half, which the caller
// may order after other views' rows) adds the anchor rows into the anchor
// arrays and the block rows, in block order, into the weight gradients: no
// atomics, the same result on every run.  The anchor count lives on the
// device.
//
// MFMA 16x16x4 operand layouts (lane l, group g = l / 16, c = l % 16):
//   A[m][k]: row m = c, k = g;  B[k][n]: column n = c, k = g;
//   D[m][n]: column n = c, rows m = 4 g + i, i = 0..3.
#include "octgs_internal.h"

namespace octgs {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + __expf(-x)); }
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int kRB = 16;                // anchors per tile
constexpr int kIn = 36;                // feature (32) + distance + direction (3)
constexpr int kInP = 48;               // inputs padded to three column tiles
constexpr int kMaxW = 64;
constexpr int kMaxOutP = 176;          // padded head outputs: 16 + 48 + 112 at k = 16
constexpr int kXS = kInP + 4;          // LDS row pitches (floats)
constexpr int kHS = 3 * kMaxW + 4;
constexpr int kYS = kMaxOutP + 4;
constexpr int kW1P = kMaxW + 4;        // W1 row pitch: conflict-free column reads for dX
constexpr int kMaxT1 = 9;              // dW1 output tiles per wave (3 x 12 / 4)
constexpr int kMaxT2 = 11;             // dW2 output tiles per wave (4 x 11 / 4)
constexpr int kDecBwdGrid = 256;       // persistent blocks (one per CU: ~159 KB of LDS each)
constexpr int kDecGroups = 2;          // wave groups per block, one tile each
// A listed anchor's gradient row: position, feature, k offsets, offset
// scale, base scale (41 + 3k floats).
constexpr int kRowPos = 0, kRowFeat = 3, kRowOff = 35;
__host__ __device__ inline int row_osc(int k) { return kRowOff + 3 * k; }
__host__ __device__ inline int row_bsc(int k) { return kRowOff + 3 * k + 3; }
__host__ __device__ inline int row_len(int k) { return kRowOff + 3 * k + 6; }
constexpr int kDecBwdThreads = kDecGroups * kBlock;

struct DecBwdArgs {
  int k, W, cap_anchors;
  int t[3];        // output column tiles per head
  int outs[3];     // head widths k, 3k, 7k
  int offp[3];     // head offsets in the padded output row (16 t[0], 16 (t[0] + t[1]))
  int wo[3];       // offsets of the W2 heads in the staged block (0, W k, 4 W k)
  int P;           // partial vector length
  int p_w2, p_b1, p_b2;  // its regions: dW1 heads at 0, then dW2, db1, db2
  float inv_dmax;
  float C[3];
  const float *pos, *feat, *offsets, *oscale, *bscale;
  const float *w1[3], *b1[3], *w2[3], *b2[3];
  const uint32_t *idx, *count;
  const float *dgauss;
  int64_t dstride;
  float *rows;     // [cap_anchors][rstride]: each listed anchor's gradient row (kRow* layout)
  int rstride;
  float *part;     // [gridDim.x][P]
};

// one group's tile buffers
struct DecBwdTile {
  float X[kRB][kXS];
  float Hp[kRB][kHS];
  float Yd[kRB][kYS];            // Y, overwritten in place by dY
  float dH[kRB][kHS];
  float dX[kRB][kInP];
  float Dn[kRB][4];              // distance and unit direction per anchor
  float dp[kRB][3];              // position gradient through the decoded means
  uint32_t aidx[kRB];
};

// the second group's weight-gradient sums, handed to the first at the end
// (in the tile buffers, which are free by then): per lane kMaxT1 + kMaxT2
// accumulator tiles of 4 floats and the two bias sums
constexpr int kXchSlots = 4 * (kMaxT1 + kMaxT2) + 2;

struct DecBwdLds {
  float W1s[3 * kIn * kW1P];     // W1 heads, rows of kW1P
  float W2s[kMaxW * 11 * kMaxK]; // W2 heads [W][k], [W][3k], [W][7k], packed
  float b1s[3 * kMaxW];
  float b2s[kMaxOutP];           // padded output layout
  DecBwdTile tl[kDecGroups];
};
static_assert(sizeof(DecBwdTile) * kDecGroups >= sizeof(float) * kXchSlots * kBlock,
              "the hand-over of the second group's sums fits in the tile buffers");
static_assert(sizeof(DecBwdLds) <= 160 * 1024, "LDS of one CU");

__device__ __forceinline__ const float *pick3(const float *const p[3], int h) {
  return h == 0 ? p[0] : (h == 1 ? p[1] : p[2]);
}
__device__ __forceinline__ float *pick3(float *const p[3], int h) {
  return h == 0 ? p[0] : (h == 1 ? p[1] : p[2]);
}

// one of three kernel-argument values by a lane-varying index, without
// indexing the argument array through scratch memory
__device__ __forceinline__ int sel3(const int (&v)[3], int h) {
  return h == 0 ? v[0] : (h == 1 ? v[1] : v[2]);
}

// padded output tile c -> head and the tile's first column within the head
__device__ __forceinline__ int out_head(const DecBwdArgs &a, int c, int &col0) {
  if (c < a.t[0]) { col0 = c * 16; return 0; }
  if (c < a.t[0] + a.t[1]) { col0 = (c - a.t[0]) * 16; return 1; }
  col0 = (c - a.t[0] - a.t[1]) * 16;
  return 2;
}

// Sum over the 16 lanes of a DPP row (every lane of the row gets it).
__device__ __forceinline__ float row16_sum(float v) {
  v += __uint_as_float(dpp_u<kDppXor1>(__float_as_uint(v)));
  v += __uint_as_float(dpp_u<kDppXor2>(__float_as_uint(v)));
  v += __uint_as_float(dpp_u<kDppHalfMirror>(__float_as_uint(v)));
  v += __uint_as_float(dpp_u<kDppRor8>(__float_as_uint(v)));
  return v;
}

// U float4 loads per thread (thread t of the block's kDecBwdThreads), all in
// flight before the first store
template <int U>
struct Ld4 {
  float4 v[U];
  __device__ __forceinline__ void load(const float *src, int n4, int t) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = reinterpret_cast<const float4 *>(src)[min(t + u * kDecBwdThreads, n4 - 1)];
  }
};

__global__ __launch_bounds__(kDecBwdThreads) void k_dec_bwd(DecBwdArgs a) {
  __shared__ DecBwdLds sh;
  // tb: thread of the block (weight staging); t, w: thread and wave within
  // the group, which owns tile buffers s
  const int tb = threadIdx.x, grp = tb / kBlock, t = tb % kBlock;
  const int w = t / kWave, l = __lane_id(), g = l / 16, lc = l % 16;
  DecBwdTile &s = sh.tl[grp];
  const int k = a.k, W = a.W;
  const int nhw = W / 16, n1t = 3 * nhw;
  const int n2t = a.t[0] + a.t[1] + a.t[2];
  const uint32_t M = min(*a.count, (uint32_t)a.cap_anchors);

  // ---- weights and biases into LDS, every load in flight first ----
  {
    const int n1 = kIn * W / 4, wk4 = W * k / 4;
    {
      constexpr int kU1 = (kIn * kMaxW / 4 + kDecBwdThreads - 1) / kDecBwdThreads;  // 2
      Ld4<kU1> x0, x1, x2;
      x0.load(a.w1[0], n1, tb); x1.load(a.w1[1], n1, tb); x2.load(a.w1[2], n1, tb);
      auto put1 = [&](int h, const float4 &v, int i4) {
        // element e = 4 i4 .. 4 i4 + 3 of head h's [kIn][W], row pitch kW1P
        const int e = 4 * i4, r = e / W, c = e - r * W;
        float *d = &sh.W1s[(h * kIn + r) * kW1P + c];
        d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
      };
#pragma unroll
      for (int u = 0; u < kU1; ++u) {
        const int i4 = min(tb + u * kDecBwdThreads, n1 - 1);
        put1(0, x0.v[u], i4); put1(1, x1.v[u], i4); put1(2, x2.v[u], i4);
      }
    }
    constexpr int kWk4 = kMaxW * kMaxK / 4;  // float4s of the k-wide head at most (256)
    constexpr int kU20 = (kWk4 + kDecBwdThreads - 1) / kDecBwdThreads;          // 1
    constexpr int kU21 = (3 * kWk4 + kDecBwdThreads - 1) / kDecBwdThreads;      // 2
    constexpr int kU22 = (7 * kWk4 + kDecBwdThreads - 1) / kDecBwdThreads;      // 4
    Ld4<kU20> y0;
    Ld4<kU21> y1;
    Ld4<kU22> y2;
    y0.load(a.w2[0], wk4, tb); y1.load(a.w2[1], 3 * wk4, tb); y2.load(a.w2[2], 7 * wk4, tb);
    float4 *w2s = reinterpret_cast<float4 *>(sh.W2s);
#pragma unroll
    for (int u = 0; u < kU20; ++u) w2s[min(tb + u * kDecBwdThreads, wk4 - 1)] = y0.v[u];
#pragma unroll
    for (int u = 0; u < kU21; ++u) w2s[wk4 + min(tb + u * kDecBwdThreads, 3 * wk4 - 1)] = y1.v[u];
#pragma unroll
    for (int u = 0; u < kU22; ++u) w2s[4 * wk4 + min(tb + u * kDecBwdThreads, 7 * wk4 - 1)] = y2.v[u];
    if (tb < 3 * W) sh.b1s[tb] = pick3(a.b1, tb / W)[tb % W];
    if (tb < 16 * n2t) {
      int col0;
      const int h = out_head(a, tb / 16, col0), col = col0 + tb % 16;
      sh.b2s[tb] = col < sel3(a.outs, h) ? pick3(a.b2, h)[col] : 0.0f;
    }
  }
  __syncthreads();

  f4 acc1[kMaxT1], acc2[kMaxT2];
#pragma unroll
  for (int q = 0; q < kMaxT1; ++q) acc1[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int q = 0; q < kMaxT2; ++q) acc2[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  float db1r = 0.0f, db2r = 0.0f;  // thread t owns hidden column t / padded output column t

  // pairs of tiles, one per group; a group past the last anchor runs the
  // pass on zero rows (every barrier is the whole block's)
  for (uint32_t pair = blockIdx.x; (uint64_t)pair * kDecGroups * kRB < M; pair += gridDim.x) {
    const uint32_t r0 = (pair * kDecGroups + grp) * kRB;
    const int rows = r0 < M ? (int)min((uint32_t)kRB, M - r0) : 0;
    // ---- inputs: 16 threads per anchor ----
    {
      const int r = t / 16, part = t % 16;
      if (r < rows) {
        const uint32_t j = a.idx[r0 + r];
        if (part < 8) {
          const float4 v = *(const float4 *)(a.feat + (size_t)j * 32 + part * 4);
          s.X[r][part * 4 + 0] = v.x; s.X[r][part * 4 + 1] = v.y;
          s.X[r][part * 4 + 2] = v.z; s.X[r][part * 4 + 3] = v.w;
        } else if (part == 8) {
          s.aidx[r] = j;
          const float d0 = a.pos[3 * (size_t)j] - a.C[0], d1 = a.pos[3 * (size_t)j + 1] - a.C[1];
          const float d2 = a.pos[3 * (size_t)j + 2] - a.C[2];
          const float dist = sqrtf(fma_(d0, d0, fma_(d1, d1, d2 * d2)));
          const float inv = 1.0f / dist;
          s.X[r][32] = dist * a.inv_dmax;
          s.X[r][33] = d0 * inv; s.X[r][34] = d1 * inv; s.X[r][35] = d2 * inv;
          s.Dn[r][0] = dist; s.Dn[r][1] = d0 * inv; s.Dn[r][2] = d1 * inv; s.Dn[r][3] = d2 * inv;
        } else if (part < 12) {
          const int c0 = kIn + 4 * (part - 9);
          s.X[r][c0] = 0.0f; s.X[r][c0 + 1] = 0.0f; s.X[r][c0 + 2] = 0.0f; s.X[r][c0 + 3] = 0.0f;
        }
      } else {
        for (int c = part; c < kInP; c += 16) s.X[r][c] = 0.0f;
      }
    }
    __syncthreads();
    // ---- Hp = X W1 + b1 ----
    // The wave's three column tiles share the A operand; each chunk of k-steps
    // loads all of its operands before its products, so the matrix pipe does
    // not wait on LDS between them.  (A tile past n1t reads a valid address
    // and is not stored.)
    {
      f4 acc[3];
      int boff[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        acc[q] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        const int ct = min(w + 4 * q, n1t - 1);
        const int h = ct / nhw, hc = (ct - h * nhw) * 16 + lc;
        boff[q] = (h * kIn + g) * kW1P + hc;
      }
#pragma unroll
      for (int k0 = 0; k0 < kIn / 4; k0 += 3) {
        float av[3], bv[3][3];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          av[kk] = s.X[lc][(k0 + kk) * 4 + g];
#pragma unroll
          for (int q = 0; q < 3; ++q) bv[q][kk] = sh.W1s[boff[q] + (k0 + kk) * 4 * kW1P];
        }
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
#pragma unroll
          for (int q = 0; q < 3; ++q) acc[q] = mfma(av[kk], bv[q][kk], acc[q]);
        // the chunk's 12 LDS reads first, then its 9 products
        __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 9, 0);
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int ct = w + 4 * q;
        if (ct < n1t) {
#pragma unroll
          for (int i = 0; i < 4; ++i) s.Hp[4 * g + i][ct * 16 + lc] = acc[q][i] + sh.b1s[ct * 16 + lc];
        }
      }
    }
    __syncthreads();
    // ---- Y = relu(Hp) W2 + b2 (padded output columns stay 0) ----
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int c = w + 4 * q;
      if (c < n2t) {
        int col0;
        const int h = out_head(a, c, col0);
        const int ncol = sel3(a.outs, h), col = col0 + lc;
        const bool cv = col < ncol;
        const float *wb = sh.W2s + sel3(a.wo, h);
        f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        // chunks of four k-steps, operands loaded first (W / 4 is a multiple of 4)
        for (int k0 = 0; k0 < W / 4; k0 += 4) {
          float av[4], bv[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int ks = k0 + kk;
            av[kk] = fmaxf(s.Hp[lc][h * W + ks * 4 + g], 0.0f);
            bv[kk] = wb[(ks * 4 + g) * ncol + (cv ? col : 0)];
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) acc = mfma(av[kk], cv ? bv[kk] : 0.0f, acc);
          __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) s.Yd[4 * g + i][c * 16 + lc] = cv ? acc[i] + sh.b2s[c * 16 + lc] : 0.0f;
      }
    }
    __syncthreads();
    // ---- activation derivatives: row r = anchor, lane i = Gaussian ----
    {
      const int r = t / 16, i = t % 16;
      if (r < rows) {
        const uint32_t j = s.aidx[r];
        const bool act = i < k;
        const int ii = act ? i : 0;
        float *yr = s.Yd[r];
        const size_t sl = (size_t)(r0 + r) * k + ii;
        const float *lv = a.oscale + 3 * (size_t)j;
        const float *bs = a.bscale + 3 * (size_t)j;
        const float *o = a.offsets + ((size_t)j * k + ii) * 3;
        float dgv[kGaussFields];
#pragma unroll
        for (int f = 0; f < kGaussFields; ++f) dgv[f] = act ? a.dgauss[f * a.dstride + sl] : 0.0f;
        float dp[3], dl[3], dbs[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          dp[c] = dgv[c];
          dl[c] = dgv[c] * o[c];
        }
        float *row = a.rows + (size_t)(r0 + r) * a.rstride;
        if (act) {
#pragma unroll
          for (int c = 0; c < 3; ++c) row[kRowOff + 3 * ii + c] = dgv[c] * lv[c];
        }
        const int ys = a.offp[2] + 7 * ii, yc = a.offp[1] + 3 * ii, ya = a.offp[0] + ii;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float sg = sigm(yr[ys + c]);
          dbs[c] = dgv[3 + c] * sg;
          if (act) yr[ys + c] = dgv[3 + c] * bs[c] * sg * (1.0f - sg);
        }
        if (act) {
          const float q0 = yr[ys + 3], q1 = yr[ys + 4], q2 = yr[ys + 5], q3 = yr[ys + 6];
          const float n2 = fma_(q0, q0, fma_(q1, q1, fma_(q2, q2, q3 * q3)));
          float dq[4] = {0, 0, 0, 0};
          if (n2 > 0.0f) {
            const float inv = 1.0f / sqrtf(n2);
            const float u[4] = {q0 * inv, q1 * inv, q2 * inv, q3 * inv};
            float dot = 0.0f;
#pragma unroll
            for (int c = 0; c < 4; ++c) dot = fma_(u[c], dgv[6 + c], dot);
#pragma unroll
            for (int c = 0; c < 4; ++c) dq[c] = (dgv[6 + c] - u[c] * dot) * inv;
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) yr[ys + 3 + c] = dq[c];
          const float op = tanhf(yr[ya]);
          yr[ya] = dgv[10] * (1.0f - op * op);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float sg = sigm(yr[yc + c]);
            yr[yc + c] = dgv[11 + c] * sg * (1.0f - sg);
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
            s.dp[r][c] = dp[c];
            row[row_osc(k) + c] = dl[c];
            row[row_bsc(k) + c] = dbs[c];
          }
        }
      } else {
        for (int c = i; c < 16 * n2t; c += 16) s.Yd[r][c] = 0.0f;
      }
    }
    __syncthreads();
    // ---- dHp = (dY W2^T) * [Hp > 0]; dW2 += relu(Hp)^T dY; db2 ----
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int ct = w + 4 * q;
      if (ct < n1t) {
        const int h = ct / nhw, hc = (ct - h * nhw) * 16 + lc;
        const int ncol = sel3(a.outs, h);
        const float *wb = sh.W2s + sel3(a.wo, h) + hc * ncol;
        const float *yr = s.Yd[lc] + sel3(a.offp, h);
        const int nks = (ncol + 3) / 4;
        f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        // chunks of four k-steps, operands loaded first (clamped reads; a
        // k past ncol multiplies by 0)
        for (int k0 = 0; k0 < nks; k0 += 4) {
          float av[4], bv[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int kq = min((k0 + kk) * 4 + g, ncol - 1);
            av[kk] = yr[kq];
            bv[kk] = wb[kq];
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            if (k0 + kk < nks) acc = mfma(av[kk], (k0 + kk) * 4 + g < ncol ? bv[kk] : 0.0f, acc);
          __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int col = ct * 16 + lc;
          s.dH[4 * g + i][col] = s.Hp[4 * g + i][col] > 0.0f ? acc[i] : 0.0f;
        }
      }
    }
    // two output tiles at a time, their 16 operands loaded first (a tile
    // past the last reads tile 0's and is skipped)
#pragma unroll
    for (int q0 = 0; q0 < kMaxT2; q0 += 2) {
      float av[2][kRB / 4], bv[2][kRB / 4];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int T = w + 4 * (q0 + u);
        const int Tc = T < nhw * n2t ? T : 0;
        const int rt = Tc / n2t, c = Tc - rt * n2t;
        int col0;
        const int h = out_head(a, c, col0);
#pragma unroll
        for (int ks = 0; ks < kRB / 4; ++ks) {
          const int row = ks * 4 + g;
          av[u][ks] = fmaxf(s.Hp[row][h * W + rt * 16 + lc], 0.0f);
          bv[u][ks] = s.Yd[row][c * 16 + lc];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int q = q0 + u;
        if (q < kMaxT2 && w + 4 * q < nhw * n2t) {
#pragma unroll
          for (int ks = 0; ks < kRB / 4; ++ks) acc2[q] = mfma(av[u][ks], bv[u][ks], acc2[q]);
        }
      }
      __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
    }
    if (t < 16 * n2t)
      for (int r = 0; r < kRB; ++r) db2r += s.Yd[r][t];
    __syncthreads();
    // ---- dX = dHp W1^T; dW1 += X^T dHp; db1 ----
    if (w < 3) {
      const int n = w * 16 + lc;
      const bool nv = n < kIn;
      f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      // chunks of eight k-steps (3 W / 4 is a multiple of 12), operands first
      const int nn = nv ? n : 0;
      for (int k0 = 0; k0 < 3 * W / 4; k0 += 4) {
        float av[4], bv[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int kq = (k0 + kk) * 4 + g, h = kq / W, kh = kq - h * W;
          av[kk] = s.dH[lc][kq];
          bv[kk] = sh.W1s[(h * kIn + nn) * kW1P + kh];
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = mfma(av[kk], nv ? bv[kk] : 0.0f, acc);
        __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) s.dX[4 * g + i][n] = acc[i];
    }
#pragma unroll
    for (int q0 = 0; q0 < kMaxT1; q0 += 2) {
      float av[2][kRB / 4], bv[2][kRB / 4];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int T = w + 4 * (q0 + u);
        const int Tc = T < 3 * n1t ? T : 0;
        const int rt = Tc / n1t, ct = Tc - rt * n1t;
#pragma unroll
        for (int ks = 0; ks < kRB / 4; ++ks) {
          const int row = ks * 4 + g;
          av[u][ks] = s.X[row][rt * 16 + lc];
          bv[u][ks] = s.dH[row][ct * 16 + lc];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int q = q0 + u;
        if (q < kMaxT1 && w + 4 * q < 3 * n1t) {
#pragma unroll
          for (int ks = 0; ks < kRB / 4; ++ks) acc1[q] = mfma(av[u][ks], bv[u][ks], acc1[q]);
        }
      }
      __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
    }
    if (t < 3 * W)
      for (int r = 0; r < kRB; ++r) db1r += s.dH[r][t];
    __syncthreads();
    // ---- features and position: 32 lanes per anchor ----
    for (int r = t / 32; r < rows; r += kBlock / 32) {
      const int f = t % 32;
      float *row = a.rows + (size_t)(r0 + r) * a.rstride;
      row[kRowFeat + f] = s.dX[r][f];
      if (f == 0) {
        // the position enters through the decoded means and through the
        // distance and direction inputs
        const float dist = s.Dn[r][0], u0 = s.Dn[r][1], u1 = s.Dn[r][2], u2 = s.Dn[r][3];
        const float *dx = s.dX[r];
        const float dot = fma_(u0, dx[33], fma_(u1, dx[34], u2 * dx[35]));
        const float sd = dx[32] * a.inv_dmax, id = 1.0f / dist;
        row[kRowPos + 0] = s.dp[r][0] + fma_(u0, sd, (dx[33] - u0 * dot) * id);
        row[kRowPos + 1] = s.dp[r][1] + fma_(u1, sd, (dx[34] - u1 * dot) * id);
        row[kRowPos + 2] = s.dp[r][2] + fma_(u2, sd, (dx[35] - u2 * dot) * id);
      }
    }
    __syncthreads();
  }

  // ---- the second group's sums into the first's (group order), then this
  // block's weight-gradient sums, one row of the workspace ----
  float *xch = reinterpret_cast<float *>(&sh.tl[0]);
  __syncthreads();  // every group is done with its tile buffers
  if (grp == 1) {
#pragma unroll
    for (int q = 0; q < kMaxT1; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) xch[(4 * q + i) * kBlock + t] = acc1[q][i];
#pragma unroll
    for (int q = 0; q < kMaxT2; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) xch[(4 * (kMaxT1 + q) + i) * kBlock + t] = acc2[q][i];
    xch[(kXchSlots - 2) * kBlock + t] = db1r;
    xch[(kXchSlots - 1) * kBlock + t] = db2r;
  }
  __syncthreads();
  if (grp == 1) return;
#pragma unroll
  for (int q = 0; q < kMaxT1; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc1[q][i] += xch[(4 * q + i) * kBlock + t];
#pragma unroll
  for (int q = 0; q < kMaxT2; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc2[q][i] += xch[(4 * (kMaxT1 + q) + i) * kBlock + t];
  db1r += xch[(kXchSlots - 2) * kBlock + t];
  db2r += xch[(kXchSlots - 1) * kBlock + t];
  float *pp = a.part + (size_t)blockIdx.x * a.P;
#pragma unroll
  for (int q = 0; q < kMaxT1; ++q) {
    const int T = w + 4 * q;
    if (T < 3 * n1t) {
      const int rt = T / n1t, ct = T - rt * n1t;
      const int col = ct * 16 + lc, h = col / W, hc = col - h * W;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int in = rt * 16 + 4 * g + i;
        if (in < kIn) pp[(h * kIn + in) * W + hc] = acc1[q][i];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kMaxT2; ++q) {
    const int T = w + 4 * q;
    if (T < nhw * n2t) {
      const int rt = T / n2t, c = T - rt * n2t;
      int col0;
      const int h = out_head(a, c, col0);
      const int col = col0 + lc, ncol = sel3(a.outs, h);
      if (col < ncol) {
#pragma unroll
        for (int i = 0; i < 4; ++i) pp[a.p_w2 + sel3(a.wo, h) + (rt * 16 + 4 * g + i) * ncol + col] = acc2[q][i];
      }
    }
  }
  if (t < 3 * W) pp[a.p_b1 + t] = db1r;
  if (t < 16 * n2t) {
    int col0;
    const int h = out_head(a, t / 16, col0), col = col0 + t % 16;
    const int hoff = h == 0 ? 0 : (h == 1 ? k : 4 * k);
    if (col < sel3(a.outs, h)) pp[a.p_b2 + hoff + col] = db2r;
  }
}

// Adds the blocks' rows, in block order, into the weight and bias gradients.
struct DecRedArgs {
  int P, nblk, k, W;
  int p_w2, p_b1, p_b2;
  const float *part;
  float *w1[3], *b1[3], *w2[3], *b2[3];
};

// 64 outputs per block, four thread groups per output, each summing every
// fourth row with eight loads in flight; the four group sums are added in a
// fixed order.
constexpr int kRedOut = 64;

__global__ __launch_bounds__(kBlock) void k_dec_bwd_reduce(DecRedArgs a) {
  __shared__ float red[kBlock / kRedOut][kRedOut];
  const int oc = threadIdx.x % kRedOut, grp = threadIdx.x / kRedOut;
  const int o = blockIdx.x * kRedOut + oc;
  const int oo = min(o, a.P - 1);
  float part = 0.0f;
  for (int b0 = grp; b0 < a.nblk; b0 += 8 * (kBlock / kRedOut)) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = min(b0 + u * (kBlock / kRedOut), a.nblk - 1);
      v[u] = a.part[(size_t)b * a.P + oo];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + u * (kBlock / kRedOut) < a.nblk) part += v[u];
  }
  red[grp][oc] = part;
  __syncthreads();
  if (grp != 0 || o >= a.P) return;
  float sum = 0.0f;
#pragma unroll
  for (int q = 0; q < kBlock / kRedOut; ++q) sum += red[q][oc];
  const int k = a.k, W = a.W;
  float *dst;
  if (o < a.p_w2) {
    const int h = o / (kIn * W);
    dst = pick3(a.w1, h) + (o - h * kIn * W);
  } else if (o < a.p_b1) {
    const int r = o - a.p_w2;
    const int h = r < W * k ? 0 : (r < 4 * W * k ? 1 : 2);
    dst = pick3(a.w2, h) + (r - (h == 0 ? 0 : (h == 1 ? W * k : 4 * W * k)));
  } else if (o < a.p_b2) {
    const int r = o - a.p_b1, h = r / W;
    dst = pick3(a.b1, h) + (r - h * W);
  } else {
    const int r = o - a.p_b2;
    const int h = r < k ? 0 : (r < 4 * k ? 1 : 2);
    dst = pick3(a.b2, h) + (r - (h == 0 ? 0 : (h == 1 ? k : 4 * k)));
  }
  *dst += sum;
}

// Adds each listed anchor's gradient row into the anchor arrays; one
// thread per row element.  The anchors of one list are distinct, so no two
// threads touch the same element.
struct DecApplyArgs {
  int k, rstride, cap_anchors;
  const uint32_t *idx, *count;
  const float *rows;
  float *gpos, *gfeat, *goff, *gosc, *gbsc;
};

__global__ __launch_bounds__(kBlock) void k_dec_bwd_apply(DecApplyArgs a) {
  const uint32_t M = min(*a.count, (uint32_t)a.cap_anchors);
  const uint64_t n = (uint64_t)M * a.rstride;
  const int k = a.k;
  for (uint64_t e = (uint64_t)blockIdx.x * kBlock + threadIdx.x; e < n;
       e += (uint64_t)gridDim.x * kBlock) {
    const uint32_t r = (uint32_t)(e / a.rstride);
    const int q = (int)(e - (uint64_t)r * a.rstride);
    const size_t j = a.idx[r];
    float *d;
    if (q < kRowFeat) d = a.gpos + 3 * j + q;
    else if (q < kRowOff) d = a.gfeat + 32 * j + (q - kRowFeat);
    else if (q < row_osc(k)) d = a.goff + 3 * (size_t)k * j + (q - kRowOff);
    else if (q < row_bsc(k)) d = a.gosc + 3 * j + (q - row_osc(k));
    else d = a.gbsc + 3 * j + (q - row_bsc(k));
    *d += a.rows[e];
  }
}

int partial_len(int k, int W) { return 3 * kIn * W + 11 * k * W + 3 * W + 11 * k; }


// persistent blocks, each taking pairs of 16-anchor tiles
int grid_for(int64_t mcap) {
  const int64_t per = (int64_t)kDecGroups * kRB;
  return (int)std::max<int64_t>(1, std::min<int64_t>((mcap + per - 1) / per, kDecBwdGrid));
}

// the anchor rows follow the block partial rows, 256-byte aligned
size_t rows_offset(int64_t mcap, int k, int W) {
  return ((size_t)grid_for(mcap) * (size_t)partial_len(k, W) * sizeof(float) + 255) & ~(size_t)255;
}

}  // namespace

}  // namespace octgs

using namespace octgs;

extern "C" {

size_t octgs_decode_bwd_workspace_bytes(int64_t max_anchors, int32_t k, int32_t width) {
  if (max_anchors < 0 || max_anchors > 0x7fffffff || k < 1 || k > kMaxK || width < 16 ||
      width > kMaxW || width % 16)
    return 0;
  return rows_offset(max_anchors, k, width) + (size_t)max_anchors * row_len(k) * sizeof(float) + 256;
}

namespace {

// Shared argument checks of the two halves; 0 or an octgs_status.
int check_shapes(const octgs_anchors *an, const octgs_mlp *mlp, int64_t gauss_capacity,
                 size_t ws_bytes) {
  if (an->feat_dim != 32) return OCTGS_EUNSUPPORTED;
  if (an->k < 1 || an->k > kMaxK) return OCTGS_EUNSUPPORTED;
  if (mlp->width < 16 || mlp->width > kMaxW || mlp->width % 16) return OCTGS_EUNSUPPORTED;
  if (gauss_capacity < an->k) return OCTGS_EINVAL;
  const int64_t mcap = gauss_capacity / an->k;
  if (mcap > 0x7fffffff) return OCTGS_EINVAL;
  if (ws_bytes < octgs_decode_bwd_workspace_bytes(mcap, an->k, mlp->width)) return OCTGS_ENOSPC;
  return OCTGS_OK;
}

}  // namespace

int octgs_decode_bwd_rows(const octgs_anchors *an, const octgs_mlp *mlp, const octgs_camera *cam,
                          const uint32_t *idx, const uint32_t *count, const float *d_gauss,
                          int64_t gauss_capacity, void *ws, size_t ws_bytes, octgs_stream stream) {
  if (!an || !mlp || !cam || !idx || !count || !d_gauss || !ws) return OCTGS_EINVAL;
  // transition blending is an inference-time mode; training uses Eq. 7 alone
  if (cam->lod_blend) return OCTGS_EUNSUPPORTED;
  if (const int e = check_shapes(an, mlp, gauss_capacity, ws_bytes)) return e;
  if (!an->pos || !an->feat || !an->offsets || !an->offset_scale || !an->base_scale)
    return OCTGS_EINVAL;
  for (int h = 0; h < 3; ++h) {
    if (!mlp->w1[h] || !mlp->b1[h] || !mlp->w2[h] || !mlp->b2[h]) return OCTGS_EINVAL;
    if (((uintptr_t)mlp->w1[h] | (uintptr_t)mlp->w2[h]) & 15) return OCTGS_EINVAL;
  }
  if (!(an->d_max > 0.0f)) return OCTGS_EINVAL;
  const int k = an->k, W = mlp->width;
  const int64_t mcap = gauss_capacity / k;
  DecBwdArgs a;
  a.k = k; a.W = W; a.cap_anchors = (int)mcap;
  a.outs[0] = k; a.outs[1] = 3 * k; a.outs[2] = 7 * k;
  for (int h = 0; h < 3; ++h) a.t[h] = (a.outs[h] + 15) / 16;
  a.offp[0] = 0; a.offp[1] = 16 * a.t[0]; a.offp[2] = 16 * (a.t[0] + a.t[1]);
  a.wo[0] = 0; a.wo[1] = W * k; a.wo[2] = 4 * W * k;
  a.P = partial_len(k, W);
  a.p_w2 = 3 * kIn * W; a.p_b1 = a.p_w2 + 11 * k * W; a.p_b2 = a.p_b1 + 3 * W;
  a.inv_dmax = 1.0f / an->d_max;
  for (int c = 0; c < 3; ++c) a.C[c] = cam->C[c];
  a.pos = an->pos; a.feat = an->feat; a.offsets = an->offsets;
  a.oscale = an->offset_scale; a.bscale = an->base_scale;
  for (int h = 0; h < 3; ++h) {
    a.w1[h] = mlp->w1[h]; a.b1[h] = mlp->b1[h]; a.w2[h] = mlp->w2[h]; a.b2[h] = mlp->b2[h];
  }
  a.idx = idx; a.count = count;
  a.dgauss = d_gauss; a.dstride = gauss_capacity;
  a.part = (float *)ws;
  a.rows = (float *)((char *)ws + rows_offset(mcap, k, W));
  a.rstride = row_len(k);
  hipLaunchKernelGGL(k_dec_bwd, dim3(grid_for(mcap)), dim3(kDecBwdThreads), 0, (hipStream_t)stream, a);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_decode_bwd_apply(const octgs_anchors *an, const octgs_mlp *mlp, const uint32_t *idx,
                           const uint32_t *count, int64_t gauss_capacity,
                           const octgs_anchor_grads *ga, const octgs_mlp_grads *gm, const void *ws,
                           size_t ws_bytes, octgs_stream stream) {
  if (!an || !mlp || !idx || !count || !ga || !gm || !ws) return OCTGS_EINVAL;
  if (const int e = check_shapes(an, mlp, gauss_capacity, ws_bytes)) return e;
  if (!ga->pos || !ga->feat || !ga->offsets || !ga->offset_scale || !ga->base_scale)
    return OCTGS_EINVAL;
  for (int h = 0; h < 3; ++h)
    if (!gm->w1[h] || !gm->b1[h] || !gm->w2[h] || !gm->b2[h]) return OCTGS_EINVAL;
  const int k = an->k, W = mlp->width;
  const int64_t mcap = gauss_capacity / k;
  hipStream_t s = (hipStream_t)stream;
  DecApplyArgs ap;
  ap.k = k; ap.rstride = row_len(k); ap.cap_anchors = (int)mcap;
  ap.idx = idx; ap.count = count;
  ap.rows = (const float *)((const char *)ws + rows_offset(mcap, k, W));
  ap.gpos = ga->pos; ap.gfeat = ga->feat; ap.goff = ga->offsets;
  ap.gosc = ga->offset_scale; ap.gbsc = ga->base_scale;
  const int agrid = (int)std::min<int64_t>(std::max<int64_t>((mcap * row_len(k) + kBlock - 1) / kBlock, 1), 4096);
  hipLaunchKernelGGL(k_dec_bwd_apply, dim3(agrid), dim3(kBlock), 0, s, ap);
  DecRedArgs r;
  r.P = partial_len(k, W); r.nblk = grid_for(mcap); r.k = k; r.W = W;
  r.p_w2 = 3 * kIn * W; r.p_b1 = r.p_w2 + 11 * k * W; r.p_b2 = r.p_b1 + 3 * W;
  r.part = (const float *)ws;
  for (int h = 0; h < 3; ++h) {
    r.w1[h] = gm->w1[h]; r.b1[h] = gm->b1[h]; r.w2[h] = gm->w2[h]; r.b2[h] = gm->b2[h];
  }
  hipLaunchKernelGGL(k_dec_bwd_reduce, dim3((r.P + kRedOut - 1) / kRedOut), dim3(kBlock), 0, s, r);
  return hipGetLastError() == hipSuccess ? OCTGS_OK : OCTGS_EHIP;
}

int octgs_decode_bwd(const octgs_anchors *an, const octgs_mlp *mlp, const octgs_camera *cam,
                     const uint32_t *idx, const uint32_t *count, const float *d_gauss,
                     int64_t gauss_capacity, const octgs_anchor_grads *ga,
                     const octgs_mlp_grads *gm, void *ws, size_t ws_bytes, octgs_stream stream) {
  if (!ga || !gm) return OCTGS_EINVAL;
  if (!ga->pos || !ga->feat || !ga->offsets || !ga->offset_scale || !ga->base_scale)
    return OCTGS_EINVAL;
  for (int h = 0; h < 3; ++h)
    if (!gm->w1[h] || !gm->b1[h] || !gm->w2[h] || !gm->b2[h]) return OCTGS_EINVAL;
  const int e = octgs_decode_bwd_rows(an, mlp, cam, idx, count, d_gauss, gauss_capacity, ws,
                                      ws_bytes, stream);
  if (e != OCTGS_OK) return e;
  return octgs_decode_bwd_apply(an, mlp, idx, count, gauss_capacity, ga, gm, ws, ws_bytes, stream);
}

}  // extern "C"
