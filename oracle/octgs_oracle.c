/*
 * Octree-GS render path: plain, slow CPU oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * This file is the reference the HIP library is checked against.  It shares
 * no code, header, table or constant with the HIP path.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it; the product
 * path never calls it.
 *
 * Arithmetic:
 *  - Continuous quantities (decoded attributes, 2D means, conics, colours,
 *    transmittance, gradients) are computed in double precision from the
 *    float inputs.
 *  - Discrete decisions (anchor selection, visibility, Gaussian culls, screen
 *    tile rectangles and depth keys) are taken in single precision by a fixed,
 *    written-out sequence of operations (the "canonical FP32 decisions"),
 *    because a GPU kernel working in float must reach bit-identical integer
 *    results.  Each decision function below lists its operation order; every
 *    fused multiply-add is an explicit fmaf and the file is compiled with
 *    -ffp-contract=off so no other operation is fused.
 *
 * Paper passages followed (Octree-GS, arXiv 2403.17898):
 *  - Eq. 1 and the covariance factorisation Sigma = R S S^T R^T (Sec. III-A).
 *  - Eq. 2, front-to-back alpha blending (Sec. III-A).
 *  - Eq. 3, neural Gaussian positions mu_i = x_v + O_i * l_v (Sec. III-B).
 *  - Eq. 4, attributes decoded by MLPs from feature, relative viewing
 *    distance and viewing direction (Sec. III-B).
 *  - Eq. 7 and the cumulative selection rule L_j <= L_hat (Sec. IV-A,
 *    "Anchor Selection").
 *
 * Parity pins (checked by tests that do not call the HIP path): closed-form
 * single- and two-Gaussian images, brute-force per-pixel compositing, the
 * threshold form of Eq. 7 against its literal log2 form, invariants of the
 * transmittance, and central finite differences of the backward pass;
 * visibility against points and spheres placed just inside and outside each
 * frustum plane of a generic camera (planes built from back-projected edge
 * rays), conservativeness (culling never changes the image), invariance of
 * lists and images under a rotation of scene and camera together, and the
 * closed-form conic of Gaussians given in camera space under a rotated
 * camera; the predictor's inputs in closed form, its loss against the
 * textbook cross-entropy and its gradient against finite differences.  The
 * pin families are shown to catch mistakes planted in copies of this file.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_API __attribute__((visibility("default")))

/* Camera record as passed from Python: R (9, row-major world->camera),
 * C (3), fx, fy, cx, cy, z_near, s^2 (focal scale of Eq. 7, squared). */
typedef struct {
  float R[9], C[3], fx, fy, cx, cy, z_near, s2;
  int W, H;
} cam_t;

static cam_t load_cam(const float *c, int W, int H) {
  cam_t k;
  memcpy(k.R, c, 9 * sizeof(float));
  memcpy(k.C, c + 9, 3 * sizeof(float));
  k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
  k.z_near = c[16]; k.s2 = c[17];
  k.W = W; k.H = H;
  return k;
}

/* Raster parameters: alpha_max, alpha_min, t_min, dilation, jac_clamp, bg[3]. */
typedef struct {
  float alpha_max, alpha_min, t_min, dilation, jac_clamp, bg[3];
} prm_t;

static prm_t load_prm(const float *p) {
  prm_t q;
  q.alpha_max = p[0]; q.alpha_min = p[1]; q.t_min = p[2];
  q.dilation = p[3]; q.jac_clamp = p[4];
  q.bg[0] = p[5]; q.bg[1] = p[6]; q.bg[2] = p[7];
  return q;
}

/* ======================================================================
 * Canonical FP32 decisions
 * ====================================================================== */

/* camera-space position, float: d = p - C; x_c = R d with each row as
 * fmaf(R0, d0, fmaf(R1, d1, R2 * d2)). */
static void cam_xform_f(const cam_t *k, float px, float py, float pz,
                        float *xc, float *yc, float *zc) {
  float d0 = px - k->C[0], d1 = py - k->C[1], d2 = pz - k->C[2];
  *xc = fmaf(k->R[0], d0, fmaf(k->R[1], d1, k->R[2] * d2));
  *yc = fmaf(k->R[3], d0, fmaf(k->R[4], d1, k->R[5] * d2));
  *zc = fmaf(k->R[6], d0, fmaf(k->R[7], d1, k->R[8] * d2));
}

/* Visibility of an anchor's bound sphere (camera-space centre, radius rho),
 * conservative for the render: the sphere is culled only if no Gaussian
 * inside it can reach a pixel centre of the image.  Reading of "visible
 * anchors" (Sec. IV-A) with the EWA projection of Sec. III-A:
 *  - near plane: every Gaussian centre of a sphere entirely in front of
 *    z_near fails the projection's z > z_near cull;
 *  - side planes: the drawn footprint of a Gaussian is the 3-sigma ellipse of
 *    J W Sigma W^T J^T + dilation I.  It lies inside the linear image of the
 *    3-sigma ellipsoid widened by 3 sqrt(dilation) pixels (support functions
 *    add under the square root bound), so each side plane is moved out by
 *    pad = 3 sqrt(dilation) pixels.  The linear image uses the Jacobian at the
 *    Gaussian's centre with x/z clamped to +-lx (lx = jac_clamp * half-image
 *    tangent); for the right plane x = t z (t = (W - cx + pad) / fx) a point p
 *    of the ellipsoid maps to u - (cx + fx t) = (fx / z_mu) [h(p) -
 *    (t_c - t)(z_p - z_mu)] with h = x - t z and t_c the clamped slope, and
 *    |t_c - t| <= |lx - t| whenever the centre is beyond the plane, while
 *    |z_p - z_mu| <= 3 max scale <= rho.  So the sphere is culled only if
 *    h(centre) > rho (sec + |lx - t|), sec = sqrt(1 + t^2) (the plane
 *    normal's length); the other three planes alike.
 * Canonical FP32 sequence:
 *   pad = 3 * sqrtf(dilation)
 *   tl = (cx + pad) / fx, tr = ((W - cx) + pad) / fx, tt = (cy + pad) / fy,
 *   tb = ((H - cy) + pad) / fy
 *   lx = jac_clamp * ((0.5 * W) / fx), ly = jac_clamp * ((0.5 * H) / fy)
 *   m_side = sqrtf(fmaf(t, t, 1)) + fabsf(l - t) with (t, l) of that side
 *   visible iff zc + rho >= z_near and xc <= fmaf(tr, zc, rho * mr),
 *   -xc <= fmaf(tl, zc, rho * ml), yc <= fmaf(tb, zc, rho * mb),
 *   -yc <= fmaf(tt, zc, rho * mt). */
static int sphere_visible_f(const cam_t *k, const prm_t *pp, float xc, float yc, float zc,
                            float rho) {
  float pad = 3.0f * sqrtf(pp->dilation);
  float tl = (k->cx + pad) / k->fx, tr = (((float)k->W - k->cx) + pad) / k->fx;
  float tt = (k->cy + pad) / k->fy, tb = (((float)k->H - k->cy) + pad) / k->fy;
  float lx = pp->jac_clamp * ((0.5f * (float)k->W) / k->fx);
  float ly = pp->jac_clamp * ((0.5f * (float)k->H) / k->fy);
  float ml = sqrtf(fmaf(tl, tl, 1.0f)) + fabsf(lx - tl);
  float mr = sqrtf(fmaf(tr, tr, 1.0f)) + fabsf(lx - tr);
  float mt = sqrtf(fmaf(tt, tt, 1.0f)) + fabsf(ly - tt);
  float mb = sqrtf(fmaf(tb, tb, 1.0f)) + fabsf(ly - tb);
  if (!(zc + rho >= k->z_near)) return 0;
  if (!(xc <= fmaf(tr, zc, rho * mr))) return 0;
  if (!(-xc <= fmaf(tl, zc, rho * ml))) return 0;
  if (!(yc <= fmaf(tb, zc, rho * mb))) return 0;
  if (!(-yc <= fmaf(tt, zc, rho * mt))) return 0;
  return 1;
}

/* Eq. 7 selection threshold.  With integer level L in [0, K-1] and the clamp
 * Phi applied to the sum log2(d_max / (d s)) + Delta L, the rule
 * L <= floor(Phi(...)) holds for every anchor of level 0 and, for L >= 1, iff
 * L - Delta L <= log2(d_max / (d s)), i.e. iff d^2 s^2 <= (d_max 2^(Delta L - L))^2.
 * thr2 is that square rounded once to float (computed in double); level-0
 * anchors get +inf. */
ORC_API void orc_lod_thr2(int64_t n, const uint8_t *level, const float *lod_bias,
                          float d_max, float *thr2) {
  for (int64_t j = 0; j < n; ++j) {
    if (level[j] == 0) { thr2[j] = INFINITY; continue; }
    double t = (double)d_max * exp2((double)lod_bias[j] - (double)level[j]);
    thr2[j] = (float)(t * t);
  }
}

/* Conservative bound radius of an anchor's Gaussians: the farthest offset
 * |O_i * l| plus three times the largest base scale (decoded scales are the
 * base scale times a sigmoid, so never larger).  Canonical float:
 * a = O0*l0, b = O1*l1, c = O2*l2; n = sqrtf(fmaf(a,a,fmaf(b,b,c*c)));
 * m = max_i n; rho = fmaf(3, max(bs0, bs1, bs2), m). */
ORC_API void orc_bound_radius(int64_t n, int k, const float *offsets,
                              const float *offset_scale, const float *base_scale,
                              float *rho) {
  for (int64_t j = 0; j < n; ++j) {
    const float *l = offset_scale + 3 * j;
    float m = 0.0f;
    for (int i = 0; i < k; ++i) {
      const float *o = offsets + (j * k + i) * 3;
      float a = o[0] * l[0], b = o[1] * l[1], c = o[2] * l[2];
      float nn = sqrtf(fmaf(a, a, fmaf(b, b, c * c)));
      m = fmaxf(m, nn);
    }
    const float *bs = base_scale + 3 * j;
    float bmax = fmaxf(fmaxf(bs[0], bs[1]), bs[2]);
    rho[j] = fmaf(3.0f, bmax, m);
  }
}

/* Bound radius of an anchor carrying explicit Gaussians (the 3D-GS
 * instance of the anchor framework): the largest centre distance from the
 * anchor plus three times the largest scale, so the sphere holds every
 * Gaussian's 3-sigma extent.  Canonical FP32: d = mean - pos,
 * |d| = sqrtf(fmaf(d0, d0, fmaf(d1, d1, d2 * d2))); the largest scale is
 * exp of the largest log-scale, evaluated in double and rounded once.
 * mean and log_scale are [n][k][3]. */
ORC_API void orc_bound_radius_explicit(int64_t n, int k, const float *pos, const float *mean,
                                       const float *log_scale, float *rho) {
  for (int64_t j = 0; j < n; ++j) {
    const float *p = pos + 3 * j;
    float m = 0.0f, lmax = -INFINITY;
    for (int i = 0; i < k; ++i) {
      const float *mu = mean + (j * k + i) * 3;
      const float *ls = log_scale + (j * k + i) * 3;
      float a = mu[0] - p[0], b = mu[1] - p[1], c = mu[2] - p[2];
      float nn = sqrtf(fmaf(a, a, fmaf(b, b, c * c)));
      m = fmaxf(m, nn);
      lmax = fmaxf(lmax, fmaxf(fmaxf(ls[0], ls[1]), ls[2]));
    }
    const float smax = (float)exp((double)lmax);
    rho[j] = fmaf(3.0f, smax, m);
  }
}

/* Canonical FP32 selection: visible(sphere) && d^2 * s^2 <= thr2, with
 * d^2 = fmaf(d0, d0, fmaf(d1, d1, d2 * d2)) for d = p - C.  Writes a 0/1
 * mask and returns the selected count. pos is [n][3]. */
ORC_API int64_t orc_select_fp32(int64_t n, const float *pos, const float *thr2,
                                const float *rho, int blend, const float *camf, int W, int H,
                                const float *prmf, uint8_t *mask) {
  cam_t k = load_cam(camf, W, H);
  prm_t pp = load_prm(prmf);
  int64_t cnt = 0;
  for (int64_t j = 0; j < n; ++j) {
    float px = pos[3 * j], py = pos[3 * j + 1], pz = pos[3 * j + 2];
    float d0 = px - k.C[0], d1 = py - k.C[1], d2 = pz - k.C[2];
    float dd = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
    /* LOD transition blending also takes level L_hat + 1, i.e. L <= L* + 1:
     * the threshold of level L - 1, 4 thr2 (exact in FP32).  An anchor of
     * level 1 whose unclamped L* is negative gets factor 0 and is left out */
    const float th = blend ? 4.0f * thr2[j] : thr2[j];
    int sel = (dd * k.s2 <= th);
    if (sel) {
      float xc, yc, zc;
      cam_xform_f(&k, px, py, pz, &xc, &yc, &zc);
      sel = sphere_visible_f(&k, &pp, xc, yc, zc, rho[j]);
    }
    mask[j] = (uint8_t)sel;
    cnt += sel;
  }
  return cnt;
}

/* Literal Eq. 7 in double: L_hat = floor(Phi(log2(d_max / (d s)) + Delta L)),
 * Phi clamping to [0, K-1]; select iff L <= L_hat, plus the same sphere
 * visibility evaluated in double.  Used only to pin the threshold form. */
ORC_API int64_t orc_select_eq7(int64_t n, const float *pos, const uint8_t *level,
                               const float *lod_bias, float d_max, int n_levels,
                               const float *rho, int blend, const float *camf, int W, int H,
                               const float *prmf, uint8_t *mask) {
  cam_t k = load_cam(camf, W, H);
  prm_t pp = load_prm(prmf);
  double s = sqrt((double)k.s2);
  double pad = 3.0 * sqrt((double)pp.dilation);
  double tl = ((double)k.cx + pad) / k.fx, tr = ((double)W - k.cx + pad) / k.fx;
  double tt = ((double)k.cy + pad) / k.fy, tb = ((double)H - k.cy + pad) / k.fy;
  double lx = (double)pp.jac_clamp * 0.5 * W / k.fx, ly = (double)pp.jac_clamp * 0.5 * H / k.fy;
  double ml = sqrt(tl * tl + 1) + fabs(lx - tl), mr = sqrt(tr * tr + 1) + fabs(lx - tr);
  double mt = sqrt(tt * tt + 1) + fabs(ly - tt), mb = sqrt(tb * tb + 1) + fabs(ly - tb);
  int64_t cnt = 0;
  for (int64_t j = 0; j < n; ++j) {
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = (double)pos[3 * j + a] - (double)k.C[a];
    double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double lstar = log2((double)d_max / (dist * s)) + (double)lod_bias[j];
    if (lstar < 0) lstar = 0;
    if (lstar > n_levels - 1) lstar = n_levels - 1;
    /* cumulative rule L <= L_hat; with transition blending also L = L_hat + 1
     * when its opacity factor L* - L_hat is not 0 */
    int sel = ((double)level[j] <= floor(lstar)) ||
              (blend && (double)level[j] == floor(lstar) + 1.0 && lstar > floor(lstar));
    if (sel) {
      double xc = k.R[0] * d[0] + k.R[1] * d[1] + k.R[2] * d[2];
      double yc = k.R[3] * d[0] + k.R[4] * d[1] + k.R[5] * d[2];
      double zc = k.R[6] * d[0] + k.R[7] * d[1] + k.R[8] * d[2];
      double r = rho[j];
      sel = (zc + r >= k.z_near) && (xc <= tr * zc + r * mr) && (-xc <= tl * zc + r * ml) &&
            (yc <= tb * zc + r * mb) && (-yc <= tt * zc + r * mt);
    }
    mask[j] = (uint8_t)sel;
    cnt += sel;
  }
  return cnt;
}

/* Canonical FP32 projection decisions for one Gaussian given its float
 * attributes g[14] = mean(3), scale(3), quat(w,x,y,z), opacity, rgb(3).
 * Returns 1 if it survives; fills the tile rectangle [x0,x1) x [y0,y1) and
 * the camera-space depth.  Sequence:
 *   cull unless opacity > 0
 *   (xc, yc, zc) = cam_xform_f(mean); cull unless zc > z_near
 *   rotation from q:  yy=y*y zz=z*z xx=x*x xy=x*y xz=x*z yz=y*z wx=w*x wy=w*y wz=w*z
 *     R00=1-2*(yy+zz) R01=2*(xy-wz) R02=2*(xz+wy)
 *     R10=2*(xy+wz)   R11=1-2*(xx+zz) R12=2*(yz-wx)
 *     R20=2*(xz-wy)   R21=2*(yz+wx)   R22=1-2*(xx+yy)
 *   M_ab = R_ab * s_b;  S_ab = fmaf(M_a0, M_b0, fmaf(M_a1, M_b1, M_a2 * M_b2))
 *   txz = xc / zc clamped to [-lx, lx], lx = jac_clamp * ((0.5 * W) / fx); tx = txz * zc
 *   (same for y with H, fy);  zc2 = zc * zc
 *   J00 = fx / zc, J02 = -((fx * tx) / zc2), J11 = fy / zc, J12 = -((fy * ty) / zc2)
 *   T0c = fmaf(J00, Rc_0c, J02 * Rc_2c),  T1c = fmaf(J11, Rc_1c, J12 * Rc_2c)
 *   u = S T0^T, v = S T1^T (rows with the fmaf chain above)
 *   a = dot(T0, u) + dil, b = dot(T1, u), c = dot(T1, v) + dil
 *   det = a * c - b * b (two products, one subtraction); cull unless det > 0
 *   mid = 0.5 * (a + c); lam = mid + sqrtf(fmaxf(mid * mid - det, 0))
 *   r = ceilf(3 * sqrtf(lam))
 *   px = fmaf(fx, xc / zc, cx), py = fmaf(fy, yc / zc, cy)
 *   x0 = floorf((px - r) * 0.0625), x1 = floorf((px + r) * 0.0625) + 1,
 *   each clamped to [0, tiles_x] by fminf/fmaxf; same for y; cull if empty.
 * dot(p, q) = fmaf(p0, q0, fmaf(p1, q1, p2 * q2)). */
static int project_decide_f(const cam_t *k, const prm_t *pp, const float *g, int tiles_x,
                            int tiles_y, int rect[4], float *depth, float cf[5]) {
  if (!(g[10] > 0.0f)) return 0;
  float xc, yc, zc;
  cam_xform_f(k, g[0], g[1], g[2], &xc, &yc, &zc);
  if (!(zc > k->z_near)) return 0;
  float w = g[6], x = g[7], y = g[8], z = g[9];
  float yy = y * y, zz = z * z, xx = x * x, xy = x * y, xz = x * z, yz = y * z;
  float wx = w * x, wy = w * y, wz = w * z;
  float Rq[9];
  Rq[0] = 1.0f - 2.0f * (yy + zz); Rq[1] = 2.0f * (xy - wz); Rq[2] = 2.0f * (xz + wy);
  Rq[3] = 2.0f * (xy + wz); Rq[4] = 1.0f - 2.0f * (xx + zz); Rq[5] = 2.0f * (yz - wx);
  Rq[6] = 2.0f * (xz - wy); Rq[7] = 2.0f * (yz + wx); Rq[8] = 1.0f - 2.0f * (xx + yy);
  float M[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * g[3 + b];
  float S[9];
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      float v = fmaf(M[3 * a], M[3 * b], fmaf(M[3 * a + 1], M[3 * b + 1], M[3 * a + 2] * M[3 * b + 2]));
      S[3 * a + b] = v; S[3 * b + a] = v;
    }
  float lx = pp->jac_clamp * ((0.5f * (float)k->W) / k->fx);
  float ly = pp->jac_clamp * ((0.5f * (float)k->H) / k->fy);
  float rx = xc / zc, ry = yc / zc;
  float tx = fminf(lx, fmaxf(-lx, rx)) * zc;
  float ty = fminf(ly, fmaxf(-ly, ry)) * zc;
  float zc2 = zc * zc;
  float J00 = k->fx / zc, J02 = -((k->fx * tx) / zc2);
  float J11 = k->fy / zc, J12 = -((k->fy * ty) / zc2);
  const float *Rc = k->R;
  float T0[3], T1[3];
  for (int c = 0; c < 3; ++c) {
    T0[c] = fmaf(J00, Rc[c], J02 * Rc[6 + c]);
    T1[c] = fmaf(J11, Rc[3 + c], J12 * Rc[6 + c]);
  }
  float u[3], v[3];
  for (int a = 0; a < 3; ++a) {
    u[a] = fmaf(S[3 * a], T0[0], fmaf(S[3 * a + 1], T0[1], S[3 * a + 2] * T0[2]));
    v[a] = fmaf(S[3 * a], T1[0], fmaf(S[3 * a + 1], T1[1], S[3 * a + 2] * T1[2]));
  }
  float ca = fmaf(T0[0], u[0], fmaf(T0[1], u[1], T0[2] * u[2])) + pp->dilation;
  float cb = fmaf(T1[0], u[0], fmaf(T1[1], u[1], T1[2] * u[2]));
  float cc = fmaf(T1[0], v[0], fmaf(T1[1], v[1], T1[2] * v[2])) + pp->dilation;
  float det = ca * cc - cb * cb;
  if (!(det > 0.0f)) return 0;
  float mid = 0.5f * (ca + cc);
  float lam = mid + sqrtf(fmaxf(mid * mid - det, 0.0f));
  float r = ceilf(3.0f * sqrtf(lam));
  float px = fmaf(k->fx, rx, k->cx), py = fmaf(k->fy, ry, k->cy);
  float fx0 = floorf((px - r) * 0.0625f), fx1 = floorf((px + r) * 0.0625f) + 1.0f;
  float fy0 = floorf((py - r) * 0.0625f), fy1 = floorf((py + r) * 0.0625f) + 1.0f;
  float tX = (float)tiles_x, tY = (float)tiles_y;
  int x0 = (int)fminf(fmaxf(fx0, 0.0f), tX), x1 = (int)fminf(fmaxf(fx1, 0.0f), tX);
  int y0 = (int)fminf(fmaxf(fy0, 0.0f), tY), y1 = (int)fminf(fmaxf(fy1, 0.0f), tY);
  if (x0 >= x1 || y0 >= y1) return 0;
  rect[0] = x0; rect[1] = y0; rect[2] = x1; rect[3] = y1;
  *depth = zc;
  /* float 2D mean and conic (inverse of (ca cb; cb cc)) for the tile test */
  float inv = 1.0f / det;
  cf[0] = px; cf[1] = py;
  cf[2] = cc * inv; cf[3] = -cb * inv; cf[4] = ca * inv;
  return 1;
}

/* Tile test (canonical FP32): does the 3-sigma ellipse {q(p) <= 9},
 * q(p) = qa dx^2 + 2 qb dx dy + qc dy^2 around the float 2D mean, meet the
 * rectangle spanned by the tile's pixel centres that lie in the W x H image,
 * [16 tx + 0.5, min(16 tx + 15.5, W - 0.5)] x [16 ty + 0.5, min(16 ty + 15.5,
 * H - 0.5)]?  The minimum of the convex quadratic over the rectangle is 0
 * when the mean is inside, else it lies on an edge facing the mean, where
 * the one-dimensional minimiser is clamped to the edge:
 *   X0 = (float)(16 tx) + 0.5, X1 = fminf(X0 + 15, (float)W - 0.5) (Y alike)
 *   if the mean's x is outside [X0, X1]: xe = nearer of X0, X1; dx = xe - mx;
 *     ys = min(max(my - (qb * dx) / qc, Y0), Y1); dy = ys - my;
 *     q1 = fmaf(qa * dx, dx, fmaf(2 * qb * dx, dy, qc * dy * dy))
 *   if the mean's y is outside [Y0, Y1]: ye, dy = ye - my;
 *     xs = min(max(mx - (qb * dy) / qa, X0), X1); dx = xs - mx; q2 = same form
 *   keep iff min(q1, q2) <= 9. */
static int tile_meets_ellipse_f(const float cf[5], int tx, int ty, int W, int H) {
  float mx = cf[0], my = cf[1], qa = cf[2], qb = cf[3], qc = cf[4];
  float X0 = (float)(16 * tx) + 0.5f, X1 = fminf(X0 + 15.0f, (float)W - 0.5f);
  float Y0 = (float)(16 * ty) + 0.5f, Y1 = fminf(Y0 + 15.0f, (float)H - 0.5f);
  int in_x = !(mx < X0) && !(mx > X1), in_y = !(my < Y0) && !(my > Y1);
  if (in_x && in_y) return 1;
  float q = INFINITY;
  if (!in_x) {
    float xe = mx < X0 ? X0 : X1;
    float dx = xe - mx;
    float ys = fminf(fmaxf(my - (qb * dx) / qc, Y0), Y1);
    float dy = ys - my;
    q = fmaf(qa * dx, dx, fmaf(2.0f * qb * dx, dy, qc * dy * dy));
  }
  if (!in_y) {
    float ye = my < Y0 ? Y0 : Y1;
    float dy = ye - my;
    float xs = fminf(fmaxf(mx - (qb * dy) / qa, X0), X1);
    float dx = xs - mx;
    q = fminf(q, fmaf(qa * dx, dx, fmaf(2.0f * qb * dx, dy, qc * dy * dy)));
  }
  return q <= 9.0f;
}

/* ======================================================================
 * Decode (Eq. 3 and Eq. 4), double precision
 * ====================================================================== */

static double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

/* One 2-layer head: out = W2^T relu(W1^T x + b1) + b2; W1 is [in][W],
 * W2 is [W][out], both row-major.  Hidden pre-activations are returned for
 * the backward pass. */
static void head_fwd(const double *x, int in, int Wd, int out, const float *w1,
                     const float *b1, const float *w2, const float *b2, double *hpre,
                     double *y) {
  for (int h = 0; h < Wd; ++h) {
    double s = b1[h];
    for (int i = 0; i < in; ++i) s += x[i] * (double)w1[i * Wd + h];
    hpre[h] = s;
  }
  for (int o = 0; o < out; ++o) {
    double s = b2[o];
    for (int h = 0; h < Wd; ++h) s += (hpre[h] > 0 ? hpre[h] : 0.0) * (double)w2[h * out + o];
    y[o] = s;
  }
}

/* Network input of Eq. 4 for anchor position p seen from camera centre C:
 * [feature (F), |p - C| / d_max, (p - C) / |p - C|]. */
static void decode_input(const float *feat, int F, const float *p, const float *C,
                         double d_max, double *x) {
  double d[3], n2 = 0;
  for (int a = 0; a < 3; ++a) { d[a] = (double)p[a] - (double)C[a]; n2 += d[a] * d[a]; }
  double dist = sqrt(n2);
  for (int i = 0; i < F; ++i) x[i] = feat[i];
  x[F] = dist / d_max;
  for (int a = 0; a < 3; ++a) x[F + 1 + a] = d[a] / dist;
}

/* Decode the selected anchors idx[0..m) into m*k Gaussians, planar
 * out[14][m*k] (double).  Slot s*k + i holds Gaussian i of anchor idx[s]:
 *   mean    = x_v + O_i * l_v                         (Eq. 3)
 *   opacity = tanh(F_alpha(x)_i)                      (Eq. 4; kept iff > 0)
 *   rgb     = sigmoid(F_c(x)_{3i..3i+2})
 *   scale   = base_scale * sigmoid(F_cov(x)_{7i..7i+2})
 *   quat    = F_cov(x)_{7i+3..7i+6} / |.| (identity when the norm is 0)
 * mlp: w1a,b1a,w2a,b2a, w1c,b1c,w2c,b2c, w1s,b1s,w2s,b2s. */
/* Opacity factor of LOD transition blending (Sec. IV-A): the fractional
 * level L* = clamp(log2(d_max / (d s)) + Delta L, 0, K - 1) gives anchors of
 * level L_hat + 1 the factor L* - L_hat; min(1, max(0, L* - L + 1)) is that
 * for them and 1 for every anchor of level <= L_hat. */
static double lod_blend_factor(double dist, double s, float d_max, float bias, int level,
                               int n_levels) {
  double lstar = log2((double)d_max / (dist * s)) + (double)bias;
  if (lstar < 0) lstar = 0;
  if (lstar > n_levels - 1) lstar = n_levels - 1;
  double f = lstar - (double)level + 1.0;
  return f < 0 ? 0 : (f > 1 ? 1 : f);
}

ORC_API double orc_lod_blend_factor(double dist, double s, float d_max, float bias, int level,
                                    int n_levels) {
  return lod_blend_factor(dist, s, d_max, bias, level, n_levels);
}

ORC_API void orc_decode(int64_t m, const int64_t *idx, const float *pos, const float *feat,
                        const float *offsets, const float *offset_scale,
                        const float *base_scale, int k, int F, int Wd,
                        const float *const *mlp, const float *Cw, float d_max,
                        int blend, const uint8_t *level, const float *lod_bias, int n_levels,
                        float s2, double *out) {
  int64_t G = m * k;
  int in = F + 4;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t s = 0; s < m; ++s) {
    int64_t j = idx[s];
    double x[64], hp[256], ya[64], yc[192], ys[448];
    decode_input(feat + j * F, F, pos + 3 * j, Cw, d_max, x);
    head_fwd(x, in, Wd, k, mlp[0], mlp[1], mlp[2], mlp[3], hp, ya);
    head_fwd(x, in, Wd, 3 * k, mlp[4], mlp[5], mlp[6], mlp[7], hp, yc);
    head_fwd(x, in, Wd, 7 * k, mlp[8], mlp[9], mlp[10], mlp[11], hp, ys);
    for (int i = 0; i < k; ++i) {
      int64_t g = s * k + i;
      const float *o = offsets + (j * k + i) * 3;
      for (int a = 0; a < 3; ++a)
        out[a * G + g] = (double)pos[3 * j + a] + (double)o[a] * (double)offset_scale[3 * j + a];
      for (int a = 0; a < 3; ++a)
        out[(3 + a) * G + g] = (double)base_scale[3 * j + a] * sigm(ys[7 * i + a]);
      double q[4], qn = 0;
      for (int a = 0; a < 4; ++a) { q[a] = ys[7 * i + 3 + a]; qn += q[a] * q[a]; }
      qn = sqrt(qn);
      for (int a = 0; a < 4; ++a)
        out[(6 + a) * G + g] = qn > 0 ? q[a] / qn : (a == 0 ? 1.0 : 0.0);
      double op = tanh(ya[i]);
      if (blend) {
        double dv[3];
        for (int a = 0; a < 3; ++a) dv[a] = (double)pos[3 * j + a] - (double)Cw[a];
        double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        op *= lod_blend_factor(dist, sqrt((double)s2), d_max, lod_bias[j], level[j], n_levels);
      }
      out[10 * G + g] = op;
      for (int a = 0; a < 3; ++a) out[(11 + a) * G + g] = sigm(yc[3 * i + a]);
    }
  }
}

/* ======================================================================
 * Projection (EWA local-affine, Sec. III-A) in double, with the canonical
 * FP32 decisions.
 * ====================================================================== */

typedef struct {
  double mx, my;        /* 2D mean, pixels */
  double ca, cb, cc;    /* conic = inverse 2D covariance (a b; b c)^-1 entries */
  double op, rgb[3];
} proj_t;

/* Double-precision continuous projection of one Gaussian (same formulas as
 * the canonical decision sequence, evaluated in double).  Also returns the
 * intermediate 2D covariance (a, b, c) before inversion. */
static void project_cont(const cam_t *k, const prm_t *pp, const double *g, proj_t *o,
                         double cov[3]) {
  double d[3] = {g[0] - k->C[0], g[1] - k->C[1], g[2] - k->C[2]};
  double xc = k->R[0] * d[0] + k->R[1] * d[1] + k->R[2] * d[2];
  double yc = k->R[3] * d[0] + k->R[4] * d[1] + k->R[5] * d[2];
  double zc = k->R[6] * d[0] + k->R[7] * d[1] + k->R[8] * d[2];
  double w = g[6], x = g[7], y = g[8], z = g[9];
  double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                  2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                  2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  double M[9], S[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * g[3 + b];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      S[3 * a + b] = M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];
  double lx = (double)pp->jac_clamp * (0.5 * k->W / (double)k->fx);
  double ly = (double)pp->jac_clamp * (0.5 * k->H / (double)k->fy);
  double rx = xc / zc, ry = yc / zc;
  double tx = fmin(lx, fmax(-lx, rx)) * zc, ty = fmin(ly, fmax(-ly, ry)) * zc;
  double J00 = k->fx / zc, J02 = -k->fx * tx / (zc * zc);
  double J11 = k->fy / zc, J12 = -k->fy * ty / (zc * zc);
  double T0[3], T1[3];
  for (int c = 0; c < 3; ++c) {
    T0[c] = J00 * k->R[c] + J02 * k->R[6 + c];
    T1[c] = J11 * k->R[3 + c] + J12 * k->R[6 + c];
  }
  double a = 0, b = 0, c = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      a += T0[i] * S[3 * i + j] * T0[j];
      b += T1[i] * S[3 * i + j] * T0[j];
      c += T1[i] * S[3 * i + j] * T1[j];
    }
  a += pp->dilation; c += pp->dilation;
  cov[0] = a; cov[1] = b; cov[2] = c;
  double det = a * c - b * b;
  o->mx = k->fx * rx + k->cx;
  o->my = k->fy * ry + k->cy;
  o->ca = c / det; o->cb = -b / det; o->cc = a / det;
  o->op = g[10];
  o->rgb[0] = g[11]; o->rgb[1] = g[12]; o->rgb[2] = g[13];
}

/* Project n Gaussians given planar float attributes gf[14][stride] (the
 * values the decisions are taken on) and optionally double attributes
 * gd[14][stride] for the continuous part (NULL: use the float values).
 * Outputs per Gaussian: vis (0/1), rect[4] (x0,y0,x1,y1), depth (float
 * canonical camera z), and proj[9] = mx, my, ca, cb, cc, op, r, g, b in
 * double.  Returns the number of visible Gaussians. */
ORC_API int64_t orc_project(int64_t n, int64_t stride, const float *gf, const double *gd,
                            const float *camf, int W, int H, const float *prmf,
                            uint8_t *vis, int32_t *rect, float *depth, double *proj, float *cf) {
  cam_t k = load_cam(camf, W, H);
  prm_t pp = load_prm(prmf);
  int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
  int64_t cnt = 0;
#pragma omp parallel for reduction(+ : cnt) schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    float g[14];
    double gdd[14];
    for (int f = 0; f < 14; ++f) {
      g[f] = gf[f * stride + i];
      gdd[f] = gd ? gd[f * stride + i] : (double)g[f];
    }
    int r[4] = {0, 0, 0, 0};
    float dz = 0;
    float c5[5] = {0, 0, 0, 0, 0};
    int v = project_decide_f(&k, &pp, g, tiles_x, tiles_y, r, &dz, c5);
    for (int a = 0; a < 5; ++a) cf[5 * i + a] = c5[a];
    vis[i] = (uint8_t)v;
    for (int a = 0; a < 4; ++a) rect[4 * i + a] = r[a];
    depth[i] = dz;
    proj_t o;
    double cov[3];
    memset(&o, 0, sizeof o);
    if (v) project_cont(&k, &pp, gdd, &o, cov);
    double *p = proj + 9 * i;
    p[0] = o.mx; p[1] = o.my; p[2] = o.ca; p[3] = o.cb; p[4] = o.cc;
    p[5] = o.op; p[6] = o.rgb[0]; p[7] = o.rgb[1]; p[8] = o.rgb[2];
    cnt += v;
  }
  return cnt;
}

/* ======================================================================
 * Decisions near their thresholds
 *
 * The HIP path decodes in FP32, so its decoded attributes differ from the
 * oracle's FP64 ones by up to a known per-attribute bound, and its discrete
 * decisions (the culls, the tile rectangle, the tile test, the depth order)
 * are taken on those slightly different values.  A decision whose
 * continuous quantity lies within that bound (propagated to first order,
 * times 1.5) plus an FP32 evaluation slack of its threshold may legitimately
 * come out either way.  These functions flag such Gaussians, so that a
 * parity test can ask for bit-exact lists and images everywhere else.
 * ====================================================================== */

/* Continuous quantities behind the canonical decisions of one Gaussian, in
 * double, in the order of project_decide_f: v[0] opacity, v[1] zc,
 * v[2] det of the dilated 2D covariance, v[3] 3 sqrt(lambda_max),
 * v[4] px, v[5] py, v[6..8] conic (qa, qb, qc), v[9] |a c| + b^2. */
enum { DQ_OP, DQ_Z, DQ_DET, DQ_R3, DQ_PX, DQ_PY, DQ_QA, DQ_QB, DQ_QC, DQ_DETSCALE, DQ_N };

static void decision_values(const cam_t *k, const prm_t *pp, const double *g, double *v) {
  double d[3] = {g[0] - k->C[0], g[1] - k->C[1], g[2] - k->C[2]};
  double xc = k->R[0] * d[0] + k->R[1] * d[1] + k->R[2] * d[2];
  double yc = k->R[3] * d[0] + k->R[4] * d[1] + k->R[5] * d[2];
  double zc = k->R[6] * d[0] + k->R[7] * d[1] + k->R[8] * d[2];
  v[DQ_OP] = g[10];
  v[DQ_Z] = zc;
  double zs = zc > 1e-30 ? zc : 1e-30;
  /* the decoded quaternion is unit; a perturbed one is taken back to unit
   * length, so that its change is a rotation */
  double qn = sqrt(g[6] * g[6] + g[7] * g[7] + g[8] * g[8] + g[9] * g[9]);
  if (!(qn > 0)) qn = 1;
  double w = g[6] / qn, x = g[7] / qn, y = g[8] / qn, z = g[9] / qn;
  double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                  2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                  2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  double M[9], S[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * g[3 + b];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      S[3 * a + b] = M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];
  double lx = (double)pp->jac_clamp * (0.5 * k->W / (double)k->fx);
  double ly = (double)pp->jac_clamp * (0.5 * k->H / (double)k->fy);
  double rx = xc / zs, ry = yc / zs;
  double tx = fmin(lx, fmax(-lx, rx)) * zs, ty = fmin(ly, fmax(-ly, ry)) * zs;
  double J00 = k->fx / zs, J02 = -k->fx * tx / (zs * zs);
  double J11 = k->fy / zs, J12 = -k->fy * ty / (zs * zs);
  double T0[3], T1[3];
  for (int c = 0; c < 3; ++c) {
    T0[c] = J00 * k->R[c] + J02 * k->R[6 + c];
    T1[c] = J11 * k->R[3 + c] + J12 * k->R[6 + c];
  }
  double a = 0, b = 0, c = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      a += T0[i] * S[3 * i + j] * T0[j];
      b += T1[i] * S[3 * i + j] * T0[j];
      c += T1[i] * S[3 * i + j] * T1[j];
    }
  a += pp->dilation;
  c += pp->dilation;
  double det = a * c - b * b;
  double mid = 0.5 * (a + c);
  double lam = mid + sqrt(fmax(mid * mid - det, 0.0));
  v[DQ_DET] = det;
  v[DQ_R3] = 3.0 * sqrt(fmax(lam, 0.0));
  v[DQ_PX] = k->fx * rx + k->cx;
  v[DQ_PY] = k->fy * ry + k->cy;
  double dd = det != 0 ? det : 1e-300;
  v[DQ_QA] = c / dd;
  v[DQ_QB] = -b / dd;
  v[DQ_QC] = a / dd;
  v[DQ_DETSCALE] = fabs(a * c) + b * b;
}

/* Minimum of q = qa dx^2 + 2 qb dx dy + qc dy^2 over the box of tile
 * (tx, ty)'s pixel centres inside the image, in double (0 with the mean
 * inside); also the sum of the magnitudes of its three terms there. */
static double tile_qmin_d(double mx, double my, double qa, double qb, double qc, int tx, int ty,
                          int W, int H, double *scale) {
  double X0 = 16.0 * tx + 0.5, X1 = fmin(X0 + 15.0, W - 0.5);
  double Y0 = 16.0 * ty + 0.5, Y1 = fmin(Y0 + 15.0, H - 0.5);
  int in_x = mx >= X0 && mx <= X1, in_y = my >= Y0 && my <= Y1;
  *scale = 0;
  if (in_x && in_y) return 0.0;
  double q = INFINITY;
  if (!in_x) {
    double dx = (mx < X0 ? X0 : X1) - mx;
    double ys = fmin(fmax(my - qb * dx / qc, Y0), Y1), dy = ys - my;
    q = qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy;
    *scale = fabs(qa * dx * dx) + fabs(2 * qb * dx * dy) + fabs(qc * dy * dy);
  }
  if (!in_y) {
    double dy = (my < Y0 ? Y0 : Y1) - my;
    double xs = fmin(fmax(mx - qb * dy / qa, X0), X1), dx = xs - mx;
    double q2 = qa * dx * dx + 2 * qb * dx * dy + qc * dy * dy;
    if (q2 < q) {
      q = q2;
      *scale = fabs(qa * dx * dx) + fabs(2 * qb * dx * dy) + fabs(qc * dy * dy);
    }
  }
  return q;
}

static int near_integer(double v, double m) { return fabs(v - nearbyint(v)) <= m; }

/* Marks tile t of the W x H image (tx, ty in range) in the tile mask. */
static void mark_tile(uint8_t *tmask, int tiles_x, int tiles_y, int tx, int ty) {
  if (tx < 0 || ty < 0 || tx >= tiles_x || ty >= tiles_y) return;
#pragma omp atomic write
  tmask[(size_t)ty * tiles_x + tx] = 1;
}

/* Near-threshold decisions of Gaussians with planar double attributes
 * gd[14][stride], each within eb[14][stride] of what the HIP path decodes;
 * vis / rect are the oracle's canonical projection of the same Gaussians.
 * For each Gaussian, the quantities behind its decisions are evaluated in
 * double and their change under eb is propagated to first order (one
 * perturbation of +-eb per attribute, the changes added, times 1.5); a
 * decision is near its threshold when the quantity lies within that change
 * plus slack (relative FP32 evaluation slack) of it.  Tiles whose list or
 * pixels such a decision can change are marked in tmask [tiles_y][tiles_x]:
 *   bit 0 (flags): a whole-Gaussian cull (opacity > 0, zc > z_near,
 *          det > 0) is near its threshold: every tile of the 3-sigma
 *          square, one tile wider on each side, is marked;
 *   bit 1: the tile test of a tile of the rectangle is near q = 9: that tile;
 *   bit 3: the rectangle (ceil of 3 sqrt(lambda), floor of (p -+ r) / 16) is
 *          near a threshold: the tiles on its border, one tile either way,
 *          where the tile test does not reject the Gaussian with margin.
 * zdepth[i], zmargin[i]: camera depth and its margin, for the depth-order
 * check the caller makes over the visible Gaussians (the depth is one
 * canonical FP32 sequence on the mean, which both sides form with one
 * rounding of x_v + O l, so its margin comes from the mean's bound alone).
 * Returns the number of flagged Gaussians. */
ORC_API int64_t orc_fragile(int64_t n, int64_t stride, const double *gd, const double *eb,
                            const float *camf, int W, int H, const float *prmf,
                            const uint8_t *vis, const int32_t *rect, double slack,
                            uint8_t *flags, double *zdepth, double *zmargin, uint8_t *tmask) {
  cam_t k = load_cam(camf, W, H);
  prm_t pp = load_prm(prmf);
  const int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
  int64_t cnt = 0;
#pragma omp parallel for reduction(+ : cnt) schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    double g[14], v0[DQ_N], e[DQ_N] = {0};
    for (int f = 0; f < 14; ++f) g[f] = gd[f * stride + i];
    decision_values(&k, &pp, g, v0);
    for (int f = 0; f < 11; ++f) {  /* colour takes no decision */
      double h = eb[f * stride + i];
      if (!(h > 0)) continue;
      double best[DQ_N] = {0};
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        double gp[14], v[DQ_N];
        memcpy(gp, g, sizeof gp);
        gp[f] += sgn * h;
        decision_values(&k, &pp, gp, v);
        for (int q = 0; q < DQ_N; ++q) best[q] = fmax(best[q], fabs(v[q] - v0[q]));
      }
      for (int q = 0; q < DQ_N; ++q) e[q] += best[q];
    }
    /* first order, with half again for the second-order terms */
    for (int q = 0; q < DQ_N; ++q) e[q] *= 1.5;
    uint8_t fl = 0;
    const double r3 = v0[DQ_R3], r = ceil(r3), px = v0[DQ_PX], py = v0[DQ_PY];
    const double in5[5] = {px, py, v0[DQ_QA], v0[DQ_QB], v0[DQ_QC]};
    const double e5[5] = {e[DQ_PX], e[DQ_PY], e[DQ_QA], e[DQ_QB], e[DQ_QC]};
    /* q_min of tile (tx, ty) and its margin */
#define QMIN_MARGIN(tx, ty, q0, mq)                                                          \
    do {                                                                                       \
      double sc0_, eq_ = 0;                                                                    \
      q0 = tile_qmin_d(in5[0], in5[1], in5[2], in5[3], in5[4], tx, ty, W, H, &sc0_);           \
      for (int a_ = 0; a_ < 5; ++a_) {                                                         \
        double b_ = 0;                                                                         \
        for (int s_ = -1; s_ <= 1; s_ += 2) {                                                  \
          double p_[5], sc1_;                                                                  \
          memcpy(p_, in5, sizeof p_);                                                          \
          p_[a_] += s_ * e5[a_];                                                               \
          b_ = fmax(b_, fabs(tile_qmin_d(p_[0], p_[1], p_[2], p_[3], p_[4], tx, ty, W, H,      \
                                         &sc1_) - q0));                                        \
        }                                                                                      \
        eq_ += b_;                                                                             \
      }                                                                                        \
      mq = eq_ + slack * (9.0 + sc0_);                                                         \
    } while (0)
    const int cull_near =
        fabs(v0[DQ_OP]) <= e[DQ_OP] + slack * 1e-2 ||
        fabs(v0[DQ_Z] - k.z_near) <= e[DQ_Z] + slack * fabs(v0[DQ_Z]) ||
        fabs(v0[DQ_DET]) <= e[DQ_DET] + slack * v0[DQ_DETSCALE];
    if (cull_near) {
      fl |= 1;
      if (isfinite(px) && isfinite(py) && isfinite(r)) {
        int x0 = (int)fmax(floor((px - r) / 16.0) - 1, -1), x1 = (int)fmin(floor((px + r) / 16.0) + 1, tiles_x);
        int y0 = (int)fmax(floor((py - r) / 16.0) - 1, -1), y1 = (int)fmin(floor((py + r) / 16.0) + 1, tiles_y);
        for (int ty = y0; ty <= y1; ++ty)
          for (int tx = x0; tx <= x1; ++tx) mark_tile(tmask, tiles_x, tiles_y, tx, ty);
      } else {
        for (int t = 0; t < tiles_x * tiles_y; ++t) mark_tile(tmask, tiles_x, tiles_y, t % tiles_x, t / tiles_x);
      }
    } else if (v0[DQ_Z] > k.z_near && v0[DQ_DET] > 0 && v0[DQ_OP] > 0) {
      /* the rectangle: the possible radii ceil(3 sqrt(lambda) -+ margin) and
       * 2D means give a range for each edge x0 = floor((px - r) / 16),
       * x1 = floor((px + r) / 16) + 1 (rows alike); the columns (rows)
       * between an edge's extremes are candidates on one side only.  Such a
       * tile changes the list only where the tile test may keep the
       * Gaussian. */
      const double mr = e[DQ_R3] + slack * r3;
      const double rlo = ceil(r3 - mr), rhi = ceil(r3 + mr);
      const double ex = e[DQ_PX] + slack * (fabs(px) + rhi), ey = e[DQ_PY] + slack * (fabs(py) + rhi);
      const int x0a = (int)floor((px - ex - rhi) / 16.0), x0b = (int)floor((px + ex - rlo) / 16.0);
      const int x1a = (int)floor((px - ex + rlo) / 16.0) + 1, x1b = (int)floor((px + ex + rhi) / 16.0) + 1;
      const int y0a = (int)floor((py - ey - rhi) / 16.0), y0b = (int)floor((py + ey - rlo) / 16.0);
      const int y1a = (int)floor((py - ey + rlo) / 16.0) + 1, y1b = (int)floor((py + ey + rhi) / 16.0) + 1;
      if (x0a != x0b || x1a != x1b || y0a != y0b || y1a != y1b) {
        for (int ty = (y0a > 0 ? y0a : 0); ty < y1b && ty < tiles_y; ++ty)
          for (int tx = (x0a > 0 ? x0a : 0); tx < x1b && tx < tiles_x; ++tx) {
            const int sure = tx >= x0b && tx < x1a && ty >= y0b && ty < y1a;
            if (sure) continue;  /* a candidate whichever way the edges go */
            double q0, mq;
            QMIN_MARGIN(tx, ty, q0, mq);
            if (q0 <= 9.0 + mq) {
              fl |= 8;
              mark_tile(tmask, tiles_x, tiles_y, tx, ty);
            }
          }
      }
      if (vis[i]) {
        const int32_t *rc = rect + 4 * i;
        for (int ty = rc[1]; ty < rc[3]; ++ty)
          for (int tx = rc[0]; tx < rc[2]; ++tx) {
            double q0, mq;
            QMIN_MARGIN(tx, ty, q0, mq);
            if (fabs(q0 - 9.0) <= mq) {
              fl |= 2;
              mark_tile(tmask, tiles_x, tiles_y, tx, ty);
            }
          }
      }
    }
#undef QMIN_MARGIN
    flags[i] = fl;
    zdepth[i] = v0[DQ_Z];
    zmargin[i] = e[DQ_Z];
    cnt += fl != 0;
  }
  return cnt;
}

/* ======================================================================
 * Tile binning and depth ordering
 * ====================================================================== */

typedef struct {
  uint32_t tile, dkey, gid;
} pair_t;

static int pair_cmp(const void *a, const void *b) {
  const pair_t *p = a, *q = b;
  if (p->tile != q->tile) return p->tile < q->tile ? -1 : 1;
  if (p->dkey != q->dkey) return p->dkey < q->dkey ? -1 : 1;
  if (p->gid != q->gid) return p->gid < q->gid ? -1 : 1;
  return 0;
}

static uint32_t fbits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

/* Count the (tile, Gaussian) pairs: tiles of each visible Gaussian's
 * rectangle that its 3-sigma ellipse meets. */
ORC_API int64_t orc_count_pairs(int64_t n, const uint8_t *vis, const int32_t *rect,
                                const float *cf, int W, int H) {
  int64_t p = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!vis[i]) continue;
    const int32_t *r = rect + 4 * i;
    for (int y = r[1]; y < r[3]; ++y)
      for (int x = r[0]; x < r[2]; ++x) p += tile_meets_ellipse_f(cf + 5 * i, x, y, W, H);
  }
  return p;
}

/* Rectangle candidates (before the ellipse test). */
ORC_API int64_t orc_count_rect_pairs(int64_t n, const uint8_t *vis, const int32_t *rect) {
  int64_t p = 0;
  for (int64_t i = 0; i < n; ++i)
    if (vis[i]) p += (int64_t)(rect[4 * i + 2] - rect[4 * i]) * (rect[4 * i + 3] - rect[4 * i + 1]);
  return p;
}

ORC_API int orc_tile_test(const float *cf, int tx, int ty, int W, int H) {
  return tile_meets_ellipse_f(cf, tx, ty, W, H);
}

/* All (tile, Gaussian) pairs (tiles of the rectangle that the 3-sigma
 * ellipse meets) ordered by tile, then depth (positive float bits order like
 * the values), then Gaussian index; ranges[t] = [start, end) of tile t in
 * that list.  Writes tile_of[P], gid_of[P]. */
ORC_API int64_t orc_bin_sort(int64_t n, const uint8_t *vis, const int32_t *rect,
                             const float *cf, const float *depth, int W, int H, uint32_t *tile_of,
                             uint32_t *gid_of, uint32_t *ranges) {
  int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
  int64_t P = orc_count_pairs(n, vis, rect, cf, W, H);
  pair_t *pr = (pair_t *)malloc(sizeof(pair_t) * (size_t)(P > 0 ? P : 1));
  int64_t q = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!vis[i]) continue;
    const int32_t *r = rect + 4 * i;
    for (int y = r[1]; y < r[3]; ++y)
      for (int x = r[0]; x < r[2]; ++x) {
        if (!tile_meets_ellipse_f(cf + 5 * i, x, y, W, H)) continue;
        pr[q].tile = (uint32_t)(y * tiles_x + x);
        pr[q].dkey = fbits(depth[i]);
        pr[q].gid = (uint32_t)i;
        ++q;
      }
  }
  qsort(pr, (size_t)P, sizeof(pair_t), pair_cmp);
  int ntiles = tiles_x * tiles_y;
  for (int t = 0; t < ntiles; ++t) { ranges[2 * t] = 0; ranges[2 * t + 1] = 0; }
  for (int64_t i = 0; i < P; ++i) {
    tile_of[i] = pr[i].tile;
    gid_of[i] = pr[i].gid;
    if (i == 0 || pr[i].tile != pr[i - 1].tile) ranges[2 * pr[i].tile] = (uint32_t)i;
    if (i == P - 1 || pr[i].tile != pr[i + 1].tile) ranges[2 * pr[i].tile + 1] = (uint32_t)(i + 1);
  }
  free(pr);
  return P;
}

/* ======================================================================
 * Compositing (Eq. 2), double precision
 * ====================================================================== */

/* Blend one pixel over an ordered Gaussian list (Eq. 2):
 *   a_i = min(alpha_max, op_i * exp(-0.5 (ca dx^2 + cc dy^2) - cb dx dy)),
 *   dx = pixel_x - mx_i (pixel centres at integer + 0.5),
 *   skip if a_i < alpha_min; C += T a_i c_i; T *= (1 - a_i);
 *   stop after the Gaussian that takes T below t_min.
 * Returns the count of list entries consumed; optional per-Gaussian blend
 * weight accumulation w[gid] += a_i T_i. */
static int blend_pixel(const prm_t *pp, const double *proj, const uint32_t *list, int n,
                       double px, double py, double out[3], double *T_out, double *w) {
  double T = 1.0, C[3] = {0, 0, 0};
  int last = 0;
  for (int i = 0; i < n; ++i) {
    const double *p = proj + 9 * (size_t)list[i];
    double dx = px - p[0], dy = py - p[1];
    double pw = -0.5 * (p[2] * dx * dx + p[4] * dy * dy) - p[3] * dx * dy;
    double a = p[5] * exp(pw);
    if (a > pp->alpha_max) a = pp->alpha_max;
    last = i + 1;
    if (a < pp->alpha_min) continue;
    double wt = a * T;
    for (int c = 0; c < 3; ++c) C[c] += wt * p[6 + c];
    if (w) {
#pragma omp atomic
      w[list[i]] += wt;
    }
    T *= (1.0 - a);
    if (T < pp->t_min) break;
  }
  for (int c = 0; c < 3; ++c) out[c] = C[c] + T * pp->bg[c];
  *T_out = T;
  return last;
}

/* Tiled renderer: for each 16x16 tile, blend its pixels over the tile's
 * range of the sorted pair list.  img is planar [3][H][W]; Tf [H][W];
 * last [H][W] = entries of the tile list consumed by that pixel; w (nullable)
 * accumulates per-Gaussian blend weights. */
ORC_API void orc_composite(const uint32_t *gid_of, const uint32_t *ranges, const double *proj,
                           int W, int H, const float *prmf, double *img, double *Tf,
                           int32_t *last, double *w) {
  prm_t pp = load_prm(prmf);
  int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < tiles_x * tiles_y; ++t) {
    int tx = t % tiles_x, ty = t / tiles_x;
    uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
    for (int yy = 0; yy < 16; ++yy)
      for (int xx = 0; xx < 16; ++xx) {
        int x = tx * 16 + xx, y = ty * 16 + yy;
        if (x >= W || y >= H) continue;
        double c[3], T;
        int l = blend_pixel(&pp, proj, gid_of + s, (int)(e - s), x + 0.5, y + 0.5, c, &T, w);
        size_t pix = (size_t)y * W + x;
        for (int a = 0; a < 3; ++a) img[(size_t)a * W * H + pix] = c[a];
        Tf[pix] = T;
        last[pix] = l;
      }
  }
}

typedef struct {
  uint32_t dkey, gid;
} dk_t;

static int dk_cmp(const void *a, const void *b) {
  const dk_t *p = a, *q = b;
  if (p->dkey != q->dkey) return p->dkey < q->dkey ? -1 : 1;
  return p->gid < q->gid ? -1 : (p->gid > q->gid);
}

/* Brute-force renderer: for every pixel, scan all Gaussians, keep those
 * whose 3-sigma ellipse meets the pixel's tile (inside its rectangle), order
 * them by (depth, index) and blend.  No pair list, no global sort. */
ORC_API void orc_render_bruteforce(int64_t n, const uint8_t *vis, const int32_t *rect,
                                   const float *cf, const float *depth, const double *proj, int W,
                                   int H, const float *prmf, double *img, double *Tf) {
  prm_t pp = load_prm(prmf);
#pragma omp parallel for schedule(dynamic, 1)
  for (int y = 0; y < H; ++y) {
    dk_t *buf = (dk_t *)malloc(sizeof(dk_t) * (size_t)(n > 0 ? n : 1));
    uint32_t *lst = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    for (int x = 0; x < W; ++x) {
      int tx = x / 16, ty = y / 16, m = 0;
      for (int64_t i = 0; i < n; ++i) {
        const int32_t *r = rect + 4 * i;
        if (vis[i] && tx >= r[0] && tx < r[2] && ty >= r[1] && ty < r[3] &&
            tile_meets_ellipse_f(cf + 5 * i, tx, ty, W, H)) {
          buf[m].dkey = fbits(depth[i]);
          buf[m].gid = (uint32_t)i;
          ++m;
        }
      }
      qsort(buf, (size_t)m, sizeof(dk_t), dk_cmp);
      for (int i = 0; i < m; ++i) lst[i] = buf[i].gid;
      double c[3], T;
      blend_pixel(&pp, proj, lst, m, x + 0.5, y + 0.5, c, &T, NULL);
      size_t pix = (size_t)y * W + x;
      for (int a = 0; a < 3; ++a) img[(size_t)a * W * H + pix] = c[a];
      Tf[pix] = T;
    }
    free(buf);
    free(lst);
  }
}

ORC_API int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel regions that follow (timing on fewer cores). */
ORC_API void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ======================================================================
 * Backward passes (double precision), for the training step of Sec. V
 * (losses on rendered images) and the gradient checks.
 * ====================================================================== */

/* Compositing backward.  For each pixel the forward blend over its tile list
 * is replayed (a_i, T_i), then walked in reverse:
 *   dL/dc_i = a_i T_i dL/dC
 *   dL/da_i = T_i (c_i . dL/dC) - (B_i . dL/dC) / (1 - a_i),
 *     B_i = sum_{j>i} a_j T_j c_j + T_final bg  (colour behind entry i)
 *   a_i = min(alpha_max, op_i G_i): no gradient to op_i or G_i when clamped
 *   G_i = exp(p_i), p_i = -0.5 (ca dx^2 + cc dy^2) - cb dx dy, dx = px - mx.
 * dproj[9 * g + .] accumulates dmx, dmy, dca, dcb, dcc, dop, dr, dg, db. */
ORC_API void orc_composite_backward(const uint32_t *gid_of, const uint32_t *ranges,
                                    const double *proj, int W, int H, const float *prmf,
                                    const double *dimg, double *dproj) {
  prm_t pp = load_prm(prmf);
  int tiles_x = (W + 15) / 16, tiles_y = (H + 15) / 16;
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < tiles_x * tiles_y; ++t) {
    int tx = t % tiles_x, ty = t / tiles_x;
    uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
    int n = (int)(e - s);
    double *aa = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *TT = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int yy = 0; yy < 16; ++yy)
      for (int xx = 0; xx < 16; ++xx) {
        int x = tx * 16 + xx, y = ty * 16 + yy;
        if (x >= W || y >= H) continue;
        double px = x + 0.5, py = y + 0.5;
        size_t pix = (size_t)y * W + x;
        double dC[3];
        for (int c = 0; c < 3; ++c) dC[c] = dimg[(size_t)c * W * H + pix];
        /* forward replay */
        double T = 1.0;
        int last = 0;
        for (int i = 0; i < n; ++i) {
          const double *p = proj + 9 * (size_t)gid_of[s + i];
          double dx = px - p[0], dy = py - p[1];
          double pw = -0.5 * (p[2] * dx * dx + p[4] * dy * dy) - p[3] * dx * dy;
          double a = p[5] * exp(pw);
          if (a > pp.alpha_max) a = pp.alpha_max;
          last = i + 1;
          if (a < pp.alpha_min) { aa[i] = -1; TT[i] = T; continue; }
          aa[i] = a;
          TT[i] = T;
          T *= (1.0 - a);
          if (T < pp.t_min) break;
        }
        /* reverse walk */
        double B[3];
        for (int c = 0; c < 3; ++c) B[c] = T * pp.bg[c];
        for (int i = last - 1; i >= 0; --i) {
          if (aa[i] < 0) continue;
          uint32_t g = gid_of[s + i];
          const double *p = proj + 9 * (size_t)g;
          double a = aa[i], Ti = TT[i], w = a * Ti;
          double cdot = 0, bdot = 0;
          for (int c = 0; c < 3; ++c) { cdot += p[6 + c] * dC[c]; bdot += B[c] * dC[c]; }
          double dLda = Ti * cdot - bdot / (1.0 - a);
          double dx = px - p[0], dy = py - p[1];
          double pw = -0.5 * (p[2] * dx * dx + p[4] * dy * dy) - p[3] * dx * dy;
          double G = exp(pw);
          double d[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
          for (int c = 0; c < 3; ++c) d[6 + c] = w * dC[c];
          if (p[5] * G <= pp.alpha_max) {
            double dG = dLda * p[5];
            d[5] = dLda * G;
            double dpw = dG * G;
            d[2] = dpw * (-0.5 * dx * dx);
            d[4] = dpw * (-0.5 * dy * dy);
            d[3] = dpw * (-dx * dy);
            /* dp/dmx = ca dx + cb dy, dp/dmy = cb dx + cc dy */
            d[0] = dpw * (p[2] * dx + p[3] * dy);
            d[1] = dpw * (p[3] * dx + p[4] * dy);
          }
          for (int c = 0; c < 3; ++c) B[c] += w * p[6 + c];
          for (int q = 0; q < 9; ++q) {
#pragma omp atomic
            dproj[9 * (size_t)g + q] += d[q];
          }
        }
      }
    free(aa);
    free(TT);
  }
}

/* Projection backward for one Gaussian with double attributes g[14] (the
 * forward of project_cont), from dL/d(mx, my, ca, cb, cc, op, r, g, b) to
 * dL/d(mean, scale, quat, opacity, rgb).  The inverse 2x2 covariance
 * Q = Sigma2D^-1 has dL/dSigma2D = -Q Gq Q with Gq the gradient with respect
 * to the symmetric conic (off-diagonal counted on both entries). */
static void project_bwd_one(const cam_t *k, const prm_t *pp, const double *g, const double *dp,
                            double *dg) {
  double d[3] = {g[0] - k->C[0], g[1] - k->C[1], g[2] - k->C[2]};
  const float *R = k->R;
  double xc = R[0] * d[0] + R[1] * d[1] + R[2] * d[2];
  double yc = R[3] * d[0] + R[4] * d[1] + R[5] * d[2];
  double zc = R[6] * d[0] + R[7] * d[1] + R[8] * d[2];
  double w = g[6], x = g[7], y = g[8], z = g[9];
  double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                  2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                  2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  double M[9], S[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) M[3 * a + b] = Rq[3 * a + b] * g[3 + b];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      S[3 * a + b] = M[3 * a] * M[3 * b] + M[3 * a + 1] * M[3 * b + 1] + M[3 * a + 2] * M[3 * b + 2];
  double lx = (double)pp->jac_clamp * (0.5 * k->W / (double)k->fx);
  double ly = (double)pp->jac_clamp * (0.5 * k->H / (double)k->fy);
  double rx = xc / zc, ry = yc / zc;
  int clx = (rx > lx || rx < -lx), cly = (ry > ly || ry < -ly);
  double txz = fmin(lx, fmax(-lx, rx)), tyz = fmin(ly, fmax(-ly, ry));
  double tx = txz * zc, ty = tyz * zc;
  double fx = k->fx, fy = k->fy;
  double J00 = fx / zc, J02 = -fx * tx / (zc * zc);
  double J11 = fy / zc, J12 = -fy * ty / (zc * zc);
  double T0[3], T1[3];
  for (int c = 0; c < 3; ++c) {
    T0[c] = J00 * R[c] + J02 * R[6 + c];
    T1[c] = J11 * R[3 + c] + J12 * R[6 + c];
  }
  double ST0[3], ST1[3];
  for (int i = 0; i < 3; ++i) {
    ST0[i] = S[3 * i] * T0[0] + S[3 * i + 1] * T0[1] + S[3 * i + 2] * T0[2];
    ST1[i] = S[3 * i] * T1[0] + S[3 * i + 1] * T1[1] + S[3 * i + 2] * T1[2];
  }
  double a = T0[0] * ST0[0] + T0[1] * ST0[1] + T0[2] * ST0[2] + pp->dilation;
  double b = T1[0] * ST0[0] + T1[1] * ST0[1] + T1[2] * ST0[2];
  double c = T1[0] * ST1[0] + T1[1] * ST1[1] + T1[2] * ST1[2] + pp->dilation;
  double det = a * c - b * b;
  double Q[4] = {c / det, -b / det, -b / det, a / det};
  double Gq[4] = {dp[2], 0.5 * dp[3], 0.5 * dp[3], dp[4]};
  /* H = -Q Gq Q */
  double QG[4] = {Q[0] * Gq[0] + Q[1] * Gq[2], Q[0] * Gq[1] + Q[1] * Gq[3],
                  Q[2] * Gq[0] + Q[3] * Gq[2], Q[2] * Gq[1] + Q[3] * Gq[3]};
  double Hm[4] = {-(QG[0] * Q[0] + QG[1] * Q[2]), -(QG[0] * Q[1] + QG[1] * Q[3]),
                  -(QG[2] * Q[0] + QG[3] * Q[2]), -(QG[2] * Q[1] + QG[3] * Q[3])};
  double da = Hm[0], db = Hm[1] + Hm[2], dc = Hm[3];
  /* a = T0 S T0, b = T1 S T0, c = T1 S T1 */
  double GS[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      GS[3 * i + j] = da * T0[i] * T0[j] + db * T1[i] * T0[j] + dc * T1[i] * T1[j];
  double dT0[3], dT1[3];
  for (int i = 0; i < 3; ++i) {
    dT0[i] = 2 * da * ST0[i] + db * ST1[i];
    dT1[i] = db * ST0[i] + 2 * dc * ST1[i];
  }
  /* M: S = M M^T, dM = (GS + GS^T) M */
  double dM[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int l = 0; l < 3; ++l) s += (GS[3 * i + l] + GS[3 * l + i]) * M[3 * l + j];
      dM[3 * i + j] = s;
    }
  double ds[3] = {0, 0, 0}, dR[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      ds[j] += dM[3 * i + j] * Rq[3 * i + j];
      dR[3 * i + j] = dM[3 * i + j] * g[3 + j];
    }
  double dw = 0, dx = 0, dy = 0, dz = 0;
  dy += -4 * y * dR[0]; dz += -4 * z * dR[0];
  dx += 2 * y * dR[1]; dy += 2 * x * dR[1]; dw += -2 * z * dR[1]; dz += -2 * w * dR[1];
  dx += 2 * z * dR[2]; dz += 2 * x * dR[2]; dw += 2 * y * dR[2]; dy += 2 * w * dR[2];
  dx += 2 * y * dR[3]; dy += 2 * x * dR[3]; dw += 2 * z * dR[3]; dz += 2 * w * dR[3];
  dx += -4 * x * dR[4]; dz += -4 * z * dR[4];
  dy += 2 * z * dR[5]; dz += 2 * y * dR[5]; dw += -2 * x * dR[5]; dx += -2 * w * dR[5];
  dx += 2 * z * dR[6]; dz += 2 * x * dR[6]; dw += -2 * y * dR[6]; dy += -2 * w * dR[6];
  dy += 2 * z * dR[7]; dz += 2 * y * dR[7]; dw += 2 * x * dR[7]; dx += 2 * w * dR[7];
  dx += -4 * x * dR[8]; dy += -4 * y * dR[8];
  /* T0 = J00 R0 + J02 R2, T1 = J11 R1 + J12 R2 */
  double dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
  for (int i = 0; i < 3; ++i) {
    dJ00 += dT0[i] * R[i];
    dJ02 += dT0[i] * R[6 + i];
    dJ11 += dT1[i] * R[3 + i];
    dJ12 += dT1[i] * R[6 + i];
  }
  double dxc = 0, dyc = 0, dzc = 0;
  dzc += dJ00 * (-fx / (zc * zc));
  dzc += dJ11 * (-fy / (zc * zc));
  double dtx = dJ02 * (-fx / (zc * zc)), dty = dJ12 * (-fy / (zc * zc));
  dzc += dJ02 * (2 * fx * tx / (zc * zc * zc)) + dJ12 * (2 * fy * ty / (zc * zc * zc));
  if (clx) dzc += dtx * txz; else dxc += dtx;
  if (cly) dzc += dty * tyz; else dyc += dty;
  /* mean2d */
  dxc += dp[0] * fx / zc;
  dzc += dp[0] * (-fx * xc / (zc * zc));
  dyc += dp[1] * fy / zc;
  dzc += dp[1] * (-fy * yc / (zc * zc));
  for (int a2 = 0; a2 < 3; ++a2) dg[a2] = R[a2] * dxc + R[3 + a2] * dyc + R[6 + a2] * dzc;
  for (int a2 = 0; a2 < 3; ++a2) dg[3 + a2] = ds[a2];
  dg[6] = dw; dg[7] = dx; dg[8] = dy; dg[9] = dz;
  dg[10] = dp[5];
  dg[11] = dp[6]; dg[12] = dp[7]; dg[13] = dp[8];
}

/* dL/dGaussian [14][stride] (double) from dproj [n][9] for visible ones. */
ORC_API void orc_project_backward(int64_t n, int64_t stride, const double *gd, const uint8_t *vis,
                                  const float *camf, int W, int H, const float *prmf,
                                  const double *dproj, double *dgauss) {
  cam_t k = load_cam(camf, W, H);
  prm_t pp = load_prm(prmf);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double g[14], dg[14];
    for (int f = 0; f < 14; ++f) { g[f] = gd[f * stride + i]; dg[f] = 0; }
    if (vis[i]) project_bwd_one(&k, &pp, g, dproj + 9 * i, dg);
    for (int f = 0; f < 14; ++f) dgauss[f * stride + i] = dg[f];
  }
}

/* Decode backward.  dgauss [14][m*k] -> gradients of the anchor arrays
 * (accumulated; caller zeroes) and of the 12 MLP arrays (accumulated).
 * dmlp follows the order of mlp: w1a, b1a, w2a, b2a, w1c, ... */
ORC_API void orc_decode_backward(int64_t m, const int64_t *idx, const float *pos,
                                 const float *feat, const float *offsets,
                                 const float *offset_scale, const float *base_scale, int k,
                                 int F, int Wd, const float *const *mlp, const float *Cw,
                                 float d_max, const double *dgauss, double *dpos, double *dfeat,
                                 double *doffsets, double *doscale, double *dbscale,
                                 double *const *dmlp) {
  int64_t G = m * k;
  int in = F + 4;
  int outs[3] = {k, 3 * k, 7 * k};
  for (int64_t s = 0; s < m; ++s) {
    int64_t j = idx[s];
    double x[64], hp[3][64], y[3][448];
    decode_input(feat + j * F, F, pos + 3 * j, Cw, d_max, x);
    for (int h = 0; h < 3; ++h)
      head_fwd(x, in, Wd, outs[h], mlp[4 * h], mlp[4 * h + 1], mlp[4 * h + 2], mlp[4 * h + 3],
               hp[h], y[h]);
    double dy[3][448];
    memset(dy, 0, sizeof dy);
    for (int i = 0; i < k; ++i) {
      int64_t g = s * k + i;
      const float *o = offsets + (j * k + i) * 3;
      for (int a = 0; a < 3; ++a) {
        double dm = dgauss[a * G + g];
        dpos[3 * j + a] += dm;
        doffsets[(j * k + i) * 3 + a] += dm * offset_scale[3 * j + a];
        doscale[3 * j + a] += dm * o[a];
      }
      for (int a = 0; a < 3; ++a) {
        double sg = sigm(y[2][7 * i + a]);
        double dsc = dgauss[(3 + a) * G + g];
        dbscale[3 * j + a] += dsc * sg;
        dy[2][7 * i + a] = dsc * base_scale[3 * j + a] * sg * (1 - sg);
      }
      double q[4], qn = 0;
      for (int a = 0; a < 4; ++a) { q[a] = y[2][7 * i + 3 + a]; qn += q[a] * q[a]; }
      qn = sqrt(qn);
      if (qn > 0) {
        double u[4], dqn[4], dot = 0;
        for (int a = 0; a < 4; ++a) { u[a] = q[a] / qn; dqn[a] = dgauss[(6 + a) * G + g]; dot += u[a] * dqn[a]; }
        for (int a = 0; a < 4; ++a) dy[2][7 * i + 3 + a] = (dqn[a] - u[a] * dot) / qn;
      }
      double op = tanh(y[0][i]);
      dy[0][i] = dgauss[10 * G + g] * (1 - op * op);
      for (int a = 0; a < 3; ++a) {
        double sg = sigm(y[1][3 * i + a]);
        dy[1][3 * i + a] = dgauss[(11 + a) * G + g] * sg * (1 - sg);
      }
    }
    double dx[64];
    memset(dx, 0, sizeof dx);
    for (int h = 0; h < 3; ++h) {
      const float *w1 = mlp[4 * h], *w2 = mlp[4 * h + 2];
      double *dw1 = dmlp[4 * h], *db1 = dmlp[4 * h + 1], *dw2 = dmlp[4 * h + 2], *db2 = dmlp[4 * h + 3];
      int out = outs[h];
      double dh[64];
      for (int u = 0; u < Wd; ++u) {
        double hv = hp[h][u] > 0 ? hp[h][u] : 0.0, acc = 0;
        for (int o = 0; o < out; ++o) {
          dw2[u * out + o] += hv * dy[h][o];
          acc += (double)w2[u * out + o] * dy[h][o];
        }
        dh[u] = hp[h][u] > 0 ? acc : 0.0;
      }
      for (int o = 0; o < out; ++o) db2[o] += dy[h][o];
      for (int u = 0; u < Wd; ++u) {
        db1[u] += dh[u];
        for (int i2 = 0; i2 < in; ++i2) {
          dw1[i2 * Wd + u] += x[i2] * dh[u];
          dx[i2] += (double)w1[i2 * Wd + u] * dh[u];
        }
      }
    }
    for (int i2 = 0; i2 < F; ++i2) dfeat[j * F + i2] += dx[i2];
    /* x[F] = |p - C| / d_max, x[F+1..F+3] = (p - C) / |p - C| */
    double dd[3], n2 = 0;
    for (int a = 0; a < 3; ++a) { dd[a] = (double)pos[3 * j + a] - (double)Cw[a]; n2 += dd[a] * dd[a]; }
    double dist = sqrt(n2), u[3], dot = 0;
    for (int a = 0; a < 3; ++a) { u[a] = dd[a] / dist; dot += u[a] * dx[F + 1 + a]; }
    for (int a = 0; a < 3; ++a)
      dpos[3 * j + a] += u[a] * dx[F] / d_max + (dx[F + 1 + a] - u[a] * dot) / dist;
  }
}

/* ======================================================================
 * Anchor-skip predictor (extension of the per-view anchor selection):
 * inputs, forward and binary cross-entropy gradient, double precision.
 * ====================================================================== */

/* z[s][0..36] = feature (32), unit direction camera -> anchor in camera
 * coordinates R (x - C) / |x - C| (3), log2(|x - C| / d_max), level. */
ORC_API void orc_skip_features(int64_t m, const int64_t *idx, const float *pos, const float *feat,
                               const uint8_t *level, const float *Rw, const float *Cw, float d_max,
                               double *z) {
  for (int64_t s = 0; s < m; ++s) {
    int64_t j = idx[s];
    double *o = z + 37 * s;
    for (int f = 0; f < 32; ++f) o[f] = feat[32 * j + f];
    double d[3], n2 = 0;
    for (int a = 0; a < 3; ++a) { d[a] = (double)pos[3 * j + a] - (double)Cw[a]; n2 += d[a] * d[a]; }
    double dist = sqrt(n2);
    for (int a = 0; a < 3; ++a)
      o[32 + a] = (Rw[3 * a] * d[0] + Rw[3 * a + 1] * d[1] + Rw[3 * a + 2] * d[2]) / dist;
    o[35] = log2(dist / (double)d_max);
    o[36] = level[j];
  }
}

/* Predictor 37 -> 64 -> ReLU -> 64 -> ReLU -> 1 on B rows of z.  logit[B];
 * with labels y: *loss = mean of w (softplus(x) - y x), w = pos_weight for
 * positives, and (grads non-NULL) its gradient w.r.t. w1, b1, w2, b2, w3, b3
 * (overwritten).  net: w1 [37][64], b1, w2 [64][64], b2, w3 [64], b3 [1]. */
ORC_API void orc_skip_mlp(int64_t B, const double *z, const float *y, float pos_weight,
                          const float *const *net, double *logit, double *loss,
                          double *const *grads) {
  const float *w1 = net[0], *b1 = net[1], *w2 = net[2], *b2 = net[3], *w3 = net[4], *b3 = net[5];
  if (grads) {
    int sizes[6] = {37 * 64, 64, 64 * 64, 64, 64, 1};
    for (int q = 0; q < 6; ++q) memset(grads[q], 0, sizeof(double) * (size_t)sizes[q]);
  }
  double L = 0;
  for (int64_t r = 0; r < B; ++r) {
    const double *x = z + 37 * r;
    double h1[64], h2[64], a1[64], a2[64];
    for (int u = 0; u < 64; ++u) {
      double s = b1[u];
      for (int i = 0; i < 37; ++i) s += x[i] * (double)w1[i * 64 + u];
      h1[u] = s;
      a1[u] = s > 0 ? s : 0;
    }
    for (int u = 0; u < 64; ++u) {
      double s = b2[u];
      for (int i = 0; i < 64; ++i) s += a1[i] * (double)w2[i * 64 + u];
      h2[u] = s;
      a2[u] = s > 0 ? s : 0;
    }
    double out = b3[0];
    for (int i = 0; i < 64; ++i) out += a2[i] * (double)w3[i];
    logit[r] = out;
    if (!y) continue;
    double yy = y[r], wgt = yy > 0.5 ? pos_weight : 1.0;
    double sp = (out > 0 ? out : 0) + log1p(exp(-fabs(out)));
    L += wgt * (sp - yy * out);
    if (!grads) continue;
    double dout = wgt * (1.0 / (1.0 + exp(-out)) - yy) / (double)B;
    double da2[64], dh2[64], da1[64], dh1[64];
    grads[5][0] += dout;
    for (int i = 0; i < 64; ++i) {
      grads[4][i] += a2[i] * dout;
      da2[i] = (double)w3[i] * dout;
      dh2[i] = h2[i] > 0 ? da2[i] : 0;
    }
    for (int i = 0; i < 64; ++i) {
      double s = 0;
      for (int u = 0; u < 64; ++u) {
        grads[2][i * 64 + u] += a1[i] * dh2[u];
        s += (double)w2[i * 64 + u] * dh2[u];
      }
      da1[i] = s;
      dh1[i] = h1[i] > 0 ? s : 0;
    }
    for (int u = 0; u < 64; ++u) {
      grads[3][u] += dh2[u];
      grads[1][u] += dh1[u];
      for (int i = 0; i < 37; ++i) grads[0][i * 64 + u] += x[i] * dh1[u];
    }
  }
  if (loss) *loss = L / (double)B;
}
