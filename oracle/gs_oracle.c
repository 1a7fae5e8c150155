/*
 * gs_oracle.c — plain, slow, FP64 CPU oracle of one 3D Gaussian Splatting
 * training step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the GPU library; the two are
 * compared on the same seeded inputs.
 *
 * What it follows.  The paper (Sec. II, "Parallel Training") trains every
 * partition with the 3D Gaussian Splatting method of Kerbl et al. (cited in
 * Sec. I); its masks come from Sec. II ("Image Rendering and Masking") and
 * Sec. III-A.  The paper prints no formula of its own, so every function below
 * restates the standard definition of the step it implements; the readings
 * taken where the paper is silent (near plane, dilation, support, cut-off,
 * tie-break, colour model) are listed with the design notes.  Every number is
 * FP64.  There is no tiling, blocking or reordering beyond what a definition
 * states: the per-pixel loop runs over ALL Gaussians in (depth, index) order
 * and only consults a Gaussian's tile set (or_support_tiles) because the
 * method's own binning defines the per-pixel list that way.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared gs_oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_DILATE 0.3               /* low-pass added to the 2D covariance  */
#define OR_FRUSTUM 1.3              /* Jacobian clamp, x tan(fov/2)         */
#define OR_ALPHA_MAX 0.99
#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_T_MIN 1e-4

/* ---------------------------------------------------------------------- */
/* Activations and 3D covariance                                            */
/* ---------------------------------------------------------------------- */

/* Rotation matrix of a unit quaternion (w, x, y, z), row-major.           */
static void quat_to_rot(const double q[4], double R[9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* ---------------------------------------------------------------------- */
/* View-dependent colour: real spherical harmonics                          */
/* ---------------------------------------------------------------------- */

#define OR_SH_MAX 3                 /* highest degree of the colour model   */
#define OR_SH_K ((OR_SH_MAX + 1) * (OR_SH_MAX + 1))

/* Coefficients c[0..l] of the Legendre polynomial P_l (Bonnet recurrence
 * (j+1) P_{j+1} = (2j+1) z P_j - j P_{j-1}).                               */
static void legendre_coeffs(int l, double c[OR_SH_MAX + 1]) {
  double pm[OR_SH_MAX + 2] = {0}, p[OR_SH_MAX + 2] = {0}, nx[OR_SH_MAX + 2];
  p[0] = 1.0;                                          /* P_0 */
  for (int j = 0; j < l; ++j) {
    for (int i = 0; i <= OR_SH_MAX + 1; ++i) {
      double zp = i > 0 ? p[i - 1] : 0.0;
      nx[i] = ((2 * j + 1) * zp - j * pm[i]) / (j + 1);
    }
    memcpy(pm, p, sizeof(p));
    memcpy(p, nx, sizeof(p));
  }
  for (int i = 0; i <= OR_SH_MAX; ++i) c[i] = p[i];
}

/* Value at z of the m-th derivative of the polynomial c[0..deg].           */
static double poly_deriv_eval(const double* c, int deg, int m, double z) {
  double r = 0.0;
  for (int i = deg; i >= m; --i) {
    double f = 1.0;
    for (int j = 0; j < m; ++j) f *= (double)(i - j);
    r = r * z + f * c[i];
  }
  return r;
}

static double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

/* Real spherical harmonics of degree <= D at the unit vector d, Condon-
 * Shortley phase included, index l*l + l + m (m = -l..l).  With P_l the
 * Legendre polynomial, D^m P_l its m-th derivative and
 * K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!):
 *   Y_l0  = K_l0 P_l(z)
 *   Y_lm  = (-1)^m sqrt(2) K_lm D^m P_l(z) Re((x + i y)^m)     (m > 0)
 *   Y_l-m = (-1)^m sqrt(2) K_lm D^m P_l(z) Im((x + i y)^m)
 * which is the textbook definition written with
 * sin^m(theta) e^{i m phi} = (x + i y)^m on the sphere.  grad[k] is the
 * gradient of the k-th expression as a polynomial in (x, y, z); its part
 * tangent to the sphere is the derivative of Y_k along the sphere, the only
 * part the chain rule through d = v / |v| keeps.                           */
static void sh_basis(int D, const double d[3], double* Y, double (*grad)[3]) {
  double x = d[0], y = d[1], z = d[2];
  for (int l = 0; l <= D; ++l) {
    double P[OR_SH_MAX + 1];
    legendre_coeffs(l, P);
    for (int m = 0; m <= l; ++m) {
      double K = sqrt((2.0 * l + 1.0) / (4.0 * acos(-1.0)) * factorial(l - m) / factorial(l + m));
      double q = poly_deriv_eval(P, l, m, z);
      double qz = poly_deriv_eval(P, l, m + 1, z);
      /* w = (x + i y)^m, w1 = (x + i y)^(m-1) */
      double wr = 1.0, wi = 0.0, w1r = 0.0, w1i = 0.0;
      for (int j = 0; j < m; ++j) {
        w1r = wr; w1i = wi;
        double tr = wr * x - wi * y, ti = wr * y + wi * x;
        wr = tr; wi = ti;
      }
      if (m == 0) {
        Y[l * l + l] = K * q;
        grad[l * l + l][0] = 0.0;
        grad[l * l + l][1] = 0.0;
        grad[l * l + l][2] = K * qz;
        continue;
      }
      double s = ((m & 1) ? -1.0 : 1.0) * sqrt(2.0) * K;
      int kp = l * l + l + m, kn = l * l + l - m;
      /* d/dx (x+iy)^m = m w1, d/dy (x+iy)^m = i m w1 */
      Y[kp] = s * q * wr;
      grad[kp][0] = s * q * m * w1r;
      grad[kp][1] = -s * q * m * w1i;
      grad[kp][2] = s * qz * wr;
      Y[kn] = s * q * wi;
      grad[kn][0] = s * q * m * w1i;
      grad[kn][1] = s * q * m * w1r;
      grad[kn][2] = s * qz * wi;
    }
  }
}

/* sh_basis at npts unit vectors d [npts][3]: Y [npts][(D+1)^2],
 * grad [npts][(D+1)^2][3].                                                 */
void or_sh_basis(int D, int64_t npts, const double* d, double* Y, double* grad) {
  int K = (D + 1) * (D + 1);
  for (int64_t p = 0; p < npts; ++p) {
    double y[OR_SH_K], g[OR_SH_K][3];
    sh_basis(D, d + 3 * p, y, g);
    for (int k = 0; k < K; ++k) {
      Y[p * K + k] = y[k];
      for (int j = 0; j < 3; ++j) grad[(p * K + k) * 3 + j] = g[k][j];
    }
  }
}

/* Everything the projection computes for one Gaussian in one view, kept so
 * that the backward pass can reuse the forward's intermediate values.      */
typedef struct {
  double s[3], qn[4], qnorm, o, rgb[3], pre_rgb[3];
  int sh_deg;
  double dir[3], vlen;        /* unit vector camera centre -> mean, |v|   */
  double Y[OR_SH_K], dY[OR_SH_K][3];
  double R[9], Sigma[9];
  double t[3], mean2d[2];
  double J[6], xclamp, yclamp; int xclamped, yclamped;
  double T[6];                /* J * Rv (2x3)                             */
  double a, b, c, det;        /* dilated 2D covariance entries            */
  double conic[3];
  double kappa, hx, hy;
  int pix[4], tile[4], n_tiles, valid;
} or_proj;

/* cam: R[9], t[3], fx, fy, cx, cy (16 doubles).  color: the (D+1)^2 x 3
 * spherical-harmonic coefficients of one Gaussian, coefficient-major
 * (color[k*3 + channel]), D = sh_deg.  The colour seen from the camera is
 * max(0, sum_k Y_k(d) color[k] + 1/2) with d the unit vector from the camera
 * centre -R^T t to the mean (3D-GS colour model).                          */
static void project_one(const double* mean, const double* ls, const double* quat,
                        double opac_logit, const double* color, int sh_deg, const double* cam,
                        double znear, int W, int H, int tw, int th, or_proj* P) {
  memset(P, 0, sizeof(*P));
  for (int k = 0; k < 3; ++k) P->s[k] = exp(ls[k]);
  double qn = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
  P->qnorm = qn;
  for (int k = 0; k < 4; ++k) P->qn[k] = quat[k] / qn;
  P->o = 1.0 / (1.0 + exp(-opac_logit));
  P->sh_deg = sh_deg;
  {
    const double* Rc = cam; const double* tc = cam + 9;
    double v[3];
    for (int i = 0; i < 3; ++i)        /* mean - (-R^T t) */
      v[i] = mean[i] + Rc[0 * 3 + i] * tc[0] + Rc[1 * 3 + i] * tc[1] + Rc[2 * 3 + i] * tc[2];
    P->vlen = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int i = 0; i < 3; ++i) P->dir[i] = P->vlen > 0 ? v[i] / P->vlen : (i == 2);
  }
  sh_basis(sh_deg, P->dir, P->Y, P->dY);
  int K = (sh_deg + 1) * (sh_deg + 1);
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (int j = 0; j < K; ++j) acc += P->Y[j] * color[j * 3 + k];
    P->pre_rgb[k] = acc + 0.5;
    P->rgb[k] = P->pre_rgb[k] > 0 ? P->pre_rgb[k] : 0.0;
  }
  quat_to_rot(P->qn, P->R);
  /* Sigma = R diag(s^2) R^T */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += P->R[i * 3 + k] * P->s[k] * P->s[k] * P->R[j * 3 + k];
      P->Sigma[i * 3 + j] = acc;
    }
  const double* Rv = cam; const double* tv = cam + 9;
  double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
  for (int i = 0; i < 3; ++i)
    P->t[i] = Rv[i * 3 + 0] * mean[0] + Rv[i * 3 + 1] * mean[1] + Rv[i * 3 + 2] * mean[2] + tv[i];
  double tx = P->t[0], ty = P->t[1], tz = P->t[2];
  if (!(tz > znear)) { P->valid = 0; return; }
  P->mean2d[0] = fx * tx / tz + cx;
  P->mean2d[1] = fy * ty / tz + cy;
  double limx = OR_FRUSTUM * W / (2.0 * fx), limy = OR_FRUSTUM * H / (2.0 * fy);
  double rx = tx / tz, ry = ty / tz;
  P->xclamped = (rx < -limx || rx > limx);
  P->yclamped = (ry < -limy || ry > limy);
  if (rx < -limx) rx = -limx; if (rx > limx) rx = limx;
  if (ry < -limy) ry = -limy; if (ry > limy) ry = limy;
  P->xclamp = rx * tz; P->yclamp = ry * tz;
  double* J = P->J;
  J[0] = fx / tz; J[1] = 0;       J[2] = -fx * P->xclamp / (tz * tz);
  J[3] = 0;       J[4] = fy / tz; J[5] = -fy * P->yclamp / (tz * tz);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += J[i * 3 + k] * Rv[k * 3 + j];
      P->T[i * 3 + j] = acc;
    }
  double V[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc += P->T[i * 3 + k] * P->Sigma[k * 3 + l] * P->T[j * 3 + l];
      V[i * 2 + j] = acc;
    }
  P->a = V[0] + OR_DILATE; P->b = 0.5 * (V[1] + V[2]); P->c = V[3] + OR_DILATE;
  P->det = P->a * P->c - P->b * P->b;
  if (!(P->det > 0)) { P->valid = 0; return; }
  P->conic[0] = P->c / P->det; P->conic[1] = -P->b / P->det; P->conic[2] = P->a / P->det;
  if (!(255.0 * P->o > 1.0)) { P->valid = 0; return; }
  P->kappa = 2.0 * log(255.0 * P->o);
  P->hx = sqrt(P->kappa * P->a); P->hy = sqrt(P->kappa * P->c);
  /* padded pixel bbox; the float argument is clamped to [-4, W+4] first,
   * which cannot change the result after intersecting with the image.    */
  double xs[2] = {P->mean2d[0] - P->hx, P->mean2d[0] + P->hx};
  double ys[2] = {P->mean2d[1] - P->hy, P->mean2d[1] + P->hy};
  for (int k = 0; k < 2; ++k) {
    if (!(xs[k] > -4.0)) xs[k] = -4.0; if (xs[k] > W + 4.0) xs[k] = W + 4.0;
    if (!(ys[k] > -4.0)) ys[k] = -4.0; if (ys[k] > H + 4.0) ys[k] = H + 4.0;
  }
  int x0 = (int)floor(xs[0]) - 1, x1 = (int)floor(xs[1]) + 1;
  int y0 = (int)floor(ys[0]) - 1, y1 = (int)floor(ys[1]) + 1;
  if (x0 < 0) x0 = 0; if (y0 < 0) y0 = 0;
  if (x1 > W - 1) x1 = W - 1; if (y1 > H - 1) y1 = H - 1;
  if (x0 > x1 || y0 > y1) { P->valid = 0; return; }
  P->pix[0] = x0; P->pix[1] = y0; P->pix[2] = x1; P->pix[3] = y1;
  P->tile[0] = x0 / tw; P->tile[1] = y0 / th; P->tile[2] = x1 / tw; P->tile[3] = y1 / th;
  P->n_tiles = (P->tile[2] - P->tile[0] + 1) * (P->tile[3] - P->tile[1] + 1);
  P->valid = 1;
}

/* Project n Gaussians (planar SoA inputs) through one camera.  color is
 * [(D+1)^2][3][n] (coefficient k of channel c in row 3k + c), D = sh_deg.  */
void or_project(int64_t n, const double* mean, const double* log_scale, const double* quat,
                const double* opac_logit, const double* color, int sh_deg, const double* cam,
                double znear,
                int W, int H, int tw, int th, double* out_mean2d, double* out_conic,
                double* out_depth, double* out_opacity, double* out_rgb, double* out_cov2d,
                int32_t* out_pix_bbox, int32_t* out_tile_bbox, int32_t* out_n_tiles,
                int32_t* out_valid) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double mu[3] = {mean[i], mean[n + i], mean[2 * n + i]};
    double ls[3] = {log_scale[i], log_scale[n + i], log_scale[2 * n + i]};
    double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
    double f[3 * OR_SH_K];
    for (int r = 0; r < 3 * (sh_deg + 1) * (sh_deg + 1); ++r) f[r] = color[r * n + i];
    or_proj P;
    project_one(mu, ls, q, opac_logit[i], f, sh_deg, cam, znear, W, H, tw, th, &P);
    out_mean2d[i] = P.mean2d[0]; out_mean2d[n + i] = P.mean2d[1];
    for (int k = 0; k < 3; ++k) out_conic[k * n + i] = P.conic[k];
    out_depth[i] = P.t[2];
    out_opacity[i] = P.o;
    for (int k = 0; k < 3; ++k) out_rgb[k * n + i] = P.rgb[k];
    out_cov2d[i] = P.a; out_cov2d[n + i] = P.b; out_cov2d[2 * n + i] = P.c;
    for (int k = 0; k < 4; ++k) {
      out_pix_bbox[k * n + i] = P.valid ? P.pix[k] : 0;
      out_tile_bbox[k * n + i] = P.valid ? P.tile[k] : 0;
    }
    out_n_tiles[i] = P.valid ? P.n_tiles : 0;
    out_valid[i] = P.valid;
  }
}

/* ---------------------------------------------------------------------- */
/* Rasterisation: the per-pixel compositing definition                      */
/* ---------------------------------------------------------------------- */

typedef struct { double depth; int64_t idx; } or_key;

static int cmp_key(const void* A, const void* B) {
  const or_key* a = (const or_key*)A; const or_key* b = (const or_key*)B;
  if (a->depth < b->depth) return -1;
  if (a->depth > b->depth) return 1;
  return (a->idx < b->idx) ? -1 : (a->idx > b->idx);
}

/* Valid Gaussians in ascending (depth, index) order; returns the count.    */
static int64_t sorted_order(int64_t n, const double* depth, const int32_t* valid, int64_t* order) {
  or_key* keys = (or_key*)malloc(sizeof(or_key) * (size_t)(n > 0 ? n : 1));
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i)
    if (valid[i]) { keys[cnt].depth = depth[i]; keys[cnt].idx = i; ++cnt; }
  qsort(keys, (size_t)cnt, sizeof(or_key), cmp_key);
  for (int64_t k = 0; k < cnt; ++k) order[k] = keys[k].idx;
  free(keys);
  return cnt;
}

/* ---------------------------------------------------------------------- */
/* Tiles a pair is binned to                                                */
/* ---------------------------------------------------------------------- */

/* A pair is listed on the tiles of its tile bbox whose pixel-centre
 * rectangle [tx tw + 1/2, tx tw + tw - 1/2] x [ty th + 1/2, ty th + th - 1/2]
 * meets its support (alpha >= 1/255: Q(d) = d^T conic d <= 2 ln(255 o)),
 * widened by a margin mu = 0.02 + 1e-5 M that absorbs single-precision
 * rounding (M = a X^2 + 2|b| X Y + c Y^2 bounds the magnitudes of the terms
 * of Q over the bbox, X and Y the largest |dx|, |dy| to its pixel-centre
 * extents).  A tile whose rectangle misses the widened support holds no
 * pixel centre where the pair can pass the alpha test, so leaving it out
 * changes no image.  Pairs whose bbox has more than OR_MASK_TILES tiles are
 * listed on all of them.                                                   */
#define OR_MASK_TILES 64

/* min over the rectangle [dx0,dx1] x [dy0,dy1] of a dx^2 + 2 b dx dy + c dy^2
 * (positive definite): zero if the rectangle holds the origin, else the
 * least of the four edge minima, each at the clamped stationary point.     */
static double rect_min_quad(double dx0, double dx1, double dy0, double dy1, double a, double b,
                            double c) {
  if (dx0 <= 0 && dx1 >= 0 && dy0 <= 0 && dy1 >= 0) return 0.0;
  double best = INFINITY;
  for (int e = 0; e < 2; ++e) {
    double dx = e ? dx1 : dx0;                       /* vertical edge     */
    double dy = -b * dx / c;
    dy = dy < dy0 ? dy0 : (dy > dy1 ? dy1 : dy);
    double q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
    if (q < best) best = q;
    dy = e ? dy1 : dy0;                              /* horizontal edge   */
    dx = -b * dy / a;
    dx = dx < dx0 ? dx0 : (dx > dx1 ? dx1 : dx);
    q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
    if (q < best) best = q;
  }
  return best;
}

/* Tile set of one pair with mean (mx, my), conic (a, b, c), opacity o and
 * tile bbox (tx0, ty0, tx1, ty1): bit (ty - ty0) * span + (tx - tx0) of
 * *mask is set when tile (tx, ty) is listed; *mask = 0 when the bbox has
 * more than OR_MASK_TILES tiles (all are listed).  *amb marks the tiles
 * whose decision lies within band * threshold + 1e-6 M of the threshold,
 * where a single-precision evaluation may decide the other way.           */
static void support_mask(double mx, double my, double a, double b, double c, double o, int tx0,
                         int ty0, int tx1, int ty1, int tw, int th, double band, uint64_t* mask,
                         uint64_t* amb) {
  *mask = 0; *amb = 0;
  int span = tx1 - tx0 + 1;
  if ((int64_t)span * (ty1 - ty0 + 1) > OR_MASK_TILES) return;
  double X0 = fabs(tx0 * (double)tw + 0.5 - mx), X1 = fabs(tx1 * (double)tw + tw - 0.5 - mx);
  double Y0 = fabs(ty0 * (double)th + 0.5 - my), Y1 = fabs(ty1 * (double)th + th - 0.5 - my);
  double X = X0 > X1 ? X0 : X1, Y = Y0 > Y1 ? Y0 : Y1;
  double M = a * X * X + 2.0 * fabs(b) * X * Y + c * Y * Y;
  double thr = 2.0 * log(255.0 * o) + 0.02 + 1e-5 * M;
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) {
      double q = rect_min_quad(tx * (double)tw + 0.5 - mx, tx * (double)tw + tw - 0.5 - mx,
                               ty * (double)th + 0.5 - my, ty * (double)th + th - 0.5 - my, a,
                               b, c);
      uint64_t bit = 1ull << ((ty - ty0) * span + (tx - tx0));
      if (q <= thr) *mask |= bit;
      if (fabs(q - thr) <= band * thr + 1e-6 * M) *amb |= bit;
    }
}

/* support_mask of every pair p (SoA mean2d [2][n], conic [3][n], opacity
 * [n], tile_bbox [4][n]); pairs with valid[p] == 0 get zero masks.         */
void or_support_tiles(int64_t n, const double* mean2d, const double* conic,
                      const double* opacity, const int32_t* tile_bbox, const int32_t* valid,
                      int tw, int th, double band, uint64_t* mask, uint64_t* amb) {
  for (int64_t p = 0; p < n; ++p) {
    mask[p] = 0; amb[p] = 0;
    if (!valid[p]) continue;
    support_mask(mean2d[p], mean2d[n + p], conic[p], conic[n + p], conic[2 * n + p], opacity[p],
                 tile_bbox[p], tile_bbox[n + p], tile_bbox[2 * n + p], tile_bbox[3 * n + p], tw,
                 th, band, &mask[p], &amb[p]);
  }
}

/* Is tile (tx, ty) on pair g's list: 0 no, 1 yes; 2 no and 3 yes where the
 * decision is ambiguous.                                                   */
static int listed(int64_t n, int64_t g, int tx, int ty, const int32_t* tile_bbox,
                  const uint64_t* mask, const uint64_t* amb) {
  int tx0 = tile_bbox[g], ty0 = tile_bbox[n + g], tx1 = tile_bbox[2 * n + g],
      ty1 = tile_bbox[3 * n + g];
  if (tx < tx0 || ty < ty0 || tx > tx1 || ty > ty1) return 0;
  int span = tx1 - tx0 + 1;
  if (!mask || (int64_t)span * (ty1 - ty0 + 1) > OR_MASK_TILES) return 1;
  uint64_t bit = 1ull << ((ty - ty0) * span + (tx - tx0));
  int on = (mask[g] & bit) ? 1 : 0;
  return (amb && (amb[g] & bit)) ? 2 + on : on;
}

/* Tile sets of a render call (NULL masks when use_support is 0: every
 * bbox tile).                                                              */
static void render_masks(int64_t n, const double* mean2d, const double* conic,
                         const double* opacity, const int32_t* tile_bbox, const int32_t* valid,
                         int tw, int th, int use_support, double band, uint64_t** mask,
                         uint64_t** amb) {
  *mask = *amb = NULL;
  if (!use_support) return;
  *mask = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  *amb = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  or_support_tiles(n, mean2d, conic, opacity, tile_bbox, valid, tw, th, band, *mask, *amb);
}

typedef struct {
  int64_t g;
  double alpha, a, e, T, dx, dy;
} or_blend;

/* Composite one pixel.  Inputs are SoA per Gaussian; `order` lists the valid
 * Gaussians sorted by (depth, index).  If `rec` is non-NULL the blended
 * entries are recorded (capacity n).  Returns the number blended.
 * band_rel is the relative half-width of the guard bands around the alpha
 * thresholds (1/255 and 0.99) and the least relative half-width of the one
 * around the transmittance cut-off, inside which a pixel is marked
 * ambiguous: an input given to FP32 to within that relative error may take
 * the other branch there.  It classifies pixels only; the composite itself
 * does not depend on it.                                                   */
static int64_t composite_pixel(int px, int py, int tw, int th, int64_t n, int64_t cnt,
                               const int64_t* order, const double* mean2d, const double* conic,
                               const double* depth, const double* opacity, const double* rgb,
                               const int32_t* tile_bbox, const uint64_t* mask,
                               const uint64_t* mamb, const double* bg, double out[3],
                               double* T_out, int32_t* ncontrib_out, uint8_t* amb_out,
                               or_blend* rec, double band_rel) {
  double T = 1.0, C[3] = {0, 0, 0};
  int tx = px / tw, ty = py / th;
  double cxp = px + 0.5, cyp = py + 0.5;
  int64_t pos = 0, last = 0, nb = 0;
  int amb = 0;
  /* depth of the previous entry that passed the alpha test: two such entries
   * at near-equal depths may be sorted either way from FP32 depths, which
   * matters when either is blended or stops the pixel; after the stop, the
   * next passing entry is the one that could take the stopping one's place */
  double prev_depth = -1.0;
  int stopped = 0;
  int64_t first_amb = 0;      /* list position of the first ambiguous listing */
  for (int64_t k = 0; k < cnt; ++k) {
    int64_t g = order[k];
    int on = listed(n, g, tx, ty, tile_bbox, mask, mamb);
    /* an entry whose listing is ambiguous cannot blend here (it lies outside
     * the widened support) but shifts the list positions after it */
    if (on >= 2 && first_amb == 0 && !stopped) first_amb = pos + 1;
    if (on == 0 || on == 2) continue;             /* not in this tile's list */
    /* entries are in ascending depth: past the band nothing can tie */
    if (stopped && depth[g] - prev_depth > 5e-7 * fabs(depth[g])) break;
    ++pos;
    double dx = cxp - mean2d[g], dy = cyp - mean2d[n + g];
    double q11 = conic[g], q12 = conic[n + g], q22 = conic[2 * n + g];
    double qf = q11 * dx * dx + 2.0 * q12 * dx * dy + q22 * dy * dy;
    double qabs = fabs(q11 * dx * dx) + fabs(2.0 * q12 * dx * dy) + fabs(q22 * dy * dy);
    if (!stopped && qabs > 0 && fabs(qf) <= 1e-5 * qabs) amb |= 1;
    double power = -0.5 * qf;
    if (power > 0) continue;
    double e = exp(power);
    double a = opacity[g] * e;
    if (!stopped && fabs(a - OR_ALPHA_MIN) <= band_rel * OR_ALPHA_MIN) amb |= 2;
    if (!stopped && fabs(a - OR_ALPHA_MAX) <= band_rel * OR_ALPHA_MAX) amb |= 4;
    double alpha = a < OR_ALPHA_MAX ? a : OR_ALPHA_MAX;
    if (alpha < OR_ALPHA_MIN) continue;
    if (prev_depth >= 0 && fabs(depth[g] - prev_depth) <= 5e-7 * fabs(depth[g])) amb |= 16;
    prev_depth = depth[g];
    if (stopped) break;
    double Tn = T * (1.0 - alpha);
    double band = 8.0 * (double)(nb + 1) * 5.9604644775390625e-08;  /* 8 n 2^-24 */
    if (band < band_rel) band = band_rel;
    if (fabs(Tn - OR_T_MIN) <= band * OR_T_MIN) amb |= 8;
    if (Tn < OR_T_MIN) {
      stopped = 1;
      continue;
    }
    if (rec) {
      rec[nb].g = g; rec[nb].alpha = alpha; rec[nb].a = a; rec[nb].e = e;
      rec[nb].T = T; rec[nb].dx = dx; rec[nb].dy = dy;
    }
    for (int ch = 0; ch < 3; ++ch) C[ch] += rgb[ch * n + g] * alpha * T;
    T = Tn;
    last = pos;
    ++nb;
  }
  if (first_amb > 0 && first_amb < last) amb |= 32;   /* n_contrib may differ */
  for (int ch = 0; ch < 3; ++ch) out[ch] = C[ch] + T * bg[ch];
  if (T_out) *T_out = T;
  if (ncontrib_out) *ncontrib_out = (int32_t)last;
  if (amb_out) *amb_out = (uint8_t)amb;
  return nb;
}

/* Minimum relative band of the listing decisions (single-precision
 * evaluation of the tile test on the same records).                       */
#define OR_LIST_BAND 2e-4

/* Render the pixel window [x0,x1) x [y0,y1) of one W x H image.  image is a
 * full [3][H][W] buffer; T_final, n_contrib, n_blended, ambiguous are full
 * [H][W] buffers (each may be NULL).  tile_bbox is SoA [4][n].  Tile lists
 * hold the pairs binned there (or_support_tiles), or every pair whose bbox
 * covers the tile when use_support is 0; only n_contrib, a list position,
 * depends on it.                                                           */
void or_render(int64_t n, const double* mean2d, const double* conic, const double* depth,
               const double* opacity, const double* rgb, const int32_t* tile_bbox,
               const int32_t* valid, int W, int H, int tw, int th, const double* bg, int x0,
               int y0, int x1, int y1, double* image, double* T_final, int32_t* n_contrib,
               int32_t* n_blended, uint8_t* ambiguous, double band_rel, int use_support) {
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t cnt = sorted_order(n, depth, valid, order);
  int64_t npix = (int64_t)(x1 - x0) * (y1 - y0);
  uint64_t *mask, *mamb;
  render_masks(n, mean2d, conic, opacity, tile_bbox, valid, tw, th, use_support,
               band_rel > OR_LIST_BAND ? band_rel : OR_LIST_BAND, &mask, &mamb);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t pi = 0; pi < npix; ++pi) {
    int px = x0 + (int)(pi % (x1 - x0)), py = y0 + (int)(pi / (x1 - x0));
    int64_t o = (int64_t)py * W + px;
    double out[3], T; int32_t nc; uint8_t amb;
    int64_t nb = composite_pixel(px, py, tw, th, n, cnt, order, mean2d, conic, depth, opacity,
                                 rgb, tile_bbox, mask, mamb, bg, out, &T, &nc, &amb, NULL,
                                 band_rel);
    for (int ch = 0; ch < 3; ++ch) image[(int64_t)ch * W * H + o] = out[ch];
    if (T_final) T_final[o] = T;
    if (n_contrib) n_contrib[o] = nc;
    if (n_blended) n_blended[o] = (int32_t)nb;
    if (ambiguous) ambiguous[o] = amb;
  }
  free(order);
  free(mask);
  free(mamb);
}

/* Analytic backward of or_render over the window, decisions held fixed.
 * d_image [3][H][W].  Accumulates (+=) into the per-Gaussian SoA arrays
 * d_mean2d [2][n], d_conic [3][n], d_opacity [n], d_rgb [3][n].  abs_mass
 * [9][n] (may be NULL) receives the sum of |per-pixel contribution| of every
 * gradient element, amb_mass [9][n] (may be NULL) the same restricted to
 * ambiguous pixels (those whose ambiguity reason bits intersect amb_bits,
 * see composite_pixel); term_mass [9][n] (may be NULL) the sum over pixels
 * of the magnitudes of the terms before they cancel inside dL/dalpha (a
 * condition measure for FP32 comparisons); order of the 9: mean2d x,y,
 * conic 11,12,22, opacity, rgb.                                            */
void or_render_bwd(int64_t n, const double* mean2d, const double* conic, const double* depth,
                   const double* opacity, const double* rgb, const int32_t* tile_bbox,
                   const int32_t* valid, int W, int H, int tw, int th, const double* bg, int x0,
                   int y0, int x1, int y1, const double* d_image, double* d_mean2d,
                   double* d_conic, double* d_opacity, double* d_rgb, double* abs_mass,
                   double* amb_mass, int amb_bits, double* term_mass, double band_rel) {
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t cnt = sorted_order(n, depth, valid, order);
  int64_t npix = (int64_t)(x1 - x0) * (y1 - y0);
#pragma omp parallel
  {
    or_blend* rec = (or_blend*)malloc(sizeof(or_blend) * (size_t)(cnt > 0 ? cnt : 1));
#pragma omp for schedule(dynamic, 16)
    for (int64_t pi = 0; pi < npix; ++pi) {
      int px = x0 + (int)(pi % (x1 - x0)), py = y0 + (int)(pi / (x1 - x0));
      int64_t o = (int64_t)py * W + px;
      double out[3], Tf; int32_t nc; uint8_t amb;
      /* the gradients do not depend on which tiles list a pair that never
       * blends there, so the backward walks every bbox tile */
      int64_t nb = composite_pixel(px, py, tw, th, n, cnt, order, mean2d, conic, depth, opacity,
                                   rgb, tile_bbox, NULL, NULL, bg, out, &Tf, &nc, &amb, rec,
                                   band_rel);
      double dI[3];
      for (int ch = 0; ch < 3; ++ch) dI[ch] = d_image[(int64_t)ch * W * H + o];
      double acc[3];                      /* sum_{j>k} c_j a_j T_j + bg T_final */
      for (int ch = 0; ch < 3; ++ch) acc[ch] = bg[ch] * Tf;
      for (int64_t k = nb - 1; k >= 0; --k) {
        const or_blend* r = &rec[k];
        int64_t g = r->g;
        double contrib[9], terms[9];
        double dalpha = 0, dalpha_mag = 0;
        for (int ch = 0; ch < 3; ++ch) {
          double c = rgb[ch * n + g];
          contrib[6 + ch] = dI[ch] * r->alpha * r->T;
          terms[6 + ch] = fabs(contrib[6 + ch]);
          dalpha += dI[ch] * (c * r->T - acc[ch] / (1.0 - r->alpha));
          dalpha_mag += fabs(dI[ch]) * (fabs(c * r->T) + fabs(acc[ch] / (1.0 - r->alpha)));
          acc[ch] += c * r->alpha * r->T;
        }
        if (r->a < OR_ALPHA_MAX) {
          double dpower = dalpha * r->alpha;
          double q11 = conic[g], q12 = conic[n + g], q22 = conic[2 * n + g];
          contrib[0] = dpower * (q11 * r->dx + q12 * r->dy);
          contrib[1] = dpower * (q12 * r->dx + q22 * r->dy);
          contrib[2] = dpower * (-0.5 * r->dx * r->dx);
          contrib[3] = dpower * (-r->dx * r->dy);
          contrib[4] = dpower * (-0.5 * r->dy * r->dy);
          contrib[5] = dalpha * r->e;
          /* the same partials with |dL/dalpha| replaced by the magnitude of
           * its terms before they cancel */
          double m = dalpha_mag * r->alpha;
          terms[0] = m * fabs(q11 * r->dx + q12 * r->dy);
          terms[1] = m * fabs(q12 * r->dx + q22 * r->dy);
          terms[2] = m * 0.5 * r->dx * r->dx;
          terms[3] = m * fabs(r->dx * r->dy);
          terms[4] = m * 0.5 * r->dy * r->dy;
          terms[5] = dalpha_mag * r->e;
        } else {
          for (int k2 = 0; k2 < 6; ++k2) contrib[k2] = terms[k2] = 0.0;
        }
        double* dst[9] = {&d_mean2d[g], &d_mean2d[n + g], &d_conic[g], &d_conic[n + g],
                          &d_conic[2 * n + g], &d_opacity[g], &d_rgb[g], &d_rgb[n + g],
                          &d_rgb[2 * n + g]};
        for (int k2 = 0; k2 < 9; ++k2) {
#pragma omp atomic
          *dst[k2] += contrib[k2];
          if (abs_mass) {
#pragma omp atomic
            abs_mass[k2 * n + g] += fabs(contrib[k2]);
          }
          if (amb_mass && (amb & amb_bits)) {
#pragma omp atomic
            amb_mass[k2 * n + g] += fabs(contrib[k2]);
          }
          if (term_mass) {
#pragma omp atomic
            term_mass[k2 * n + g] += terms[k2];
          }
        }
      }
    }
    free(rec);
  }
  free(order);
}

/* ---------------------------------------------------------------------- */
/* Projection backward: chain rule to the Gaussian parameters               */
/* ---------------------------------------------------------------------- */

/* d_mean2d [2][n], d_conic [3][n], d_opacity [n], d_rgb [3][n] are the
 * gradients w.r.t. or_project's outputs; accumulates (+=) into the SoA
 * parameter gradients.  Invalid (culled) Gaussians receive nothing.        */
void or_project_bwd(int64_t n, const double* mean, const double* log_scale, const double* quat,
                    const double* opac_logit, const double* color, int sh_deg, const double* cam,
                    double znear, int W, int H, int tw, int th, const double* d_mean2d,
                    const double* d_conic, const double* d_opacity, const double* d_rgb,
                    double* g_mean, double* g_log_scale, double* g_quat, double* g_opac_logit,
                    double* g_color) {
  const double* Rv = cam;
  double fx = cam[12], fy = cam[13];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double mu[3] = {mean[i], mean[n + i], mean[2 * n + i]};
    double ls[3] = {log_scale[i], log_scale[n + i], log_scale[2 * n + i]};
    double q[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
    double f[3 * OR_SH_K];
    int K = (sh_deg + 1) * (sh_deg + 1);
    for (int r = 0; r < 3 * K; ++r) f[r] = color[r * n + i];
    or_proj P;
    project_one(mu, ls, q, opac_logit[i], f, sh_deg, cam, znear, W, H, tw, th, &P);
    if (!P.valid) continue;
    /* colour: rgb_c = max(0, sum_k Y_k(d) f_kc + 1/2); the derivative passes
     * where the argument is >= 0.  d = v/|v| moves with the mean:
     * dd/dv = (I - d d^T) / |v|.                                            */
    double gc[3], gdir[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < 3; ++c) gc[c] = P.pre_rgb[c] >= 0 ? d_rgb[c * n + i] : 0.0;
    for (int k = 0; k < K; ++k)
      for (int c = 0; c < 3; ++c) {
        g_color[(k * 3 + c) * n + i] += P.Y[k] * gc[c];
        for (int j = 0; j < 3; ++j) gdir[j] += gc[c] * f[k * 3 + c] * P.dY[k][j];
      }
    double dd = gdir[0] * P.dir[0] + gdir[1] * P.dir[1] + gdir[2] * P.dir[2];
    for (int j = 0; j < 3; ++j) g_mean[j * n + i] += (gdir[j] - P.dir[j] * dd) / P.vlen;
    /* opacity: o = sigmoid(w) */
    g_opac_logit[i] += P.o * (1.0 - P.o) * d_opacity[i];
    /* conic (Q11, Q12, Q22) = (c, -b, a) / det as functions of (a, b, c)   */
    double a = P.a, b = P.b, c = P.c, det = P.det, d2 = det * det;
    double dq11 = d_conic[i], dq12 = d_conic[n + i], dq22 = d_conic[2 * n + i];
    double da = dq11 * (-c * c / d2) + dq12 * (b * c / d2) + dq22 * (-b * b / d2);
    double db = dq11 * (2 * b * c / d2) + dq12 * (-(det + 2 * b * b) / d2) + dq22 * (2 * a * b / d2);
    double dc = dq11 * (-b * b / d2) + dq12 * (a * b / d2) + dq22 * (-a * a / d2);
    /* V = T Sigma T^T with symmetric gradient G (off-diagonal shares db)   */
    double G[4] = {da, 0.5 * db, 0.5 * db, dc};
    double dSigma[9];
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) {
        double acc = 0;
        for (int r = 0; r < 2; ++r)
          for (int s2 = 0; s2 < 2; ++s2) acc += P.T[r * 3 + k] * G[r * 2 + s2] * P.T[s2 * 3 + l];
        dSigma[k * 3 + l] = acc;
      }
    double dT[6];                       /* dL/dT = 2 G T Sigma (2x3)        */
    for (int r = 0; r < 2; ++r)
      for (int l = 0; l < 3; ++l) {
        double acc = 0;
        for (int s2 = 0; s2 < 2; ++s2)
          for (int k = 0; k < 3; ++k) acc += G[r * 2 + s2] * P.T[s2 * 3 + k] * P.Sigma[k * 3 + l];
        dT[r * 3 + l] = 2.0 * acc;
      }
    double dJ[6];                       /* T = J Rv  =>  dJ = dT Rv^T       */
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k) {
        double acc = 0;
        for (int l = 0; l < 3; ++l) acc += dT[r * 3 + l] * Rv[k * 3 + l];
        dJ[r * 3 + k] = acc;
      }
    double tx = P.t[0], ty = P.t[1], tz = P.t[2];
    double tz2 = tz * tz, tz3 = tz2 * tz;
    double dt[3] = {0, 0, 0};
    /* J00 = fx/tz, J11 = fy/tz */
    dt[2] += dJ[0] * (-fx / tz2) + dJ[4] * (-fy / tz2);
    /* J02 = -fx xc/tz^2 with xc = tx (free) or clamp*tz (clamped) */
    if (!P.xclamped) {
      dt[0] += dJ[2] * (-fx / tz2);
      dt[2] += dJ[2] * (2.0 * fx * tx / tz3);
    } else {
      dt[2] += dJ[2] * (fx * P.xclamp / tz3);
    }
    if (!P.yclamped) {
      dt[1] += dJ[5] * (-fy / tz2);
      dt[2] += dJ[5] * (2.0 * fy * ty / tz3);
    } else {
      dt[2] += dJ[5] * (fy * P.yclamp / tz3);
    }
    /* mean2d = (fx tx/tz + cx, fy ty/tz + cy) */
    double dmx = d_mean2d[i], dmy = d_mean2d[n + i];
    dt[0] += dmx * fx / tz;
    dt[1] += dmy * fy / tz;
    dt[2] += dmx * (-fx * tx / tz2) + dmy * (-fy * ty / tz2);
    /* t = Rv mu + tv  =>  dmu = Rv^T dt */
    for (int k = 0; k < 3; ++k)
      g_mean[k * n + i] += Rv[0 * 3 + k] * dt[0] + Rv[1 * 3 + k] * dt[1] + Rv[2 * 3 + k] * dt[2];
    /* Sigma = M M^T, M = R diag(s):  dM = 2 dSigma M (dSigma symmetric)    */
    double M[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) M[r * 3 + k] = P.R[r * 3 + k] * P.s[k];
    double dSs[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) dSs[r * 3 + k] = 0.5 * (dSigma[r * 3 + k] + dSigma[k * 3 + r]);
    double dM[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) {
        double acc = 0;
        for (int l = 0; l < 3; ++l) acc += dSs[r * 3 + l] * M[l * 3 + k];
        dM[r * 3 + k] = 2.0 * acc;
      }
    /* M_rk = R_rk s_k */
    for (int k = 0; k < 3; ++k) {
      double ds = 0;
      for (int r = 0; r < 3; ++r) ds += dM[r * 3 + k] * P.R[r * 3 + k];
      g_log_scale[k * n + i] += ds * P.s[k];
    }
    double dR[9];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) dR[r * 3 + k] = dM[r * 3 + k] * P.s[k];
    double w = P.qn[0], x = P.qn[1], y = P.qn[2], z = P.qn[3];
    double dqn[4];
    dqn[0] = dR[1] * (-2 * z) + dR[2] * (2 * y) + dR[3] * (2 * z) + dR[5] * (-2 * x) +
             dR[6] * (-2 * y) + dR[7] * (2 * x);
    dqn[1] = dR[1] * (2 * y) + dR[2] * (2 * z) + dR[3] * (2 * y) + dR[4] * (-4 * x) +
             dR[5] * (-2 * w) + dR[6] * (2 * z) + dR[7] * (2 * w) + dR[8] * (-4 * x);
    dqn[2] = dR[0] * (-4 * y) + dR[1] * (2 * x) + dR[2] * (2 * w) + dR[3] * (2 * x) +
             dR[5] * (2 * z) + dR[6] * (-2 * w) + dR[7] * (2 * z) + dR[8] * (-4 * y);
    dqn[3] = dR[0] * (-4 * z) + dR[1] * (-2 * w) + dR[2] * (2 * x) + dR[3] * (2 * w) +
             dR[4] * (-4 * z) + dR[5] * (2 * y) + dR[6] * (2 * x) + dR[7] * (2 * y);
    /* q^ = q/|q|  =>  dq = (dq^ - q^ (q^ . dq^)) / |q| */
    double dot = w * dqn[0] + x * dqn[1] + y * dqn[2] + z * dqn[3];
    for (int k = 0; k < 4; ++k) g_quat[k * n + i] += (dqn[k] - P.qn[k] * dot) / P.qnorm;
  }
}

/* ---------------------------------------------------------------------- */
/* Tile binning + sort                                                      */
/* ---------------------------------------------------------------------- */

typedef struct { uint64_t key; int64_t seq; uint32_t id; } or_dup;

static int cmp_dup(const void* A, const void* B) {
  const or_dup* a = (const or_dup*)A; const or_dup* b = (const or_dup*)B;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return (a->seq < b->seq) ? -1 : (a->seq > b->seq);
}

/* Emit every (pair, listed tile) entry in pair order, each pair's tiles
 * row-major over its bbox, with key ((slot * tiles_per_slot + ty * tiles_x
 * + tx) << 32) | depth_bits, then sort stably by key.  tile_bbox is
 * pair-major [m][4] (tx0, ty0, tx1, ty1), sup pair-major [m][6] (mean x, y,
 * conic a, b, c, opacity) decides the listed tiles (support_mask; NULL:
 * every bbox tile); pairs with n_tiles[p] == 0 emit nothing.  Writes up to cap entries to keys/ids
 * and the [start, end) ranges of every tile ([n_slots * tiles_per_slot][2],
 * zero for empty tiles), and per pair its entry count (count, may be NULL)
 * and whether any of its decisions is ambiguous at relative band `band`
 * (amb, may be NULL).  Returns the total count; if it exceeds cap nothing
 * is written to keys, ids and ranges.                                      */
int64_t or_bin_sort(int64_t m, const int32_t* tile_bbox, const int32_t* n_tiles,
                    const double* sup, int tw, int th, double band,
                    const uint32_t* depth_bits, const int32_t* slot, int tiles_x,
                    int tiles_per_slot, int n_slots, int64_t cap, uint64_t* keys, uint32_t* ids,
                    uint32_t* ranges, int32_t* count, uint8_t* amb) {
  uint64_t* mask = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
  int64_t total = 0;
  for (int64_t p = 0; p < m; ++p) {
    const int32_t* bb = tile_bbox + 4 * p;
    uint64_t am = 0;
    int64_t np = 0;
    mask[p] = 0;
    if (n_tiles[p] > 0) {
      int64_t area = (int64_t)(bb[2] - bb[0] + 1) * (bb[3] - bb[1] + 1);
      if (sup) {
        const double* r = sup + 6 * p;
        support_mask(r[0], r[1], r[2], r[3], r[4], r[5], bb[0], bb[1], bb[2], bb[3], tw, th,
                     band, &mask[p], &am);
      }
      np = (!sup || area > OR_MASK_TILES) ? area : (int64_t)__builtin_popcountll(mask[p]);
    }
    if (count) count[p] = (int32_t)np;
    if (amb) amb[p] = am != 0;
    total += np;
  }
  if (total > cap) { free(mask); return total; }
  or_dup* d = (or_dup*)malloc(sizeof(or_dup) * (size_t)(total > 0 ? total : 1));
  int64_t k = 0;
  for (int64_t p = 0; p < m; ++p) {
    if (n_tiles[p] <= 0) continue;
    const int32_t* bb = tile_bbox + 4 * p;
    int span = bb[2] - bb[0] + 1;
    int all = !sup || (int64_t)span * (bb[3] - bb[1] + 1) > OR_MASK_TILES;
    for (int ty = bb[1]; ty <= bb[3]; ++ty)
      for (int tx = bb[0]; tx <= bb[2]; ++tx) {
        if (!all && !(mask[p] >> ((ty - bb[1]) * span + (tx - bb[0])) & 1)) continue;
        uint64_t tile = (uint64_t)slot[p] * (uint64_t)tiles_per_slot + (uint64_t)(ty * tiles_x + tx);
        d[k].key = (tile << 32) | (uint64_t)depth_bits[p];
        d[k].seq = k;
        d[k].id = (uint32_t)p;
        ++k;
      }
  }
  qsort(d, (size_t)total, sizeof(or_dup), cmp_dup);
  int64_t ntile_all = (int64_t)n_slots * tiles_per_slot;
  memset(ranges, 0, sizeof(uint32_t) * 2 * (size_t)ntile_all);
  for (int64_t j = 0; j < total; ++j) {
    keys[j] = d[j].key;
    ids[j] = d[j].id;
    uint64_t tile = d[j].key >> 32;
    if (j == 0 || (d[j - 1].key >> 32) != tile) ranges[2 * tile] = (uint32_t)j;
    if (j == total - 1 || (d[j + 1].key >> 32) != tile) ranges[2 * tile + 1] = (uint32_t)(j + 1);
  }
  free(d);
  free(mask);
  return total;
}

/* ---------------------------------------------------------------------- */
/* Masked L1 + D-SSIM loss and its gradient                                 */
/* ---------------------------------------------------------------------- */

#define OR_SSIM_R 5
#define OR_SSIM_K 11

/* Normalised 11x11 Gaussian window (sigma 1.5) as the outer product of the
 * normalised 1D window.                                                    */
static void ssim_window(double w2[OR_SSIM_K][OR_SSIM_K]) {
  double w[OR_SSIM_K], s = 0;
  for (int k = 0; k < OR_SSIM_K; ++k) {
    double d = k - OR_SSIM_R;
    w[k] = exp(-d * d / (2.0 * 1.5 * 1.5));
    s += w[k];
  }
  for (int k = 0; k < OR_SSIM_K; ++k) w[k] /= s;
  for (int a = 0; a < OR_SSIM_K; ++a)
    for (int b = 0; b < OR_SSIM_K; ++b) w2[a][b] = w[a] * w[b];
}

/* One image: image, target [3][H][W], mask [H][W] (NULL = all ones).
 * Writes loss = (1-lambda) L1 + lambda (1 - SSIM), the L1 and SSIM terms,
 * d_image [3][H][W] = dloss/dimage and ssim_map [3][H][W] (both may be NULL).*/
void or_loss(const double* image, const double* target, const double* mask, int H, int W,
             double lambda, double* loss_out, double* l1_out, double* ssim_out, double* d_image,
             double* ssim_map) {
  const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  double w2[OR_SSIM_K][OR_SSIM_K];
  ssim_window(w2);
  int64_t P = (int64_t)H * W;
  double N = 3.0 * (double)P;
  double* x = (double*)malloc(sizeof(double) * 3 * P);
  double* y = (double*)malloc(sizeof(double) * 3 * P);
  for (int ch = 0; ch < 3; ++ch)
    for (int64_t p = 0; p < P; ++p) {
      double mk = mask ? mask[p] : 1.0;
      x[ch * P + p] = mk * image[ch * P + p];
      y[ch * P + p] = mk * target[ch * P + p];
    }
  double l1 = 0, ssim = 0;
  for (int64_t j = 0; j < 3 * P; ++j) l1 += fabs(x[j] - y[j]);
  /* per-pixel partials of S with respect to mu_x, E[x^2], E[xy]            */
  double* dmu = (double*)malloc(sizeof(double) * 3 * P);
  double* dxx = (double*)malloc(sizeof(double) * 3 * P);
  double* dxy = (double*)malloc(sizeof(double) * 3 * P);
  for (int ch = 0; ch < 3; ++ch) {
    const double* xc = x + ch * P; const double* yc = y + ch * P;
    double ssum = 0;
#pragma omp parallel for schedule(static) reduction(+ : ssum)
    for (int64_t p = 0; p < P; ++p) {
      int i = (int)(p % W), j = (int)(p / W);
      double mx = 0, my = 0, exx = 0, eyy = 0, exy = 0;
      for (int a = 0; a < OR_SSIM_K; ++a) {
        int jj = j + a - OR_SSIM_R;
        if (jj < 0 || jj >= H) continue;
        for (int b = 0; b < OR_SSIM_K; ++b) {
          int ii = i + b - OR_SSIM_R;
          if (ii < 0 || ii >= W) continue;
          double wv = w2[a][b];
          double xv = xc[(int64_t)jj * W + ii], yv = yc[(int64_t)jj * W + ii];
          mx += wv * xv; my += wv * yv;
          exx += wv * xv * xv; eyy += wv * yv * yv; exy += wv * xv * yv;
        }
      }
      double A1 = 2 * mx * my + C1, A2 = 2 * (exy - mx * my) + C2;
      double B1 = mx * mx + my * my + C1, B2 = (exx - mx * mx) + (eyy - my * my) + C2;
      double S = A1 * A2 / (B1 * B2);
      ssum += S;
      if (ssim_map) ssim_map[ch * P + p] = S;
      dmu[ch * P + p] = 2 * my * (A2 - A1) / (B1 * B2) - 2 * mx * S * (1.0 / B1 - 1.0 / B2);
      dxx[ch * P + p] = -S / B2;
      dxy[ch * P + p] = 2 * A1 / (B1 * B2);
    }
    ssim += ssum;
  }
  l1 /= N;
  ssim /= N;
  *loss_out = (1.0 - lambda) * l1 + lambda * (1.0 - ssim);
  if (l1_out) *l1_out = l1;
  if (ssim_out) *ssim_out = ssim;
  if (d_image) {
    for (int ch = 0; ch < 3; ++ch) {
      const double* xc = x + ch * P; const double* yc = y + ch * P;
#pragma omp parallel for schedule(static)
      for (int64_t q = 0; q < P; ++q) {
        int i = (int)(q % W), j = (int)(q / W);
        double gs = 0;                      /* sum_p dS(p)/dx(q)            */
        for (int a = 0; a < OR_SSIM_K; ++a) {
          int jj = j + a - OR_SSIM_R;      /* p = q + offset; w symmetric  */
          if (jj < 0 || jj >= H) continue;
          for (int b = 0; b < OR_SSIM_K; ++b) {
            int ii = i + b - OR_SSIM_R;
            if (ii < 0 || ii >= W) continue;
            int64_t pp = ch * P + (int64_t)jj * W + ii;
            gs += w2[a][b] * (dmu[pp] + 2.0 * xc[q] * dxx[pp] + yc[q] * dxy[pp]);
          }
        }
        double diff = xc[q] - yc[q];
        double sg = diff > 0 ? 1.0 : (diff < 0 ? -1.0 : 0.0);
        double dx = (1.0 - lambda) * sg / N - lambda * gs / N;
        double mk = mask ? mask[q] : 1.0;
        d_image[ch * P + q] = mk * dx;
      }
    }
  }
  free(x); free(y); free(dmu); free(dxx); free(dxy);
}

/* ---------------------------------------------------------------------- */
/* k nearest neighbours by brute force                                      */
/* ---------------------------------------------------------------------- */

/* pts [3][n]; for each point the k nearest other points sorted by
 * (distance, index): idx [n][k], dist [n][k] (Euclidean).                  */
void or_knn(int64_t n, const double* pts, int k, int32_t* idx, double* dist) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    double bd[64]; int64_t bi[64]; int cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = pts[j] - pts[i], dy = pts[n + j] - pts[n + i], dz = pts[2 * n + j] - pts[2 * n + i];
      double d2 = dx * dx + dy * dy + dz * dz;
      if (cnt == k && !(d2 < bd[k - 1] || (d2 == bd[k - 1] && j < bi[k - 1]))) continue;
      int pos = cnt < k ? cnt : k - 1;
      while (pos > 0 && (bd[pos - 1] > d2 || (bd[pos - 1] == d2 && bi[pos - 1] > j))) {
        bd[pos] = bd[pos - 1]; bi[pos] = bi[pos - 1]; --pos;
      }
      bd[pos] = d2; bi[pos] = j;
      if (cnt < k) ++cnt;
    }
    for (int r = 0; r < k; ++r) {
      idx[i * k + r] = r < cnt ? (int32_t)bi[r] : -1;
      dist[i * k + r] = r < cnt ? sqrt(bd[r]) : INFINITY;
    }
  }
}

int or_max_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
