/* vio_align.c -- CPU oracle of the realignment pre- and post-processing
 * (test infrastructure only; see vio.h).
 *
 * Paper anchors (Newson et al., "Video Inpainting of Complex Scenes"):
 *   Sec. 3.4, Alg. 2   dominant affine motion of every pair of successive
 *                       frames, composition to the middle frame, affine warp
 *                       of every frame and of the occlusion with linear
 *                       interpolation
 *   Sec. 3.4, Alg. 4   after inpainting, the inverse warp pasted into the
 *                       original occluded area
 *
 * The paper delegates the motion estimation to Odobez and Bouthemy's robust
 * multi-resolution estimator and gives no detail; the estimator here is
 * that method's usual form, written plainly (the readings are listed in the
 * design notes): grey level g = (R + G + B) / 3; a pyramid of 2x2 box means
 * with OR-pooled occlusions; at each level, from coarse to fine, a fixed
 * number of iteratively reweighted Gauss-Newton steps on the
 * brightness-constancy residual r(x) = g_{n+1}(x + w(x)) - g_n(x) with
 * Tukey's biweight (constant c), where w(x) = (p0 + p2 X + p3 Y,
 * p1 + p4 X + p5 Y) and (X, Y) are the level's coordinates relative to the
 * frame centre; gradients are central differences, sampled bilinearly at
 * the displaced position.  Everything is double precision, summed in pixel
 * order.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "vio.h"

int vio_align_params_default(vio_align_params* o) {
  if (!o) return VIO_E_INVAL;
  o->levels = 3;
  o->iters = 8;
  o->tukey_c = 20.0;
  return VIO_OK;
}

typedef struct {
  int W, H;
  double* g;   /* grey level */
  double* gx;  /* central differences, 0 on the border */
  double* gy;
  unsigned char* occ;
} glevel_t;

static void free_glevel(glevel_t* L) {
  free(L->g); free(L->gx); free(L->gy); free(L->occ);
}

/* the grey pyramid of one frame */
static int build_pyramid(const uint8_t* rgb, const uint8_t* mask, int W, int H, int levels,
                         glevel_t* P) {
  for (int l = 0; l < levels; ++l) {
    glevel_t* L = &P[l];
    L->W = l == 0 ? W : (P[l - 1].W + 1) / 2;
    L->H = l == 0 ? H : (P[l - 1].H + 1) / 2;
    size_t n = (size_t)L->W * L->H;
    L->g = (double*)calloc(n, sizeof(double));
    L->gx = (double*)calloc(n, sizeof(double));
    L->gy = (double*)calloc(n, sizeof(double));
    L->occ = (unsigned char*)calloc(n, 1);
    if (!L->g || !L->gx || !L->gy || !L->occ) return VIO_E_NOMEM;
    if (l == 0) {
      for (size_t i = 0; i < n; ++i) {
        L->occ[i] = mask[i] ? 1 : 0;
        L->g[i] = L->occ[i] ? 0.0
                            : ((double)rgb[3 * i] + (double)rgb[3 * i + 1] + (double)rgb[3 * i + 2]) /
                                  3.0;
      }
    } else {
      const glevel_t* F = &P[l - 1];
      for (int y = 0; y < L->H; ++y)
        for (int x = 0; x < L->W; ++x) {
          double s = 0.0;
          int cnt = 0, any = 0;
          for (int by = 0; by < 2; ++by)
            for (int bx = 0; bx < 2; ++bx) {
              int fx = 2 * x + bx, fy = 2 * y + by;
              if (fx >= F->W || fy >= F->H) continue;
              any |= F->occ[(size_t)fy * F->W + fx];
              s += F->g[(size_t)fy * F->W + fx];
              cnt++;
            }
          L->occ[(size_t)y * L->W + x] = (unsigned char)any;
          L->g[(size_t)y * L->W + x] = any ? 0.0 : s / (double)cnt;
        }
    }
    for (int y = 1; y < L->H - 1; ++y)
      for (int x = 1; x < L->W - 1; ++x) {
        size_t i = (size_t)y * L->W + x;
        L->gx[i] = (L->g[i + 1] - L->g[i - 1]) / 2.0;
        L->gy[i] = (L->g[i + L->W] - L->g[i - L->W]) / 2.0;
      }
  }
  return VIO_OK;
}

/* bilinear sample of a level array at (xs, ys), 0 <= floor < size - 1 */
static double bilin(const double* a, int W, int x0, int y0, double fx, double fy) {
  const double* r0 = a + (size_t)y0 * W + x0;
  const double* r1 = r0 + W;
  return (1.0 - fx) * (1.0 - fy) * r0[0] + fx * (1.0 - fy) * r0[1] + (1.0 - fx) * fy * r1[0] +
         fx * fy * r1[1];
}

/* solves the symmetric 6x6 system A d = b by Gaussian elimination with
 * partial pivoting; returns 0 if it is singular */
static int solve6(double A[6][6], double b[6], double d[6]) {
  double M[6][7];
  for (int i = 0; i < 6; ++i) {
    for (int j = 0; j < 6; ++j) M[i][j] = A[i][j];
    M[i][6] = b[i];
  }
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (fabs(M[piv][c]) < 1e-9) return 0;
    if (piv != c)
      for (int j = 0; j < 7; ++j) {
        double t = M[c][j];
        M[c][j] = M[piv][j];
        M[piv][j] = t;
      }
    for (int r = c + 1; r < 6; ++r) {
      double f = M[r][c] / M[c][c];
      for (int j = c; j < 7; ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int r = 5; r >= 0; --r) {
    double s = M[r][6];
    for (int j = r + 1; j < 6; ++j) s -= M[r][j] * d[j];
    d[r] = s / M[r][r];
  }
  return 1;
}

/* One robust Gauss-Newton step of the pair (a -> b) at a level: the normal
 * equations accumulated over every valid pixel of frame a, solved, and the
 * increment added to p. */
static void gn_step(const glevel_t* a, const glevel_t* b, double c, double p[6]) {
  const int W = a->W, H = a->H;
  const double cx = (W - 1) / 2.0, cy = (H - 1) / 2.0;
  double A[6][6], g[6];
  memset(A, 0, sizeof(A));
  memset(g, 0, sizeof(g));
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      size_t i = (size_t)y * W + x;
      if (a->occ[i]) continue;
      const double X = x - cx, Y = y - cy;
      const double u = p[0] + p[2] * X + p[3] * Y;
      const double v = p[1] + p[4] * X + p[5] * Y;
      const double xs = x + u, ys = y + v;
      /* the 2x2 stencil and its central differences must be defined */
      if (!(xs >= 1.0 && xs < W - 2.0 && ys >= 1.0 && ys < H - 2.0)) continue;
      const int x0 = (int)floor(xs), y0 = (int)floor(ys);
      const double fx = xs - x0, fy = ys - y0;
      const size_t j = (size_t)y0 * W + x0;
      if (b->occ[j] || b->occ[j + 1] || b->occ[j + W] || b->occ[j + W + 1]) continue;
      const double I2 = bilin(b->g, W, x0, y0, fx, fy);
      const double Gx = bilin(b->gx, W, x0, y0, fx, fy);
      const double Gy = bilin(b->gy, W, x0, y0, fx, fy);
      const double r = I2 - a->g[i];
      if (fabs(r) >= c) continue; /* Tukey: zero weight */
      const double q = 1.0 - (r / c) * (r / c);
      const double w = q * q;
      const double J[6] = {Gx, Gy, Gx * X, Gx * Y, Gy * X, Gy * Y};
      for (int m = 0; m < 6; ++m) {
        for (int k = 0; k < 6; ++k) A[m][k] += w * J[m] * J[k];
        g[m] += w * J[m] * r;
      }
    }
  double d[6], mg[6];
  for (int m = 0; m < 6; ++m) mg[m] = -g[m];
  if (!solve6(A, mg, d)) return;
  for (int m = 0; m < 6; ++m) p[m] += d[m];
}

int vio_align_estimate(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H,
                       int32_t T, const vio_align_params* prm, double* theta) {
  if (!rgb || !mask || !prm || !theta || T < 2 || W < 8 || H < 8) return VIO_E_INVAL;
  if (prm->levels < 1 || prm->levels > 8 || prm->iters < 0 || !(prm->tukey_c > 0.0))
    return VIO_E_INVAL;
  const int Lm = prm->levels;
  {
    int w = W, h = H;
    for (int l = 1; l < Lm; ++l) {
      w = (w + 1) / 2;
      h = (h + 1) / 2;
    }
    if (w < 8 || h < 8) return VIO_E_INVAL;
  }
  glevel_t* P = (glevel_t*)calloc((size_t)T * Lm, sizeof(glevel_t));
  if (!P) return VIO_E_NOMEM;
  int st = VIO_OK;
  const size_t fr = (size_t)W * H;
  for (int t = 0; t < T && st == VIO_OK; ++t)
    st = build_pyramid(rgb + 3 * fr * t, mask + fr * t, W, H, Lm, P + (size_t)t * Lm);
  if (st == VIO_OK) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < T - 1; ++n) {
      double p[6] = {0, 0, 0, 0, 0, 0};
      for (int l = Lm - 1; l >= 0; --l) {
        const glevel_t* a = &P[(size_t)n * Lm + l];
        const glevel_t* b = &P[(size_t)(n + 1) * Lm + l];
        for (int k = 0; k < prm->iters; ++k) gn_step(a, b, prm->tukey_c, p);
        if (l > 0) { /* to the finer level: translations double */
          p[0] *= 2.0;
          p[1] *= 2.0;
        }
      }
      /* absolute form: x' = x + u(x) with (X, Y) relative to the centre */
      const double cx = (W - 1) / 2.0, cy = (H - 1) / 2.0;
      double* th = theta + 6 * (size_t)n;
      th[0] = 1.0 + p[2];
      th[1] = p[3];
      th[2] = p[0] - p[2] * cx - p[3] * cy;
      th[3] = p[4];
      th[4] = 1.0 + p[5];
      th[5] = p[1] - p[4] * cx - p[5] * cy;
    }
  }
  for (size_t i = 0; i < (size_t)T * Lm; ++i) free_glevel(&P[i]);
  free(P);
  return st;
}

/* c = a o b for affine maps [m0 m1 m2; m3 m4 m5] (x' = m0 x + m1 y + m2,
 * y' = m3 x + m4 y + m5): c(x) = a(b(x)) */
static void compose(const double a[6], const double b[6], double c[6]) {
  double r[6];
  r[0] = a[0] * b[0] + a[1] * b[3];
  r[1] = a[0] * b[1] + a[1] * b[4];
  r[2] = a[0] * b[2] + a[1] * b[5] + a[2];
  r[3] = a[3] * b[0] + a[4] * b[3];
  r[4] = a[3] * b[1] + a[4] * b[4];
  r[5] = a[3] * b[2] + a[4] * b[5] + a[5];
  memcpy(c, r, sizeof(r));
}

int vio_affine_inverse(const double m[6], double inv[6]) {
  const double det = m[0] * m[4] - m[1] * m[3];
  if (!(fabs(det) > 1e-12)) return VIO_E_INVAL;
  inv[0] = m[4] / det;
  inv[1] = -m[1] / det;
  inv[3] = -m[3] / det;
  inv[4] = m[0] / det;
  inv[2] = -(inv[0] * m[2] + inv[1] * m[5]);
  inv[5] = -(inv[3] * m[2] + inv[4] * m[5]);
  return VIO_OK;
}

int vio_align_compose(const double* theta, int32_t T, double* M) {
  if (!theta || !M || T < 1) return VIO_E_INVAL;
  const int ref = T / 2;
  const double id[6] = {1, 0, 0, 0, 1, 0};
  memcpy(M + 6 * (size_t)ref, id, sizeof(id));
  /* frames before the reference: M_n = theta_{ref-1} o ... o theta_n */
  for (int n = ref - 1; n >= 0; --n) compose(M + 6 * (size_t)(n + 1), theta + 6 * (size_t)n,
                                             M + 6 * (size_t)n);
  /* frames after it: M_n = theta_ref^-1 o ... o theta_{n-1}^-1 */
  for (int n = ref + 1; n < T; ++n) {
    double inv[6];
    if (vio_affine_inverse(theta + 6 * (size_t)(n - 1), inv)) return VIO_E_INVAL;
    compose(M + 6 * (size_t)(n - 1), inv, M + 6 * (size_t)n);
  }
  return VIO_OK;
}

/* one bilinear sample of an RGB frame at (xs, ys) with the neighbours of
 * nonzero weight required inside the frame and (when occ is given) not
 * occluded; returns 0 and leaves out untouched otherwise */
static int sample_rgb(const uint8_t* fr, const uint8_t* occ, int W, int H, double xs, double ys,
                      uint8_t out[3]) {
  const double fl_x = floor(xs), fl_y = floor(ys);
  if (!(fl_x >= 0.0 && fl_y >= 0.0 && fl_x <= W - 1.0 && fl_y <= H - 1.0)) return 0;
  const int x0 = (int)fl_x, y0 = (int)fl_y;
  const double fx = xs - fl_x, fy = ys - fl_y;
  const double w[4] = {(1.0 - fx) * (1.0 - fy), fx * (1.0 - fy), (1.0 - fx) * fy, fx * fy};
  const int dx[4] = {0, 1, 0, 1}, dy[4] = {0, 0, 1, 1};
  double acc[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 4; ++k) {
    if (!(w[k] > 0.0)) continue;
    const int xx = x0 + dx[k], yy = y0 + dy[k];
    if (xx > W - 1 || yy > H - 1) return 0;
    const size_t i = (size_t)yy * W + xx;
    if (occ && occ[i]) return 0;
    for (int c = 0; c < 3; ++c) acc[c] += w[k] * (double)fr[3 * i + c];
  }
  for (int c = 0; c < 3; ++c) {
    double q = floor(acc[c] + 0.5);
    out[c] = (uint8_t)(q < 0.0 ? 0.0 : (q > 255.0 ? 255.0 : q));
  }
  return 1;
}

int vio_align_warp(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H, int32_t T,
                   const double* M, uint8_t* out_rgb, uint8_t* out_mask) {
  if (!rgb || !mask || !M || !out_rgb || !out_mask || W < 1 || H < 1 || T < 1)
    return VIO_E_INVAL;
  const size_t fr = (size_t)W * H;
  for (int t = 0; t < T; ++t) {
    double inv[6];
    if (vio_affine_inverse(M + 6 * (size_t)t, inv)) return VIO_E_INVAL;
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        /* the frame's pixel that the reference position (x, y) shows */
        const double xs = (inv[0] * x + inv[1] * y) + inv[2];
        const double ys = (inv[3] * x + inv[4] * y) + inv[5];
        const size_t o = fr * t + (size_t)y * W + x;
        uint8_t v[3] = {0, 0, 0};
        const int ok = sample_rgb(rgb + 3 * fr * t, mask + fr * t, W, H, xs, ys, v);
        out_mask[o] = (uint8_t)(ok ? 0 : 1);
        for (int c = 0; c < 3; ++c) out_rgb[3 * o + c] = ok ? v[c] : 0;
      }
  }
  return VIO_OK;
}

int vio_align_unwarp(const uint8_t* aligned, const uint8_t* rgb, const uint8_t* mask, int32_t W,
                     int32_t H, int32_t T, const double* M, uint8_t* out_rgb) {
  if (!aligned || !rgb || !mask || !M || !out_rgb || W < 1 || H < 1 || T < 1)
    return VIO_E_INVAL;
  const size_t fr = (size_t)W * H;
  memcpy(out_rgb, rgb, 3 * fr * (size_t)T);
  for (int t = 0; t < T; ++t) {
    const double* m = M + 6 * (size_t)t;
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        const size_t o = fr * t + (size_t)y * W + x;
        if (!mask[o]) continue;
        /* the reference position of the occluded pixel, clamped to the frame */
        double xs = (m[0] * x + m[1] * y) + m[2];
        double ys = (m[3] * x + m[4] * y) + m[5];
        xs = xs < 0.0 ? 0.0 : (xs > W - 1.0 ? W - 1.0 : xs);
        ys = ys < 0.0 ? 0.0 : (ys > H - 1.0 ? H - 1.0 : ys);
        uint8_t v[3];
        sample_rgb(aligned + 3 * fr * t, NULL, W, H, xs, ys, v);
        for (int c = 0; c < 3; ++c) out_rgb[3 * o + c] = v[c];
      }
  }
  return VIO_OK;
}
