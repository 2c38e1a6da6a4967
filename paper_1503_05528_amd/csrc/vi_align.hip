// vi_align.hip -- realignment of a video filmed by a moving camera
// (Newson et al., Sec. 3.4, Alg. 2; the inverse warp of Alg. 4).
//
// The dominant affine motion of every pair of successive frames is found by
// a robust coarse-to-fine Gauss-Newton fit of the brightness-constancy
// residual r(x) = g_{n+1}(x + w(x)) - g_n(x) (grey g = (R+G+B)/3, Tukey
// biweight, w affine in the coordinates relative to the frame centre).  All
// pairs advance together: one kernel evaluates every pixel of every pair and
// writes per-workgroup partial sums of the 6x6 normal equations, and one
// workgroup per pair sums them in a fixed order, solves the 6x6 system and
// updates the pair's parameters; every step of every level is enqueued at
// once (double precision throughout).  The warp and its inverse are pixel-parallel
// bilinear resampling kernels in double precision with the products and sums
// rounded one by one (no fused multiply-add), so that they reproduce the same
// arithmetic sequence wherever the same map is applied.
#include <hip/hip_runtime.h>

#include <cmath>
#include <utility>
#include <cstring>
#include <string>
#include <vector>

#include "vi.h"
#include "vi_internal.h"

// every product and sum rounded on its own, on the host as on the device
#pragma clang fp contract(off)

namespace vi {
namespace {

constexpr int kAB = 256;        // threads per workgroup
constexpr int kSums = 27;       // 21 entries of the symmetric 6x6 matrix + 6 of the right side
constexpr int kPixPerThread = 8;

struct GLevel {
  int32_t W, H;
  double* g;    // [T][H][W] grey
  double* gx;   // central differences (0 on the border)
  double* gy;
  uint8_t* occ; // OR-pooled occlusion
};

// Pixel kernels run on (x blocks, y, t) grids: no integer division per
// pixel.
__global__ void k_grey0(const uint8_t* __restrict__ rgb, const uint8_t* __restrict__ mask,
                        int32_t W, int32_t H, double* __restrict__ g, uint8_t* __restrict__ occ) {
  const int32_t x = blockIdx.x * kAB + threadIdx.x;
  if (x >= W) return;
  const int64_t i = ((int64_t)blockIdx.z * H + blockIdx.y) * W + x;
  const uint8_t o = mask[i] ? 1 : 0;
  occ[i] = o;
  const double s = __dadd_rn(__dadd_rn((double)rgb[3 * i], (double)rgb[3 * i + 1]),
                             (double)rgb[3 * i + 2]);
  g[i] = o ? 0.0 : s / 3.0;
}

__global__ void k_grey_down(GLevel F, GLevel C) {
  const int32_t x = blockIdx.x * kAB + threadIdx.x;
  if (x >= C.W) return;
  const int32_t y = blockIdx.y;
  const int64_t t = blockIdx.z;
  const int64_t i = (t * C.H + y) * C.W + x;
  double s = 0.0;
  int cnt = 0, any = 0;
  for (int by = 0; by < 2; ++by)
    for (int bx = 0; bx < 2; ++bx) {
      const int32_t fx = 2 * x + bx, fy = 2 * y + by;
      if (fx >= F.W || fy >= F.H) continue;
      const int64_t j = (t * F.H + fy) * F.W + fx;
      any |= F.occ[j];
      s = __dadd_rn(s, F.g[j]);
      ++cnt;
    }
  C.occ[i] = (uint8_t)any;
  C.g[i] = any ? 0.0 : s / (double)cnt;
}

__global__ void k_grey_grad(GLevel L) {
  const int32_t x = blockIdx.x * kAB + threadIdx.x;
  if (x >= L.W) return;
  const int32_t y = blockIdx.y;
  const int64_t i = ((int64_t)blockIdx.z * L.H + y) * L.W + x;
  double gx = 0.0, gy = 0.0;
  if (x >= 1 && x < L.W - 1 && y >= 1 && y < L.H - 1) {
    gx = __dsub_rn(L.g[i + 1], L.g[i - 1]) / 2.0;
    gy = __dsub_rn(L.g[i + L.W], L.g[i - L.W]) / 2.0;
  }
  L.gx[i] = gx;
  L.gy[i] = gy;
}

__device__ __forceinline__ double bilin(const double* a, int32_t W, int64_t j, double fx,
                                        double fy) {
  const double w00 = __dmul_rn(1.0 - fx, 1.0 - fy), w10 = __dmul_rn(fx, 1.0 - fy);
  const double w01 = __dmul_rn(1.0 - fx, fy), w11 = __dmul_rn(fx, fy);
  double s = __dmul_rn(w00, a[j]);
  s = __dadd_rn(s, __dmul_rn(w10, a[j + 1]));
  s = __dadd_rn(s, __dmul_rn(w01, a[j + W]));
  return __dadd_rn(s, __dmul_rn(w11, a[j + W + 1]));
}

// Partial normal equations of one workgroup: pair n = blockIdx.y, pixels
// blockIdx.x * kAB * kPixPerThread ... of frame n.  out[(n * nblk + b) * 27].
__global__ __launch_bounds__(kAB) void k_gn_partial(GLevel L, const double* __restrict__ P,
                                                    double c, int32_t nblk,
                                                    double* __restrict__ out) {
  const int32_t n = blockIdx.y;
  const int32_t fr = L.W * L.H;
  const double* p = P + 6 * n;
  const double cx = (L.W - 1) / 2.0, cy = (L.H - 1) / 2.0;
  double acc[kSums];
#pragma unroll
  for (int k = 0; k < kSums; ++k) acc[k] = 0.0;
  const int32_t base = blockIdx.x * kAB * kPixPerThread;
  for (int r = 0; r < kPixPerThread; ++r) {
    const int32_t i = base + r * kAB + (int32_t)threadIdx.x;
    if (i >= fr) break;
    const int64_t ia = (int64_t)n * fr + i;
    if (L.occ[ia]) continue;
    const int32_t y = i / L.W, x = i - y * L.W;
    const double X = x - cx, Y = y - cy;
    const double u = p[0] + p[2] * X + p[3] * Y;
    const double v = p[1] + p[4] * X + p[5] * Y;
    const double xs = x + u, ys = y + v;
    if (!(xs >= 1.0 && xs < L.W - 2.0 && ys >= 1.0 && ys < L.H - 2.0)) continue;
    const int32_t x0 = (int32_t)floor(xs), y0 = (int32_t)floor(ys);
    const double fx = xs - x0, fy = ys - y0;
    const int64_t j = (int64_t)(n + 1) * fr + (int64_t)y0 * L.W + x0;
    if (L.occ[j] | L.occ[j + 1] | L.occ[j + L.W] | L.occ[j + L.W + 1]) continue;
    const double I2 = bilin(L.g, L.W, j, fx, fy);
    const double Gx = bilin(L.gx, L.W, j, fx, fy);
    const double Gy = bilin(L.gy, L.W, j, fx, fy);
    const double res = I2 - L.g[ia];
    if (fabs(res) >= c) continue;
    const double q = 1.0 - (res / c) * (res / c);
    const double w = q * q;
    const double J[6] = {Gx, Gy, Gx * X, Gx * Y, Gy * X, Gy * Y};
    int k = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) acc[k++] += w * J[a] * J[b];
#pragma unroll
    for (int a = 0; a < 6; ++a) acc[21 + a] += w * J[a] * res;
  }
  // workgroup sums in a fixed order: wave sums with xor shuffles, then the
  // four waves in order
  __shared__ double s_w[kAB / 64][kSums];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kSums; ++k) {
    double v = acc[k];
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) s_w[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kSums) {
    double v = 0.0;
    for (int w = 0; w < kAB / 64; ++w) v += s_w[w][threadIdx.x];
    out[((int64_t)n * nblk + blockIdx.x) * kSums + threadIdx.x] = v;
  }
}

// Gaussian elimination with partial pivoting of the 6x6 system A d = b;
// false if singular
__device__ bool solve6(double A[6][6], const double b[6], double d[6]) {
  double M[6][7];
  for (int i = 0; i < 6; ++i) {
    for (int j = 0; j < 6; ++j) M[i][j] = A[i][j];
    M[i][6] = b[i];
  }
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (fabs(M[piv][c]) < 1e-9) return false;
    if (piv != c)
      for (int j = 0; j < 7; ++j) {
        const double t = M[c][j];
        M[c][j] = M[piv][j];
        M[piv][j] = t;
      }
    for (int r = c + 1; r < 6; ++r) {
      const double f = M[r][c] / M[c][c];
      for (int j = c; j < 7; ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int r = 5; r >= 0; --r) {
    double s = M[r][6];
    for (int j = r + 1; j < 6; ++j) s -= M[r][j] * d[j];
    d[r] = s / M[r][r];
  }
  return true;
}

// One workgroup per pair: the pair's workgroup partial sums added in
// workgroup order, the 6x6 system solved and the increment added to the
// pair's parameters; `scale` doubles the translations afterwards (the step
// to the next finer level).
__global__ __launch_bounds__(64) void k_gn_solve(const double* __restrict__ part, int32_t nblk,
                                                 double* __restrict__ P, int32_t scale) {
  const int32_t n = blockIdx.x;
  __shared__ double s[kSums];
  if (threadIdx.x < kSums) {
    double v = 0.0;
    for (int32_t b = 0; b < nblk; ++b) v += part[((int64_t)n * nblk + b) * kSums + threadIdx.x];
    s[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double A[6][6], rhs[6], d[6];
  int q = 0;
  for (int a = 0; a < 6; ++a)
    for (int c2 = a; c2 < 6; ++c2) {
      A[a][c2] = s[q];
      A[c2][a] = s[q];
      ++q;
    }
  for (int a = 0; a < 6; ++a) rhs[a] = -s[21 + a];
  double* p = P + 6 * n;
  if (solve6(A, rhs, d))
    for (int a = 0; a < 6; ++a) p[a] += d[a];
  if (scale) {
    p[0] *= 2.0;
    p[1] *= 2.0;
  }
}

// The bilinear sample of an RGB frame at (xs, ys): neighbours of nonzero
// weight must lie inside the frame and (occ given) not be occluded.
__device__ __forceinline__ bool sample_rgb(const uint8_t* __restrict__ fr,
                                           const uint8_t* __restrict__ occ, int32_t W, int32_t H,
                                           double xs, double ys, uint32_t out[3]) {
  const double flx = floor(xs), fly = floor(ys);
  // written so that a NaN position is refused as well
  if (!(flx >= 0.0 && fly >= 0.0 && flx <= W - 1.0 && fly <= H - 1.0)) return false;
  const int32_t x0 = (int32_t)flx, y0 = (int32_t)fly;
  const double fx = __dsub_rn(xs, flx), fy = __dsub_rn(ys, fly);
  const double w[4] = {__dmul_rn(__dsub_rn(1.0, fx), __dsub_rn(1.0, fy)),
                       __dmul_rn(fx, __dsub_rn(1.0, fy)),
                       __dmul_rn(__dsub_rn(1.0, fx), fy), __dmul_rn(fx, fy)};
  double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (!(w[k] > 0.0)) continue;
    const int32_t xx = x0 + (k & 1), yy = y0 + (k >> 1);
    if (xx > W - 1 || yy > H - 1) return false;
    const int64_t i = (int64_t)yy * W + xx;
    if (occ && occ[i]) return false;
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = __dadd_rn(acc[c], __dmul_rn(w[k], (double)fr[3 * i + c]));
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double q = floor(__dadd_rn(acc[c], 0.5));
    out[c] = (uint32_t)(q < 0.0 ? 0.0 : (q > 255.0 ? 255.0 : q));
  }
  return true;
}

// the frame position (m0 x + m1 y) + m2, (m3 x + m4 y) + m5
__device__ __forceinline__ void apply(const double* m, int32_t x, int32_t y, double& xs,
                                      double& ys) {
  xs = __dadd_rn(__dadd_rn(__dmul_rn(m[0], (double)x), __dmul_rn(m[1], (double)y)), m[2]);
  ys = __dadd_rn(__dadd_rn(__dmul_rn(m[3], (double)x), __dmul_rn(m[4], (double)y)), m[5]);
}

__global__ void k_warp(const uint8_t* __restrict__ rgb, const uint8_t* __restrict__ mask,
                       int32_t W, int32_t H, int32_t T, const double* __restrict__ Minv,
                       uint8_t* __restrict__ out_rgb, uint8_t* __restrict__ out_mask) {
  const int64_t fr = (int64_t)W * H;
  const int32_t x = blockIdx.x * kAB + threadIdx.x;
  if (x >= W) return;
  const int32_t y = blockIdx.y;
  const int64_t t = blockIdx.z;
  const int64_t i = t * fr + (int64_t)y * W + x;
  double xs, ys;
  apply(Minv + 6 * t, x, y, xs, ys);
  uint32_t v[3] = {0, 0, 0};
  const bool ok = sample_rgb(rgb + 3 * fr * t, mask + fr * t, W, H, xs, ys, v);
  out_mask[i] = ok ? 0 : 1;
  out_rgb[3 * i] = ok ? (uint8_t)v[0] : 0;
  out_rgb[3 * i + 1] = ok ? (uint8_t)v[1] : 0;
  out_rgb[3 * i + 2] = ok ? (uint8_t)v[2] : 0;
}

__global__ void k_unwarp(const uint8_t* __restrict__ aligned, const uint8_t* __restrict__ rgb,
                         const uint8_t* __restrict__ mask, int32_t W, int32_t H, int32_t T,
                         const double* __restrict__ M, uint8_t* __restrict__ out) {
  const int64_t fr = (int64_t)W * H;
  const int32_t x = blockIdx.x * kAB + threadIdx.x;
  if (x >= W) return;
  const int32_t y = blockIdx.y;
  const int64_t t = blockIdx.z;
  const int64_t i = t * fr + (int64_t)y * W + x;
  if (!mask[i]) {
    out[3 * i] = rgb[3 * i];
    out[3 * i + 1] = rgb[3 * i + 1];
    out[3 * i + 2] = rgb[3 * i + 2];
    return;
  }
  double xs, ys;
  apply(M + 6 * t, x, y, xs, ys);
  xs = xs < 0.0 ? 0.0 : (xs > W - 1.0 ? W - 1.0 : xs);
  ys = ys < 0.0 ? 0.0 : (ys > H - 1.0 ? H - 1.0 : ys);
  uint32_t v[3] = {0, 0, 0};
  sample_rgb(aligned + 3 * fr * t, nullptr, W, H, xs, ys, v);
  out[3 * i] = (uint8_t)v[0];
  out[3 * i + 1] = (uint8_t)v[1];
  out[3 * i + 2] = (uint8_t)v[2];
}

// x blocks of kAB pixels, one row per y, one frame per z
inline dim3 grid3(int32_t W, int32_t H, int32_t T) {
  return dim3((unsigned)((W + kAB - 1) / kAB), (unsigned)H, (unsigned)T);
}

// the inverse of an affine map; false if singular
bool inverse(const double* m, double* inv) {
  const double det = m[0] * m[4] - m[1] * m[3];
  if (!(std::fabs(det) > 1e-12)) return false;
  inv[0] = m[4] / det;
  inv[1] = -m[1] / det;
  inv[3] = -m[3] / det;
  inv[4] = m[0] / det;
  inv[2] = -(inv[0] * m[2] + inv[1] * m[5]);
  inv[5] = -(inv[3] * m[2] + inv[4] * m[5]);
  return true;
}

// c = a o b
void compose(const double* a, const double* b, double* c) {
  double r[6];
  r[0] = a[0] * b[0] + a[1] * b[3];
  r[1] = a[0] * b[1] + a[1] * b[4];
  r[2] = a[0] * b[2] + a[1] * b[5] + a[2];
  r[3] = a[3] * b[0] + a[4] * b[3];
  r[4] = a[3] * b[1] + a[4] * b[4];
  r[5] = a[3] * b[2] + a[4] * b[5] + a[5];
  std::memcpy(c, r, sizeof(r));
}

}  // namespace

// ---------------------------------------------------------------- host entry

vi_status align_estimate(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H, int32_t T,
                         const vi_align_params* prm, double* theta, hipStream_t st,
                         std::string* err) {
  const int Lm = prm->levels;
  const int64_t fr0 = (int64_t)W * H;
  std::vector<GLevel> lv((size_t)Lm);
  std::vector<void*> blocks;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (void* p : blocks) (void)hipFree(p);
  };
  auto dmalloc = [&](void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) return false;
    blocks.push_back(*p);
    return true;
  };
  int32_t w = W, h = H;
  for (int l = 0; l < Lm; ++l) {
    lv[(size_t)l].W = w;
    lv[(size_t)l].H = h;
    const size_t n = (size_t)w * h * (size_t)T;
    GLevel& L = lv[(size_t)l];
    if (!dmalloc((void**)&L.g, 8 * n) || !dmalloc((void**)&L.gx, 8 * n) ||
        !dmalloc((void**)&L.gy, 8 * n) || !dmalloc((void**)&L.occ, n)) {
      cleanup();
      *err = "device allocation failed";
      return VI_E_NOMEM;
    }
    w = (w + 1) / 2;
    h = (h + 1) / 2;
  }
  k_grey0<<<grid3(W, H, T), kAB, 0, st>>>(rgb, mask, W, H, lv[0].g, lv[0].occ);
  for (int l = 1; l < Lm; ++l)
    k_grey_down<<<grid3(lv[(size_t)l].W, lv[(size_t)l].H, T), kAB, 0, st>>>(
        lv[(size_t)l - 1], lv[(size_t)l]);
  for (int l = 0; l < Lm; ++l)
    k_grey_grad<<<grid3(lv[(size_t)l].W, lv[(size_t)l].H, T), kAB, 0, st>>>(lv[(size_t)l]);
  const int32_t np = T - 1;
  const int64_t per_blk = (int64_t)kAB * kPixPerThread;
  const int32_t nblk_max = (int32_t)((fr0 + per_blk - 1) / per_blk);
  double *d_p = nullptr, *d_part = nullptr;
  if (!dmalloc((void**)&d_p, sizeof(double) * 6 * (size_t)np) ||
      !dmalloc((void**)&d_part, sizeof(double) * kSums * (size_t)np * (size_t)nblk_max)) {
    cleanup();
    *err = "device allocation failed";
    return VI_E_NOMEM;
  }
  std::vector<double> p((size_t)6 * np, 0.0);
  if (hipMemcpyAsync(d_p, p.data(), sizeof(double) * p.size(), hipMemcpyHostToDevice, st) !=
      hipSuccess) {
    cleanup();
    *err = "parameter upload failed";
    return VI_E_HIP;
  }
  // every step of every level is enqueued at once: the partial sums, then
  // one workgroup per pair that solves and updates the pair's parameters
  for (int l = Lm - 1; l >= 0; --l) {
    const GLevel& L = lv[(size_t)l];
    const int64_t fr = (int64_t)L.W * L.H;
    const int32_t nblk = (int32_t)((fr + per_blk - 1) / per_blk);
    for (int k = 0; k < prm->iters; ++k) {
      k_gn_partial<<<dim3((unsigned)nblk, (unsigned)np), kAB, 0, st>>>(L, d_p, prm->tukey_c,
                                                                        nblk, d_part);
      const int32_t scale = (l > 0 && k == prm->iters - 1) ? 1 : 0;
      k_gn_solve<<<dim3((unsigned)np), 64, 0, st>>>(d_part, nblk, d_p, scale);
    }
    if (l > 0 && prm->iters == 0) k_gn_solve<<<dim3((unsigned)np), 64, 0, st>>>(d_part, 0, d_p, 1);
  }
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(p.data(), d_p, sizeof(double) * p.size(), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    cleanup();
    *err = "Gauss-Newton steps failed";
    return VI_E_HIP;
  }
  cleanup();
  const double cx = (W - 1) / 2.0, cy = (H - 1) / 2.0;
  for (int32_t n = 0; n < np; ++n) {
    const double* q = p.data() + (size_t)6 * n;
    double* th = theta + (size_t)6 * n;
    th[0] = 1.0 + q[2];
    th[1] = q[3];
    th[2] = q[0] - q[2] * cx - q[3] * cy;
    th[3] = q[4];
    th[4] = 1.0 + q[5];
    th[5] = q[1] - q[4] * cx - q[5] * cy;
  }
  return VI_OK;
}

vi_status align_compose(const double* theta, int32_t T, double* M) {
  const int ref = T / 2;
  const double id[6] = {1, 0, 0, 0, 1, 0};
  std::memcpy(M + 6 * (size_t)ref, id, sizeof(id));
  for (int n = ref - 1; n >= 0; --n)
    compose(M + 6 * (size_t)(n + 1), theta + 6 * (size_t)n, M + 6 * (size_t)n);
  for (int n = ref + 1; n < T; ++n) {
    double inv[6];
    if (!inverse(theta + 6 * (size_t)(n - 1), inv)) return VI_E_INVAL;
    compose(M + 6 * (size_t)(n - 1), inv, M + 6 * (size_t)n);
  }
  return VI_OK;
}

vi_status align_warp(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H, int32_t T,
                     const double* M, double* d_minv, uint8_t* out_rgb, uint8_t* out_mask,
                     hipStream_t st) {
  std::vector<double> inv((size_t)6 * T);
  for (int32_t t = 0; t < T; ++t)
    if (!inverse(M + 6 * (size_t)t, inv.data() + 6 * (size_t)t)) return VI_E_INVAL;
  if (hipMemcpyAsync(d_minv, inv.data(), sizeof(double) * inv.size(), hipMemcpyHostToDevice,
                     st) != hipSuccess)
    return VI_E_HIP;
  k_warp<<<grid3(W, H, T), kAB, 0, st>>>(rgb, mask, W, H, T, d_minv, out_rgb, out_mask);
  if (hipGetLastError() != hipSuccess) return VI_E_HIP;
  // the host copy of the inverses must outlive the transfer
  return hipStreamSynchronize(st) == hipSuccess ? VI_OK : VI_E_HIP;
}

vi_status align_unwarp(const uint8_t* aligned, const uint8_t* rgb, const uint8_t* mask, int32_t W,
                       int32_t H, int32_t T, const double* M, double* d_m, uint8_t* out,
                       hipStream_t st) {
  if (hipMemcpyAsync(d_m, M, sizeof(double) * 6 * (size_t)T, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return VI_E_HIP;
  k_unwarp<<<grid3(W, H, T), kAB, 0, st>>>(aligned, rgb, mask, W, H, T, d_m, out);
  if (hipGetLastError() != hipSuccess) return VI_E_HIP;
  return hipStreamSynchronize(st) == hipSuccess ? VI_OK : VI_E_HIP;
}

}  // namespace vi
