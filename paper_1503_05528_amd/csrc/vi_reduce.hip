// vi_reduce.hip -- the dimensionality-reduced patch space (Newson et al.,
// Sec. 5, which proposes such a reduction as an acceleration without fixing
// one; the construction is this library's reading): principal directions of
// a level's source patches, quantised to a 16-bit integer basis, and the
// per-voxel features the searches then compare instead of whole patches.
//
// Patch vector x(p): for the offsets o in the order dt, dy, dx, the channels
// R, G, B, Tx, Ty of voxel p + o, its coordinates clamped to the volume
// (sources lie inside it).  Weights w = 1 (colour), sqrt(lambda) (texture)
// make |w x(p) - w x(c)|^2 the patch distance.
//
//   moments     S1_i = sum_s x_i(s), S2_ij = sum_s x_i(s) x_j(s) over every
//               k-th source (ascending), exact in 64-bit integers: samples
//               are gathered into a byte matrix with one row per coordinate
//               and the sums are v_dot4_u32_u8 inner products of its rows
//   covariance  C_ij = (w_i w_j) (S2_ij / n - (S1_i / n)(S1_j / n)), double
//               precision, each operation rounded on its own
//   basis       orthogonal iteration on C (one workgroup, a thread per
//               coordinate; products with C, then classical Gram-Schmidt
//               applied twice), from a fixed pseudo-random start
//   quantised   Q[k][i] = rint(256 w_i b_ik)
//   features    f_k(p) = (sum_i Q[k][i] x_i(p) + 128) >> 8, exact int32
//               (the caller's basis is checked so that no sum overflows)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "vi.h"
#include "vi_internal.h"

#pragma clang fp contract(off)

namespace vi {
namespace {

constexpr int kRB = 256;  // threads per workgroup of the voxel kernels

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// ---------------------------------------------------------------- features
// One thread per voxel of `list` (all voxels when list is null); the basis,
// transposed to [dim][DP], is staged in LDS and read by broadcast.
template <int DP>
__global__ __launch_bounds__(kRB) void k_features(DevLevel L, const int16_t* __restrict__ Qt,
                                                  int32_t dim, const int32_t* __restrict__ list,
                                                  int32_t n, int32_t* __restrict__ feat) {
  __shared__ __align__(16) int16_t sq[kPatchDimMax * DP];
  for (int i = threadIdx.x; i < dim * DP; i += kRB) sq[i] = Qt[i];
  __syncthreads();
  const int32_t j = blockIdx.x * kRB + threadIdx.x;
  if (j >= n) return;
  const int32_t p = list ? list[j] : j;
  const int32_t t = (int32_t)fdiv((uint32_t)p, L.fdWH);
  const int32_t r = p - t * L.WH;
  const int32_t y = (int32_t)fdiv((uint32_t)r, L.fdW);
  const int32_t x = r - y * L.W;
  int32_t acc[DP];
#pragma unroll
  for (int k = 0; k < DP; ++k) acc[k] = 0;
  const int16_t* q = sq;
  for (int dt = -L.ht; dt <= L.ht; ++dt) {
    const int32_t tt = clampi(t + dt, 0, L.T - 1);
    for (int dy = -2; dy <= 2; ++dy) {
      const int32_t row = (tt * L.H + clampi(y + dy, 0, L.H - 1)) * L.W;
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        const uint2 v = L.vox[row + clampi(x + dx, 0, L.W - 1)];
        const int32_t ch[5] = {(int32_t)(v.x & 255u), (int32_t)((v.x >> 8) & 255u),
                               (int32_t)((v.x >> 16) & 255u), (int32_t)(v.y & 255u),
                               (int32_t)((v.y >> 8) & 255u)};
#pragma unroll
        for (int c = 0; c < 5; ++c) {
#pragma unroll
          for (int k = 0; k < DP; ++k) acc[k] += (int32_t)q[c * DP + k] * ch[c];
        }
        q += 5 * DP;
      }
    }
  }
  int4* out = reinterpret_cast<int4*>(feat + (size_t)p * DP);
#pragma unroll
  for (int k = 0; k < DP; k += 4)
    out[k / 4] = make_int4((acc[k] + 128) >> 8, (acc[k + 1] + 128) >> 8, (acc[k + 2] + 128) >> 8,
                           (acc[k + 3] + 128) >> 8);
}

// ----------------------------------------------------------------- moments
// XT [dim][n_pad] bytes: column s = the patch vector of source dlist[s * k]
// (zero columns beyond n).
__global__ void k_pca_gather(DevLevel L, int32_t kstride, int32_t n, int32_t n_pad,
                             uint8_t* __restrict__ XT) {
  const int32_t s = blockIdx.x * kRB + threadIdx.x;
  if (s >= n_pad) return;
  const bool ok = s < n;
  const int32_t c = ok ? L.dlist[(int64_t)s * kstride] : 0;
  const int32_t t = (int32_t)fdiv((uint32_t)c, L.fdWH);
  const int32_t r = c - t * L.WH;
  const int32_t y = (int32_t)fdiv((uint32_t)r, L.fdW);
  const int32_t x = r - y * L.W;
  int32_t i = 0;
  for (int dt = -L.ht; dt <= L.ht; ++dt)
    for (int dy = -2; dy <= 2; ++dy)
      for (int dx = -2; dx <= 2; ++dx) {
        uint2 v = make_uint2(0, 0);
        if (ok) v = L.vox[((t + dt) * L.H + (y + dy)) * L.W + (x + dx)];
        const uint8_t ch[5] = {(uint8_t)v.x, (uint8_t)(v.x >> 8), (uint8_t)(v.x >> 16),
                               (uint8_t)v.y, (uint8_t)(v.y >> 8)};
#pragma unroll
        for (int cc = 0; cc < 5; ++cc, ++i) XT[(size_t)i * n_pad + s] = ch[cc];
      }
}

// S2 over 16 x 16 tiles of the upper triangle (mirrored), S1 by the diagonal
// tiles' first column of threads.  Rows of XT as dwords (nw per row); a
// 32-bit partial holds at most 256 dwords (256 x 4 x 255^2 < 2^32).
__global__ __launch_bounds__(256) void k_pca_moments(const uint32_t* __restrict__ XT, int32_t dim,
                                                     int32_t nw, unsigned long long* S1,
                                                     unsigned long long* S2) {
  const int ti = blockIdx.y, tj = blockIdx.x;
  if (tj < ti) return;
  const int a = threadIdx.x >> 4, b = threadIdx.x & 15;
  const int32_t i = ti * 16 + a, j = tj * 16 + b;
  if (i >= dim || j >= dim) return;
  const uint32_t* ri = XT + (size_t)i * nw;
  const uint32_t* rj = XT + (size_t)j * nw;
  unsigned long long s2 = 0, s1 = 0;
  const bool first = ti == tj && b == 0;
  for (int32_t w0 = 0; w0 < nw; w0 += 256) {
    const int32_t w1 = min(nw, w0 + 256);
    uint32_t p2 = 0, p1 = 0;
    for (int32_t w = w0; w < w1; ++w) {
      const uint32_t u = ri[w];
      p2 = __builtin_amdgcn_udot4(u, rj[w], p2, false);
      if (first) p1 = __builtin_amdgcn_udot4(u, 0x01010101u, p1, false);
    }
    s2 += p2;
    s1 += p1;
  }
  S2[(size_t)i * dim + j] = s2;
  S2[(size_t)j * dim + i] = s2;
  if (first) S1[i] = s1;
}

__global__ void k_pca_cov(const unsigned long long* __restrict__ S1,
                          const unsigned long long* __restrict__ S2, int32_t dim, int64_t n,
                          double wtex, double* __restrict__ C) {
  const int32_t e = blockIdx.x * kRB + threadIdx.x;
  if (e >= dim * dim) return;
  const int32_t i = e / dim, j = e - i * dim;
  const double nn = (double)n;
  const double wi = (i % 5) >= 3 ? wtex : 1.0, wj = (j % 5) >= 3 ? wtex : 1.0;
  const double mi = (double)S1[i] / nn, mj = (double)S1[j] / nn;
  const double e2 = (double)S2[e] / nn;
  C[e] = (wi * wj) * (e2 - mi * mj);
}

// ------------------------------------------------------------------- basis
// Sum of one value per thread over the workgroup (every thread gets it).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) s += red[k];
  return s;
}

// Orthogonal iteration for the M leading eigenvectors of the symmetric
// dim x dim matrix C (dim <= NT).  Thread i owns row i of the iterate Q and
// of Z = C Q (Qg, Zg: [dim][M] in global memory); the products read C by
// columns (C is symmetric: C[k][i] = C[i][k], coalesced).  Each column is
// orthogonalised against the previous ones by classical Gram-Schmidt
// applied twice, the j dot products of a pass reduced together.
template <int NT, int M>
__global__ __launch_bounds__(NT) void k_pca_eigen(const double* __restrict__ C, int32_t dim,
                                                  int32_t iters, double* Qg, double* Zg,
                                                  double* rq) {
  constexpr int NW = NT / 64;
  __shared__ double red[NW * M];
  const int i = threadIdx.x;
  const bool own = i < dim;
  double* zi = Zg + (size_t)(own ? i : 0) * M;
  double* qi = Qg + (size_t)(own ? i : 0) * M;
  // fixed pseudo-random start (a 32-bit integer hash of (i, j))
  if (own) {
    for (int j = 0; j < M; ++j) {
      uint32_t h = (uint32_t)i * 2654435761u ^ ((uint32_t)j * 40503u + 12345u);
      h ^= h >> 15;
      h *= 2246822519u;
      h ^= h >> 13;
      h *= 3266489917u;
      h ^= h >> 16;
      zi[j] = (double)(h & 0xffff) / 32768.0 - 1.0;
    }
  }
  for (int it = 0; it <= iters + 1; ++it) {
    if (it > 0) {
      // Z = C Q (every thread has finished writing its row of Q)
      __syncthreads();
      double z[M];
#pragma unroll
      for (int j = 0; j < M; ++j) z[j] = 0.0;
      if (own) {
        for (int32_t k = 0; k < dim; ++k) {
          const double cki = C[(size_t)k * dim + i];
          const double* qk = Qg + (size_t)k * M;
#pragma unroll
          for (int j = 0; j < M; ++j) z[j] += cki * qk[j];
        }
      }
      if (it == iters + 1) {
        // Rayleigh quotients q_j' C q_j: the variance each direction captures
        for (int j = 0; j < M; ++j) {
          const double v = block_sum<NT>(own ? qi[j] * z[j] : 0.0, red);
          if (i == 0) rq[j] = v;
        }
        return;
      }
      __syncthreads();  // every thread has read Q
      if (own) {
#pragma unroll
        for (int j = 0; j < M; ++j) zi[j] = z[j];
      }
    }
    for (int j = 0; j < M; ++j) {
      double zj = own ? zi[j] : 0.0;
      for (int pass = 0; pass < 2 && j > 0; ++pass) {
        for (int l = 0; l < j; ++l) {
          double v = own ? qi[l] * zj : 0.0;
#pragma unroll
          for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
          if ((i & 63) == 0) red[(i >> 6) * M + l] = v;
        }
        __syncthreads();
        for (int l = 0; l < j; ++l) {
          double r = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) r += red[w * M + l];
          if (own) zj -= r * qi[l];
        }
        __syncthreads();
      }
      const double nrm = sqrt(block_sum<NT>(zj * zj, red));
      if (own) qi[j] = nrm > 0.0 ? zj / nrm : 0.0;
    }
  }
}

// Q[k][i] = rint(256 w_i b_ik) for k < d; Qt[i][k] for k < DP (zero rows
// beyond d), the layout of the feature kernel
__global__ void k_pca_quant(const double* __restrict__ B, int32_t dim, int32_t M, int32_t d,
                            int32_t dp, double wtex, int16_t* __restrict__ Q,
                            int16_t* __restrict__ Qt) {
  const int32_t e = blockIdx.x * kRB + threadIdx.x;
  if (e >= dim * dp) return;
  const int32_t i = e / dp, k = e - i * dp;
  int16_t v = 0;
  if (k < d) {
    const double w = (i % 5) >= 3 ? wtex : 1.0;
    v = (int16_t)rint((256.0 * w) * B[(size_t)i * M + k]);
    Q[(size_t)k * dim + i] = v;
  }
  Qt[e] = v;
}

template <int DP>
void launch_features_dp(hipStream_t st, const DevLevel& L, const int16_t* Qt, int32_t dim,
                        const int32_t* list, int32_t n, int32_t* feat) {
  k_features<DP><<<(n + kRB - 1) / kRB, kRB, 0, st>>>(L, Qt, dim, list, n, feat);
}

}  // namespace

void launch_features(hipStream_t st, const DevLevel& L, const int16_t* Qt, int32_t dim,
                     int32_t dp, const int32_t* list, int32_t n, int32_t* feat) {
  if (n <= 0) return;
  switch (dp) {
    case 4: launch_features_dp<4>(st, L, Qt, dim, list, n, feat); break;
    case 8: launch_features_dp<8>(st, L, Qt, dim, list, n, feat); break;
    case 12: launch_features_dp<12>(st, L, Qt, dim, list, n, feat); break;
    case 16: launch_features_dp<16>(st, L, Qt, dim, list, n, feat); break;
    case 20: launch_features_dp<20>(st, L, Qt, dim, list, n, feat); break;
    case 24: launch_features_dp<24>(st, L, Qt, dim, list, n, feat); break;
    case 28: launch_features_dp<28>(st, L, Qt, dim, list, n, feat); break;
    default: launch_features_dp<32>(st, L, Qt, dim, list, n, feat); break;
  }
}

size_t pca_work_bytes(int32_t dim, int32_t n_max) {
  const size_t n_pad = ((size_t)n_max + 3) & ~(size_t)3;
  return (size_t)dim * n_pad + sizeof(unsigned long long) * ((size_t)dim * dim + dim) +
         sizeof(double) * ((size_t)dim * dim + 2 * (size_t)dim * kMaxRed + kMaxRed) + 8 * 256;
}

namespace {
struct PcaWork {
  uint8_t* XT;
  unsigned long long *S1, *S2;
  double *C, *Qg, *Zg, *rq;
};

// the work block of pca_work_bytes(dim, n_max), cut into its arrays
PcaWork carve(void* work, int32_t dim, int32_t n_max) {
  const size_t n_pad = ((size_t)n_max + 3) & ~(size_t)3;
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  uint8_t* p = static_cast<uint8_t*>(work);
  PcaWork w;
  w.XT = p;
  p += up((size_t)dim * n_pad);
  w.S1 = reinterpret_cast<unsigned long long*>(p);
  p += up(sizeof(unsigned long long) * dim);
  w.S2 = reinterpret_cast<unsigned long long*>(p);
  p += up(sizeof(unsigned long long) * (size_t)dim * dim);
  w.C = reinterpret_cast<double*>(p);
  p += up(sizeof(double) * (size_t)dim * dim);
  w.Qg = reinterpret_cast<double*>(p);
  p += up(sizeof(double) * (size_t)dim * kMaxRed);
  w.Zg = reinterpret_cast<double*>(p);
  p += up(sizeof(double) * (size_t)dim * kMaxRed);
  w.rq = reinterpret_cast<double*>(p);
  return w;
}
}  // namespace

int64_t pca_moments(hipStream_t st, const DevLevel& L, int32_t dim, int32_t n_max, void* work,
                    unsigned long long** S1, unsigned long long** S2) {
  const int32_t kstride = (L.nD + n_max - 1) / n_max;
  const int32_t n = (L.nD + kstride - 1) / kstride;
  const int32_t n_pad = (n + 3) & ~3;
  PcaWork w = carve(work, dim, n_max);
  k_pca_gather<<<(n_pad + kRB - 1) / kRB, kRB, 0, st>>>(L, kstride, n, n_pad, w.XT);
  const int tiles = (dim + 15) / 16;
  k_pca_moments<<<dim3(tiles, tiles), 256, 0, st>>>(reinterpret_cast<const uint32_t*>(w.XT), dim,
                                                    n_pad / 4, w.S1, w.S2);
  *S1 = w.S1;
  *S2 = w.S2;
  return n;
}

vi_status pca_basis(hipStream_t st, const DevLevel& L, int32_t dim, int32_t d, int32_t n_max,
                    int32_t iters, double wtex, void* work, int16_t* dQ, int16_t* dQt,
                    double** rq) {
  unsigned long long *S1, *S2;
  const int64_t n = pca_moments(st, L, dim, n_max, work, &S1, &S2);
  PcaWork w = carve(work, dim, n_max);
  k_pca_cov<<<(dim * dim + kRB - 1) / kRB, kRB, 0, st>>>(S1, S2, dim, n, wtex, w.C);
  const int32_t dp = (d + 3) & ~3;
  // the iterate has dp columns; the first d are the basis
  if (dim > 128) {
    switch (dp) {
      case 4: k_pca_eigen<640, 4><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 8: k_pca_eigen<640, 8><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 12: k_pca_eigen<640, 12><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 16: k_pca_eigen<640, 16><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 20: k_pca_eigen<640, 20><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 24: k_pca_eigen<640, 24><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 28: k_pca_eigen<640, 28><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      default: k_pca_eigen<640, 32><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
    }
  } else {
    switch (dp) {
      case 4: k_pca_eigen<128, 4><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 8: k_pca_eigen<128, 8><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 12: k_pca_eigen<128, 12><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 16: k_pca_eigen<128, 16><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 20: k_pca_eigen<128, 20><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 24: k_pca_eigen<128, 24><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      case 28: k_pca_eigen<128, 28><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
      default: k_pca_eigen<128, 32><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.Zg, w.rq); break;
    }
  }
  k_pca_quant<<<(dim * dp + kRB - 1) / kRB, kRB, 0, st>>>(w.Qg, dim, dp, d, dp, wtex, dQ, dQt);
  *rq = w.rq;
  return hipGetLastError() == hipSuccess ? VI_OK : VI_E_HIP;
}

}  // namespace vi
