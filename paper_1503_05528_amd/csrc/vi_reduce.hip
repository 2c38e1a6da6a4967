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
//               coordinate, the iterate in LDS; products with C, classical
//               Gram-Schmidt applied twice after every fourth product and
//               after the last), from a fixed pseudo-random start
//   quantised   Q[k][i] = rint(256 w_i b_ik)
//   features    f_k(p) = (sum_i Q[k][i] x_i(p) + 128) >> 8, exact int32
//               (the caller's basis is checked so that no sum overflows),
//               coordinates paired for v_dot2_i32_i16
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
constexpr int kOrthEvery = 4;  // products with C between orthonormalisations
typedef short short2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int32_t clampi(int32_t v, int32_t lo, int32_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// ---------------------------------------------------------------- features
// Device layout of a basis: Qp [rows][kPairs][DP] int32, rows = the patch's
// (dt, dy) rows, each row's 25 coordinates (5 voxels x 5 channels) in 13
// pairs, the low half coordinate 2m of the row, the high half 2m + 1 (0
// beyond 25).  A feature is then 13 v_dot2_i32_i16 per row, exact in int32.
// Grid-stride loop over `list` (all voxels when null): the workgroup stages
// the basis in LDS once and reads it by broadcast.
template <int DP>
__global__ __launch_bounds__(kRB) void k_features(DevLevel L, const int32_t* __restrict__ Qp,
                                                  int32_t rows, const int32_t* __restrict__ list,
                                                  int32_t n, int32_t* __restrict__ feat) {
  __shared__ __align__(16) int32_t sq[25 * kPairs * DP];
  for (int i = threadIdx.x; i < rows * kPairs * DP; i += kRB) sq[i] = Qp[i];
  __syncthreads();
  for (int32_t j = blockIdx.x * kRB + threadIdx.x; j < n; j += gridDim.x * kRB) {
    const int32_t p = list ? list[j] : j;
    const int32_t t = (int32_t)fdiv((uint32_t)p, L.fdWH);
    const int32_t r = p - t * L.WH;
    const int32_t y = (int32_t)fdiv((uint32_t)r, L.fdW);
    const int32_t x = r - y * L.W;
    int32_t xs[5];
#pragma unroll
    for (int dx = -2; dx <= 2; ++dx) xs[dx + 2] = clampi(x + dx, 0, L.W - 1);
    int32_t acc[DP];
#pragma unroll
    for (int k = 0; k < DP; ++k) acc[k] = 0;
    const int32_t* q = sq;
    for (int dt = -L.ht; dt <= L.ht; ++dt) {
      const int32_t tt = clampi(t + dt, 0, L.T - 1);
      for (int dy = -2; dy <= 2; ++dy) {
        const uint2* row = L.vox + (tt * L.H + clampi(y + dy, 0, L.H - 1)) * L.W;
        uint32_t v[25];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const uint2 u = row[xs[k]];
          v[5 * k] = u.x & 255u;
          v[5 * k + 1] = (u.x >> 8) & 255u;
          v[5 * k + 2] = (u.x >> 16) & 255u;
          v[5 * k + 3] = u.y & 255u;
          v[5 * k + 4] = (u.y >> 8) & 255u;
        }
#pragma unroll
        for (int m = 0; m < kPairs; ++m) {
          const uint32_t pr = v[2 * m] | (2 * m + 1 < 25 ? v[2 * m + 1] << 16 : 0u);
          const short2_t a = __builtin_bit_cast(short2_t, pr);
#pragma unroll
          for (int k = 0; k < DP; ++k)
            acc[k] = __builtin_amdgcn_sdot2(a, __builtin_bit_cast(short2_t, q[m * DP + k]),
                                            acc[k], false);
        }
        q += kPairs * DP;
      }
    }
    int4* out = reinterpret_cast<int4*>(feat + (size_t)p * DP);
#pragma unroll
    for (int k = 0; k < DP; k += 4)
      out[k / 4] = make_int4((acc[k] + 128) >> 8, (acc[k + 1] + 128) >> 8,
                             (acc[k + 2] + 128) >> 8, (acc[k + 3] + 128) >> 8);
  }
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

// S2 = XT XT' over 64 x 64 tiles of the upper triangle (mirrored), the
// samples split over gridDim.z slices added with 64-bit atomics into S2
// (zeroed before).  XT rows are dwords of 4 samples (nw per row); each
// stage takes 16 dwords of 64 rows of either side into LDS and every
// thread forms a 4 x 4 block of v_dot4_u32_u8 sums (a 32-bit partial holds
// 16 dwords: 16 x 4 x 255^2 < 2^32).
constexpr int kMT = 64, kMW = 16;
__global__ __launch_bounds__(256) void k_pca_moments(const uint32_t* __restrict__ XT, int32_t dim,
                                                     int32_t nw, unsigned long long* S2) {
  const int ti = blockIdx.y, tj = blockIdx.x;
  if (tj < ti) return;
  __shared__ uint32_t sa[kMT][kMW + 1], sb[kMT][kMW + 1];
  const int tid = threadIdx.x, ta = tid >> 4, tb = tid & 15;
  const int32_t i0 = ti * kMT, j0 = tj * kMT;
  // this slice's dwords
  const int32_t per = (nw + gridDim.z - 1) / gridDim.z;
  const int32_t w0 = blockIdx.z * per, w1 = min(nw, w0 + per);
  unsigned long long acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0;
  for (int32_t wc = w0; wc < w1; wc += kMW) {
    __syncthreads();
    for (int e = tid; e < kMT * kMW; e += 256) {
      const int r = e / kMW, w = e % kMW;
      const bool okw = wc + w < w1;
      sa[r][w] = (okw && i0 + r < dim) ? XT[(size_t)(i0 + r) * nw + wc + w] : 0u;
      sb[r][w] = (okw && j0 + r < dim) ? XT[(size_t)(j0 + r) * nw + wc + w] : 0u;
    }
    __syncthreads();
    uint32_t part[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) part[a][b] = 0;
#pragma unroll
    for (int w = 0; w < kMW; ++w) {
      uint32_t va[4], vb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) va[a] = sa[ta * 4 + a][w];
#pragma unroll
      for (int b = 0; b < 4; ++b) vb[b] = sb[tb * 4 + b][w];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) part[a][b] = __builtin_amdgcn_udot4(va[a], vb[b], part[a][b], false);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += part[a][b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int32_t i = i0 + ta * 4 + a, j = j0 + tb * 4 + b;
      if (i < dim && j < dim && j >= i) {
        atomicAdd(&S2[(size_t)i * dim + j], acc[a][b]);
        if (j != i) atomicAdd(&S2[(size_t)j * dim + i], acc[a][b]);
      }
    }
}

// S1: one workgroup per coordinate
__global__ __launch_bounds__(256) void k_pca_s1(const uint32_t* __restrict__ XT, int32_t nw,
                                                unsigned long long* S1) {
  __shared__ unsigned long long red[4];
  const uint32_t* r = XT + (size_t)blockIdx.x * nw;
  unsigned long long s = 0;
  for (int32_t w = threadIdx.x; w < nw; w += 256) s += __builtin_amdgcn_udot4(r[w], 0x01010101u, 0u, false);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) S1[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_zero_u64(unsigned long long* p, int32_t n) {
  const int32_t i = blockIdx.x * kRB + threadIdx.x;
  if (i < n) p[i] = 0;
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
// Largest of one value per thread over the workgroup (every thread gets it).
template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
  constexpr int NW = NT / 64;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) s = fmax(s, red[k]);
  return s;
}

// Sum of one value per thread over the workgroup (every thread gets it);
// `red` (NT / 64 entries) serves no other purpose, so the leading barrier
// is the only one its previous readers need.
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
// dim x dim matrix C (dim <= ROWS <= NT).  The iterate q lives in LDS (row k
// at sQ[k * QS], rows padded against bank conflicts where room allows);
// thread i holds row i of z = C q in registers, reading C by columns (C is
// symmetric: C[k][i] = C[i][k], coalesced) and the rows of q by broadcast.
// Between orthonormalisations the columns take kOrthEvery products with C,
// each column scaled by a power of two near its largest magnitude (exact)
// to stay in range: the span is that of orthogonal iteration.  A column is
// orthogonalised against the previous ones by classical Gram-Schmidt
// applied twice (the dot products of a pass reduced together), then
// normalised; thread i only touches row i of q then.  The final basis goes
// to Qg [dim][M].
template <int NT, int M>
__global__ __launch_bounds__(NT) void k_pca_eigen(const double* __restrict__ C, int32_t dim,
                                                  int32_t iters, double* Qg, double* rq) {
  constexpr int NW = NT / 64;
  constexpr int ROWS = NT > 128 ? kPatchDimMax : kPatchDimMax / 5;
  constexpr int QS = M < 32 ? M + 1 : M;
  __shared__ double sQ[ROWS * QS];
  __shared__ double red[NW * M];  // Gram-Schmidt dot products
  __shared__ double redb[NW];     // block sums and maxima
  const int i = threadIdx.x;
  const bool own = i < dim;
  double* qi = sQ + (own ? i : 0) * QS;
  double z[M];
  // fixed pseudo-random start (a 32-bit integer hash of (i, j))
#pragma unroll
  for (int j = 0; j < M; ++j) {
    uint32_t h = (uint32_t)i * 2654435761u ^ ((uint32_t)j * 40503u + 12345u);
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    h *= 3266489917u;
    h ^= h >> 16;
    z[j] = own ? (double)(h & 0xffff) / 32768.0 - 1.0 : 0.0;
  }
  for (int it = 0; it <= iters + 1; ++it) {
    if (it > 0) {
      // z = C q
      __syncthreads();  // every row of q is written
#pragma unroll
      for (int j = 0; j < M; ++j) z[j] = 0.0;
      if (own) {
        for (int32_t k = 0; k < dim; ++k) {
          const double c = C[(size_t)k * dim + i];
          const double* qk = sQ + k * QS;
#pragma unroll
          for (int j = 0; j < M; ++j) z[j] += c * qk[j];
        }
      }
      if (it == iters + 1) {
        // Rayleigh quotients q_j' C q_j: the variance each direction
        // captures; the basis to global memory
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double qij = own ? qi[j] : 0.0;
          if (own) Qg[(size_t)i * M + j] = qij;
          const double v = block_sum<NT>(qij * z[j], redb);
          if (i == 0) rq[j] = v;
        }
        return;
      }
      if (it % kOrthEvery != 0 && it != iters) {
        // another product before the next orthonormalisation (the block
        // maxima's barriers also end every thread's reads of q)
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const double mx = block_max<NT>(fabs(z[j]), redb);
          const double sc = mx > 0.0 ? ldexp(1.0, -ilogb(mx)) : 1.0;
          if (own) qi[j] = z[j] * sc;
        }
        continue;
      }
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        if (j > 0) {
#pragma unroll
          for (int l = 0; l < M; ++l) {
            if (l < j) {
              double v = own ? qi[l] * z[j] : 0.0;
#pragma unroll
              for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
              if ((i & 63) == 0) red[(i >> 6) * M + l] = v;
            }
          }
          __syncthreads();
#pragma unroll
          for (int l = 0; l < M; ++l) {
            if (l < j) {
              double r = 0.0;
#pragma unroll
              for (int w = 0; w < NW; ++w) r += red[w * M + l];
              if (own) z[j] -= r * qi[l];
            }
          }
          __syncthreads();
        }
      }
      // (the block sum's barriers also end every thread's reads of q in
      // the product above, before row i of q is rewritten)
      const double nrm = sqrt(block_sum<NT>(z[j] * z[j], redb));
      if (own) qi[j] = nrm > 0.0 ? z[j] / nrm : 0.0;
    }
  }
}

// Q[k][i] = rint(256 w_i b_ik) for k < d (host layout [d][dim]), and the
// device layout Qp of the feature kernel (dp columns, zero beyond d)
__global__ void k_pca_quant(const double* __restrict__ B, int32_t dim, int32_t M, int32_t d,
                            int32_t dp, double wtex, int16_t* __restrict__ Q,
                            int32_t* __restrict__ Qp) {
  const int32_t e = blockIdx.x * kRB + threadIdx.x;
  const int32_t rows = dim / 25;
  if (e >= rows * kPairs * dp) return;
  const int32_t k = e % dp, m = (e / dp) % kPairs, row = e / (dp * kPairs);
  uint32_t packed = 0;
  for (int h = 0; h < 2; ++h) {
    const int32_t c = 2 * m + h;  // coordinate within the row
    if (c >= 25 || k >= d) continue;
    const int32_t i = row * 25 + c;
    const double w = (i % 5) >= 3 ? wtex : 1.0;
    const int16_t v = (int16_t)rint((256.0 * w) * B[(size_t)i * M + k]);
    Q[(size_t)k * dim + i] = v;
    packed |= (uint32_t)(uint16_t)v << (16 * h);
  }
  Qp[e] = (int32_t)packed;
}

template <int DP>
void launch_features_dp(hipStream_t st, const DevLevel& L, const int32_t* Qp, int32_t rows,
                        const int32_t* list, int32_t n, int32_t* feat) {
  // about 16 workgroups per compute unit, each staging the basis once
  const int32_t grid = std::min<int32_t>((n + kRB - 1) / kRB, 4096);
  k_features<DP><<<grid, kRB, 0, st>>>(L, Qp, rows, list, n, feat);
}

}  // namespace

void launch_features(hipStream_t st, const DevLevel& L, const int32_t* Qp, int32_t dim,
                     int32_t dp, const int32_t* list, int32_t n, int32_t* feat) {
  if (n <= 0) return;
  const int32_t rows = dim / 25;
  switch (dp) {
    case 4: launch_features_dp<4>(st, L, Qp, rows, list, n, feat); break;
    case 8: launch_features_dp<8>(st, L, Qp, rows, list, n, feat); break;
    case 12: launch_features_dp<12>(st, L, Qp, rows, list, n, feat); break;
    case 16: launch_features_dp<16>(st, L, Qp, rows, list, n, feat); break;
    case 20: launch_features_dp<20>(st, L, Qp, rows, list, n, feat); break;
    case 24: launch_features_dp<24>(st, L, Qp, rows, list, n, feat); break;
    case 28: launch_features_dp<28>(st, L, Qp, rows, list, n, feat); break;
    default: launch_features_dp<32>(st, L, Qp, rows, list, n, feat); break;
  }
}

size_t pca_work_bytes(int32_t dim, int32_t n_max) {
  const size_t n_pad = ((size_t)n_max + 3) & ~(size_t)3;
  return (size_t)dim * n_pad + sizeof(unsigned long long) * ((size_t)dim * dim + dim) +
         sizeof(double) * ((size_t)dim * dim + (size_t)dim * kMaxRed + kMaxRed) + 8 * 256;
}

namespace {
struct PcaWork {
  uint8_t* XT;
  unsigned long long *S1, *S2;
  double *C, *Qg, *rq;
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
  const int tiles = (dim + kMT - 1) / kMT;
  k_zero_u64<<<(dim * dim + kRB - 1) / kRB, kRB, 0, st>>>(w.S2, dim * dim);
  // slices of the samples: about 4 workgroups per compute unit in all
  const int32_t blocks = tiles * (tiles + 1) / 2;
  const int32_t slices = std::max(1, std::min(n_pad / 4 / (4 * kMW), 1024 / blocks));
  k_pca_moments<<<dim3(tiles, tiles, slices), 256, 0, st>>>(
      reinterpret_cast<const uint32_t*>(w.XT), dim, n_pad / 4, w.S2);
  k_pca_s1<<<dim, 256, 0, st>>>(reinterpret_cast<const uint32_t*>(w.XT), n_pad / 4, w.S1);
  *S1 = w.S1;
  *S2 = w.S2;
  return n;
}

vi_status pca_basis(hipStream_t st, const DevLevel& L, int32_t dim, int32_t d, int32_t n_max,
                    int32_t iters, double wtex, void* work, int16_t* dQ, int32_t* dQp,
                    double** rq) {
  unsigned long long *S1, *S2;
  const int64_t n = pca_moments(st, L, dim, n_max, work, &S1, &S2);
  PcaWork w = carve(work, dim, n_max);
  k_pca_cov<<<(dim * dim + kRB - 1) / kRB, kRB, 0, st>>>(S1, S2, dim, n, wtex, w.C);
  const int32_t dp = (d + 3) & ~3;
  // the iterate has dp columns; the first d are the basis
  if (dim > 128) {
    switch (dp) {
      case 4: k_pca_eigen<640, 4><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 8: k_pca_eigen<640, 8><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 12: k_pca_eigen<640, 12><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 16: k_pca_eigen<640, 16><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 20: k_pca_eigen<640, 20><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 24: k_pca_eigen<640, 24><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 28: k_pca_eigen<640, 28><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      default: k_pca_eigen<640, 32><<<1, 640, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
    }
  } else {
    switch (dp) {
      case 4: k_pca_eigen<128, 4><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 8: k_pca_eigen<128, 8><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 12: k_pca_eigen<128, 12><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 16: k_pca_eigen<128, 16><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 20: k_pca_eigen<128, 20><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 24: k_pca_eigen<128, 24><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      case 28: k_pca_eigen<128, 28><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
      default: k_pca_eigen<128, 32><<<1, 128, 0, st>>>(w.C, dim, iters, w.Qg, w.rq); break;
    }
  }
  const int32_t nq = dim / 25 * kPairs * dp;
  k_pca_quant<<<(nq + kRB - 1) / kRB, kRB, 0, st>>>(w.Qg, dim, dp, d, dp, wtex, dQ, dQp);
  *rq = w.rq;
  return hipGetLastError() == hipSuccess ? VI_OK : VI_E_HIP;
}

}  // namespace vi
