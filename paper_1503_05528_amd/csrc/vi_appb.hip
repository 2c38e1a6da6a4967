// vi_appb.hip -- the textured-patch experiment of App. B (Newson et al.):
// for reference patches W_r and every patch V of a grey volume, count the V
// that are closer to W_r (sum of squared differences, Sec. 2) than the
// constant patch Z of value mu.
//
// The distance is the patch distance of the search on one channel, through
// the same exact integer expansion SSD(W, V) = |W|^2 + |V|^2 - 2 <W, V>.
// All reference-candidate inner products form a dense contraction (refs x
// candidates x voxels), computed on the matrix cores with
// v_mfma_i32_16x16x64_i8 from centred bytes w' = w - 128, v' = v - 128:
//   <W, V> = <W', V'> + 128 sum V' + 128 sum W' + 128^2 N,
// so that, with a_c = |V|^2 - 256 sum V' per candidate and
// b_r = N mu^2 - 2 mu sum W + 256 sum W' + 32768 N per reference,
//   SSD(W, V) < SSD(W, Z)  <=>  a_c - 2 <W', V'> < b_r,
// every quantity an exact int32.
//
// Layout (16x16x64 i8): lane l supplies row l % 16 of A (a reference) and
// column l % 16 of B (a candidate), both with the 16 bytes of k-group l / 16
// of each 64-byte block; lane l receives D[4 (l / 16) + t][l % 16], t < 4.
//
// A workgroup owns a range of references and walks candidate blocks of kCB
// (strided over the grid): it gathers a block's packed candidates into LDS
// once (through a table of voxel offsets), then for every chunk of 256
// references each wave holds 64 references' A operands in registers, runs
// over the block's 16-candidate tiles, and accumulates per-lane hit counts;
// the counts of a chunk are summed over the 16 lanes of a row group and
// added to the workgroup's LDS counters, flushed with one global atomic per
// reference at the end.  References are packed (centred, zero padded, with
// b_r) by a first kernel into a workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "vi.h"
#include "vi_internal.h"

namespace vi {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kTB = 256;    // threads per workgroup (4 waves)
constexpr int kMaxN = 128;  // voxels per patch
constexpr int kRC = 256;    // references per chunk (64 per wave)
constexpr int kRR = 1024;   // references per workgroup range (LDS counters)
constexpr int kCB = 512;    // candidates per block staged in LDS
constexpr int kRowB = 144;  // LDS bytes per candidate: 128 + 16 against bank conflicts
// two workgroups per compute unit (160 KB of LDS)
static_assert(kCB * (kRowB + 4) + kRR * 4 + kMaxN * 4 <= 81920, "LDS of two workgroups");
// a_c of a padding candidate: above every b_r + 2 |<W', V'>|, never counts
constexpr int32_t kNever = INT_MAX / 2;

struct AppbArgs {
  const uint8_t* vol;      // [T][H][W]
  const int8_t* rp;        // packed references [n_pad][128]
  const int32_t* rb;       // b_r [n_pad]
  unsigned long long* counts;
  int32_t n_ref, W, H, pw, ph, N, mu;
  int32_t Wc, Hc, n_cand, n_blocks;
};

__global__ void k_zero_counts(unsigned long long* p, int32_t n) {
  const int32_t i = blockIdx.x * kTB + threadIdx.x;
  if (i < n) p[i] = 0;
}

// one thread per (padded) reference: centred bytes and b_r
__global__ void k_appb_pack(const uint8_t* __restrict__ ref, int32_t n_ref, int32_t n_pad,
                            int32_t N, int32_t mu, int8_t* __restrict__ rp,
                            int32_t* __restrict__ rb) {
  const int32_t r = blockIdx.x * kTB + threadIdx.x;
  if (r >= n_pad) return;
  int32_t* out = reinterpret_cast<int32_t*>(rp + (size_t)r * kMaxN);
  if (r >= n_ref) {
    for (int d = 0; d < kMaxN / 4; ++d) out[d] = 0;
    rb[r] = INT_MIN;  // a padding reference never counts
    return;
  }
  const uint8_t* w = ref + (size_t)r * N;
  int32_t sw = 0;
  for (int d = 0; d < kMaxN / 4; ++d) {
    uint32_t word = 0;
    for (int b = 0; b < 4; ++b) {
      const int k = 4 * d + b;
      if (k < N) {
        sw += w[k];
        word |= (uint32_t)(uint8_t)(int8_t)(w[k] - 128) << (8 * b);
      }
    }
    out[d] = (int32_t)word;
  }
  const int32_t swc = sw - 128 * N;  // sum of the centred bytes
  rb[r] = N * mu * mu - 2 * mu * sw + 256 * swc + 32768 * N;
}

// blockIdx.y: the reference range [y kRR, min(n_pad, (y + 1) kRR))
template <int KB>
__global__ __launch_bounds__(kTB) void k_closer_mfma(AppbArgs A, int32_t n_pad) {
  __shared__ __align__(16) uint8_t scand[kCB * kRowB];
  __shared__ int32_t sac[kCB];
  __shared__ uint32_t scnt[kRR];
  __shared__ __align__(16) int32_t soff[kMaxN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int32_t r_begin = blockIdx.y * kRR, r_end = min(n_pad, r_begin + kRR);

  for (int k = tid; k < kMaxN; k += kTB) {
    int32_t o = 0;
    if (k < A.N) {
      const int dx = k % A.pw, r = k / A.pw;
      o = ((r / A.ph) * A.H + r % A.ph) * A.W + dx;
    }
    soff[k] = o;
  }
  for (int k = tid; k < kRR; k += kTB) scnt[k] = 0;

  for (int32_t blk = blockIdx.x; blk < A.n_blocks; blk += gridDim.x) {
    __syncthreads();  // offsets ready; the previous block's readers done
    // gather the block's candidates: centred bytes (u - 128 is u ^ 0x80 in
    // two's complement), a_c.  Loads are unconditional (voxels beyond N read
    // the corner and are masked off), so a row's loads are in flight at once.
    for (int j = tid; j < kCB; j += kTB) {
      const int32_t i = blk * kCB + j;
      const bool ok = i < A.n_cand;
      const int32_t ii = ok ? i : 0;
      const int32_t x = ii % A.Wc, q = ii / A.Wc;
      const uint32_t base = (uint32_t)(((q / A.Hc) * A.H + q % A.Hc) * A.W + x);
      uint32_t* row = reinterpret_cast<uint32_t*>(scand + j * kRowB);
      uint32_t sv = 0, s1 = 0;
#pragma unroll 4
      for (int d = 0; d < KB * 16; ++d) {
        const int4 o = *reinterpret_cast<const int4*>(soff + 4 * d);
        const int rem = A.N - 4 * d;
        const uint32_t m = !ok || rem <= 0 ? 0u : (rem >= 4 ? 0xffffffffu : (1u << (8 * rem)) - 1u);
        const uint32_t raw = ((uint32_t)A.vol[base + o.x] | (uint32_t)A.vol[base + o.y] << 8 |
                              (uint32_t)A.vol[base + o.z] << 16 |
                              (uint32_t)A.vol[base + o.w] << 24) & m;
        sv = __builtin_amdgcn_udot4(raw, raw, sv, false);
        s1 = __builtin_amdgcn_udot4(raw, 0x01010101u, s1, false);
        row[d] = (raw ^ 0x80808080u) & m;
      }
      sac[j] = ok ? (int32_t)sv - 256 * ((int32_t)s1 - 128 * A.N) : kNever;
    }
    __syncthreads();

    // this wave's 64 references of a chunk: A operands and b_r of its output
    // rows; the next chunk's are fetched while the current one runs
    v4i af[4][KB], nf[4][KB];
    int32_t br[4][4], nb[4][4];
    auto fetch = [&](int32_t rc, v4i (&f)[4][KB], int32_t (&b)[4][4]) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int32_t r = rc + wave * 64 + a * 16 + c16;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
          f[a][kb] = *reinterpret_cast<const v4i*>(A.rp + (size_t)r * kMaxN + kb * 64 + g * 16);
        const v4i b4 = *reinterpret_cast<const v4i*>(A.rb + rc + wave * 64 + a * 16 + 4 * g);
        b[a][0] = b4.x;
        b[a][1] = b4.y;
        b[a][2] = b4.z;
        b[a][3] = b4.w;
      }
    };
    fetch(r_begin, nf, nb);
    for (int32_t rc = r_begin; rc < r_end; rc += kRC) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) af[a][kb] = nf[a][kb];
#pragma unroll
        for (int t = 0; t < 4; ++t) br[a][t] = nb[a][t];
      }
      if (rc + kRC < r_end) fetch(rc + kRC, nf, nb);
      uint32_t cnt[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int t = 0; t < 4; ++t) cnt[a][t] = 0;
      for (int ct = 0; ct < kCB / 16; ++ct) {
        const uint8_t* crow = scand + (ct * 16 + c16) * kRowB;
        v4i bf[KB];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
          bf[kb] = *reinterpret_cast<const v4i*>(crow + kb * 64 + g * 16);
        const int32_t ac = sac[ct * 16 + c16];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          v4i d = {0, 0, 0, 0};
#pragma unroll
          for (int kb = 0; kb < KB; ++kb)
            d = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a][kb], bf[kb], d, 0, 0, 0);
          cnt[a][0] += (ac - 2 * d.x < br[a][0]) ? 1u : 0u;
          cnt[a][1] += (ac - 2 * d.y < br[a][1]) ? 1u : 0u;
          cnt[a][2] += (ac - 2 * d.z < br[a][2]) ? 1u : 0u;
          cnt[a][3] += (ac - 2 * d.w < br[a][3]) ? 1u : 0u;
        }
      }
      // sum over the 16 candidate columns of each row group
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          uint32_t v = cnt[a][t];
          v += __shfl_xor(v, 8);
          v += __shfl_xor(v, 4);
          v += __shfl_xor(v, 2);
          v += __shfl_xor(v, 1);
          if (c16 == 0 && v != 0)
            atomicAdd(&scnt[rc - r_begin + wave * 64 + a * 16 + 4 * g + t], v);
        }
    }
  }
  __syncthreads();
  for (int k = tid; k < r_end - r_begin; k += kTB) {
    const int32_t r = r_begin + k;
    if (r < A.n_ref && scnt[k] != 0) atomicAdd(&A.counts[r], (unsigned long long)scnt[k]);
  }
}

}  // namespace

size_t closer_work_bytes(int32_t n_ref) {
  const size_t n_pad = ((size_t)n_ref + kRC - 1) / kRC * kRC;
  return n_pad * (kMaxN + sizeof(int32_t)) + 256;
}

vi_status closer_than_constant(const uint8_t* ref, int32_t n_ref, const uint8_t* vol, int32_t W,
                               int32_t H, int32_t T, int32_t pw, int32_t ph, int32_t pt,
                               int32_t mu, unsigned long long* counts, void* work,
                               hipStream_t st) {
  if (n_ref == 0) return VI_OK;
  const int32_t N = pw * ph * pt;
  const int32_t n_pad = (n_ref + kRC - 1) / kRC * kRC;
  int8_t* rp = static_cast<int8_t*>(work);
  int32_t* rb = reinterpret_cast<int32_t*>(rp + (size_t)n_pad * kMaxN);
  k_zero_counts<<<(n_ref + kTB - 1) / kTB, kTB, 0, st>>>(counts, n_ref);
  AppbArgs A{};
  A.vol = vol;
  A.rp = rp;
  A.rb = rb;
  A.counts = counts;
  A.n_ref = n_ref;
  A.W = W;
  A.H = H;
  A.pw = pw;
  A.ph = ph;
  A.N = N;
  A.mu = mu;
  A.Wc = W - pw + 1;
  A.Hc = H - ph + 1;
  const int32_t Tc = T - pt + 1;
  if (A.Wc > 0 && A.Hc > 0 && Tc > 0) {
    k_appb_pack<<<(n_pad + kTB - 1) / kTB, kTB, 0, st>>>(ref, n_ref, n_pad, N, mu, rp, rb);
    A.n_cand = A.Wc * A.Hc * Tc;
    A.n_blocks = (A.n_cand + kCB - 1) / kCB;
    // reference ranges of kRR (the last one shorter); candidate blocks spread
    // over about two workgroups per compute unit in all
    const int32_t ranges = (n_pad + kRR - 1) / kRR;
    const int32_t gx = std::max<int32_t>(1, std::min<int32_t>(A.n_blocks, 512 / ranges));
    const dim3 grid(gx, ranges);
    if (N > 64)
      k_closer_mfma<2><<<grid, kTB, 0, st>>>(A, n_pad);
    else
      k_closer_mfma<1><<<grid, kTB, 0, st>>>(A, n_pad);
  }
  return hipGetLastError() == hipSuccess ? VI_OK : VI_E_HIP;
}

}  // namespace vi
