// vi_appb.hip -- the textured-patch experiment of App. B (Newson et al.):
// for reference patches W_r and every patch V of a grey volume, count the V
// that are closer to W_r (sum of squared differences, Sec. 2) than the
// constant patch Z of value mu.
//
// The distance is the patch distance of the search, on one channel, with
// the same exact integer expansion: SSD(W, V) = |W|^2 + |V|^2 - 2 <W, V>,
// the inner product taken four bytes at a time by v_dot4_u32_u8.  Then
//   SSD(W, V) < SSD(W, Z)  <=>  |V|^2 - 2 <W, V> < N mu^2 - 2 mu sum(W),
// a per-candidate term, one inner product and a per-reference constant.
//
// Every thread holds kCPT candidate patches packed into ND dwords of
// registers (gathered once, through a table of voxel offsets); the
// workgroup stages kRB reference patches and their constants in LDS, and
// every wave walks them in lockstep (broadcast reads), so the inner loop is
// ND dot4 + 2 VALU per pair and the hit count per reference is a ballot
// popcount in scalar registers, summed in LDS and flushed with one global
// atomic per reference and workgroup.  The 2-D grid spreads both the
// candidates (x) and ranges of references (y) over the chip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <utility>

#include "vi.h"
#include "vi_internal.h"

namespace vi {
namespace {

constexpr int kTB = 256;   // threads per workgroup
constexpr int kCPT = 4;    // candidate patches per thread
constexpr int kRB = 256;   // reference patches per LDS chunk
constexpr int kMaxN = 128; // voxels per patch (32 packed dwords)
// |V|^2 of a padding candidate: above every per-reference constant
// (at most 128 * 255^2), so it never counts
constexpr int32_t kNever = 0x3fffffff;
static_assert(kTB == kRB, "one reference per thread when a chunk is staged");

struct AppbArgs {
  const uint8_t* ref;  // [n_ref][N]
  const uint8_t* vol;  // [T][H][W]
  unsigned long long* counts;
  int32_t n_ref, W, H, pw, ph, N, mu;
  int32_t Wc, Hc, n_cand;  // candidate corners: Wc x Hc x Tc
  int32_t refs_per_y;      // references of one grid row (a multiple of kRB)
};

__global__ void k_zero_counts(unsigned long long* p, int32_t n) {
  const int32_t i = blockIdx.x * kTB + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <int ND>
__global__ __launch_bounds__(kTB) void k_closer(AppbArgs A) {
  constexpr int S = (ND + 3) & ~3;  // LDS stride: whole 16-byte rows
  // candidate staging, then the reference chunks (kTB * ND <= kRB * S)
  __shared__ __align__(16) uint32_t sbuf[kRB * S];
  uint32_t* const sref = sbuf;
  __shared__ int32_t ssum[kRB];
  __shared__ uint32_t scnt[kRB];
  __shared__ __align__(16) int32_t soff[4 * ND];
  const int tid = threadIdx.x;

  // voxel k of a patch (order dt, dy, dx) lies soff[k] after its corner;
  // the padding voxels of the last dword read the corner and are masked off
  for (int k = tid; k < 4 * ND; k += kTB) {
    int32_t o = 0;
    if (k < A.N) {
      const int dx = k % A.pw, r = k / A.pw;
      o = ((r / A.ph) * A.H + r % A.ph) * A.W + dx;
    }
    soff[k] = o;
  }
  __syncthreads();
  const int rem = A.N & 3;  // ND = ceil(N / 4): only the last dword is partial
  const uint32_t last_mask = rem ? (1u << (8 * rem)) - 1u : 0xffffffffu;

  // Gather each candidate patch once: a thread assembles its own packed
  // dwords in a rolled loop and parks them in LDS (column tid, conflict
  // free), then takes them into registers with static indices.  Only this
  // thread reads what it wrote, so no barrier is needed.
  uint32_t cv[kCPT][ND];
  int32_t sv[kCPT];
#pragma unroll
  for (int j = 0; j < kCPT; ++j) {
    const int32_t i = (blockIdx.x * kCPT + j) * kTB + tid;
    const bool ok = i < A.n_cand;
    const int32_t ii = ok ? i : 0;
    const int32_t x = ii % A.Wc, q = ii / A.Wc;
    const uint32_t base = (uint32_t)(((q / A.Hc) * A.H + q % A.Hc) * A.W + x);
    uint32_t s = 0;
#pragma unroll 2
    for (int d = 0; d < ND; ++d) {
      const int4 o = *reinterpret_cast<const int4*>(soff + 4 * d);
      uint32_t w = (uint32_t)A.vol[base + o.x] | (uint32_t)A.vol[base + o.y] << 8 |
                   (uint32_t)A.vol[base + o.z] << 16 | (uint32_t)A.vol[base + o.w] << 24;
      if (d == ND - 1) w &= last_mask;
      if (!ok) w = 0;
      sbuf[d * kTB + tid] = w;
      s = __builtin_amdgcn_udot4(w, w, s, false);
    }
    sv[j] = ok ? (int32_t)s : kNever;
#pragma unroll
    for (int d = 0; d < ND; ++d) cv[j][d] = sbuf[d * kTB + tid];
  }

  const int32_t r_begin = blockIdx.y * A.refs_per_y;
  const int32_t r_end = min(A.n_ref, r_begin + A.refs_per_y);
  const int32_t nmu2 = A.N * A.mu * A.mu;
  for (int32_t r0 = r_begin; r0 < r_end; r0 += kRB) {
    const int nr = min(kRB, r_end - r0);
    __syncthreads();  // the previous chunk is consumed and flushed
    scnt[tid] = 0;
    ssum[tid] = 0;
    __syncthreads();
    // stage the chunk: dword d of reference r at sref[r * S + d], zero
    // padded, and the sum of every reference's voxels
    for (int idx = tid; idx < nr * S; idx += kTB) {
      const int r = idx / S, d = idx % S;
      const uint8_t* w = A.ref + (int64_t)(r0 + r) * A.N;
      uint32_t word = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int k = 4 * d + b;
        const uint32_t byte = w[min(k, A.N - 1)];
        word |= (k < A.N ? byte : 0u) << (8 * b);
      }
      sref[idx] = word;
      const uint32_t part = __builtin_amdgcn_udot4(word, 0x01010101u, 0u, false);
      if (part) atomicAdd(&ssum[r], (int32_t)part);
    }
    __syncthreads();

    for (int r = 0; r < nr; ++r) {
      const uint4* w4 = reinterpret_cast<const uint4*>(sref + r * S);
      uint32_t acc[kCPT];
#pragma unroll
      for (int j = 0; j < kCPT; ++j) acc[j] = 0;
#pragma unroll
      for (int d4 = 0; d4 < S / 4; ++d4) {
        const uint4 q = w4[d4];
        const uint32_t wq[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (4 * d4 + e < ND) {
#pragma unroll
            for (int j = 0; j < kCPT; ++j)
              acc[j] = __builtin_amdgcn_udot4(wq[e], cv[j][4 * d4 + e], acc[j], false);
          }
        }
      }
      // SSD(W, Z) - |W|^2 for this reference
      const int32_t c = nmu2 - 2 * A.mu * ssum[r];
      uint32_t hits = 0;
#pragma unroll
      for (int j = 0; j < kCPT; ++j)
        hits += __popcll(__ballot(sv[j] - 2 * (int32_t)acc[j] < c));
      if (hits != 0 && (tid & 63) == 0) atomicAdd(&scnt[r], hits);
    }
    __syncthreads();
    if (tid < nr && scnt[tid] != 0)
      atomicAdd(&A.counts[r0 + tid], (unsigned long long)scnt[tid]);
  }
}

template <int ND>
void launch_closer(hipStream_t st, dim3 grid, const AppbArgs& A) {
  k_closer<ND><<<grid, kTB, 0, st>>>(A);
}

using Launcher = void (*)(hipStream_t, dim3, const AppbArgs&);

template <int... I>
constexpr auto launcher_table(std::integer_sequence<int, I...>) {
  return std::array<Launcher, sizeof...(I)>{&launch_closer<I + 1>...};
}

}  // namespace

vi_status closer_than_constant(const uint8_t* ref, int32_t n_ref, const uint8_t* vol, int32_t W,
                               int32_t H, int32_t T, int32_t pw, int32_t ph, int32_t pt,
                               int32_t mu, unsigned long long* counts, hipStream_t st) {
  if (n_ref == 0) return VI_OK;
  static constexpr auto table = launcher_table(std::make_integer_sequence<int, kMaxN / 4>{});
  const int32_t N = pw * ph * pt;
  const int32_t nd = (N + 3) / 4;
  k_zero_counts<<<(n_ref + kTB - 1) / kTB, kTB, 0, st>>>(counts, n_ref);
  AppbArgs A{};
  A.ref = ref;
  A.vol = vol;
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
    A.n_cand = A.Wc * A.Hc * Tc;
    const int32_t gx = (A.n_cand + kTB * kCPT - 1) / (kTB * kCPT);
    // split the references over grid rows until the grid holds about 16
    // workgroups per compute unit
    const int32_t chunks = (n_ref + kRB - 1) / kRB;
    const int32_t want_y = std::max<int32_t>(1, (4096 + gx - 1) / gx);
    const int32_t gy0 = std::min(chunks, want_y);
    A.refs_per_y = ((chunks + gy0 - 1) / gy0) * kRB;
    const int32_t gy = (n_ref + A.refs_per_y - 1) / A.refs_per_y;
    table[nd - 1](st, dim3(gx, gy), A);
  }
  return hipGetLastError() == hipSuccess ? VI_OK : VI_E_HIP;
}

}  // namespace vi
