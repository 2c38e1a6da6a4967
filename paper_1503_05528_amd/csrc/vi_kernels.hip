// vi_kernels.hip -- gfx950 kernels of the inpainting hot path.
//
// Paper anchors (Newson et al., "Video Inpainting of Complex Scenes"):
//   patch distance           Sec. 2 Eq. (2.2), Sec. 3.3 Eq. (3.6), Sec. 3.5 Eq. (3.10)
//   ANN search               Sec. 3.1, Alg. 1, Eq. (3.1)
//   reconstruction           Sec. 3.2 Eqs. (3.2)-(3.4), Sec. 3.3 Eq. (3.8)
//   pyramids and features    Sec. 3.3 Eqs. (3.5), (3.7), Sec. 3.6, Alg. 4
//   onion peel               Sec. 3.5, Alg. 3
//
// The distance is a gather over 125 voxels, not a dense contraction, so it
// runs on the VALU: the squared difference is expanded as |a|^2 + |b|^2 -
// 2 a.b with v_dot4_u32_u8 on packed bytes, exact in uint32 arithmetic
// because every partial sum is a true partial SSD below 2^31.

#include "vi_internal.h"

namespace vi {

static constexpr int kBlock = 256;

__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_udot4(a, b, c, false);
}

__device__ __forceinline__ void unlin(const DevLevel& L, int32_t p, int32_t& x, int32_t& y,
                                      int32_t& t) {
  t = (int32_t)fdiv((uint32_t)p, L.fdWH);
  int32_t r = p - t * L.WH;
  y = (int32_t)fdiv((uint32_t)r, L.fdW);
  x = r - y * L.W;
}

// ------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// ------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// uniform integer in [0, n) from the high 32 bits of w
__device__ __forceinline__ int32_t draw_below(uint64_t w, uint32_t n) {
  return (int32_t)(((w >> 32) * (uint64_t)n) >> 32);
}

// ------------------------------------------------------------------------
// Patch distance of the target patch at p against the candidate centre c (a
// source of D~, so every candidate voxel is in the volume and known).  Target
// voxels outside the volume, or flagged in `excl`, are not compared; `nvox`
// receives the number compared.
//
// Per voxel: |a-b|^2 = a.a + b.b - 2 a.b on the colour word and on the
// texture word with v_dot4_u32_u8; every partial sum equals the true partial
// SSD (a sum of non-negative terms below 2^31), exact in uint32.  The 25 rows
// (dt, dy) are visited from the centre outwards, the centre row first, then
// in pairs of rows; after each group the partial sum is compared with `abort_above` and
// the evaluation stops when it exceeds it: the full distance could then only
// be larger, so the caller's decision is unchanged, and a hopeless candidate
// (typically a random-search draw, a cold fetch) costs one row instead of 25.
// Inside a group every load is unconditional (voxels outside the volume read
// the patch centre and are masked to zero), so the loads of a group are in
// flight together instead of one round trip per voxel.  The returned value
// is the full distance when it is <= abort_above, otherwise some value >
// abort_above.
// ------------------------------------------------------------------------
__constant__ int8_t kRowDt[25] = {0, 0, 0, -1, 1, 0, 0, -1, -1, 1, 1, -2, 2,
                                  -1, -1, 1, 1, -2, -2, 2, 2, -2, -2, 2, 2};
__constant__ int8_t kRowDy[25] = {0, -1, 1, 0, 0, -2, 2, -1, 1, -1, 1, 0, 0,
                                  -2, 2, -2, 2, -1, 1, -1, 1, -2, 2, -2, 2};
// the five rows of a 5x5x1 patch (single images), centre out
__constant__ int8_t kRowDt2[5] = {0, 0, 0, 0, 0};
__constant__ int8_t kRowDy2[5] = {0, -1, 1, -2, 2};

struct SsdAcc {
  uint32_t sc, st;  // colour and texture partial sums
  int32_t n;
};

__device__ __forceinline__ void acc_voxel(SsdAcc& q, uint2 a, uint2 b) {
  q.sc = dot4(a.x, a.x, q.sc);
  q.sc = dot4(b.x, b.x, q.sc);
  q.st = dot4(a.y, a.y, q.st);
  q.st = dot4(b.y, b.y, q.st);
  q.sc -= 2u * dot4(a.x, b.x, 0u);
  q.st -= 2u * dot4(a.y, b.y, 0u);
}

// rows [R0, R1) of the centre-out order; FULL: every target voxel is in the
// volume and compared (no masks)
// Five consecutive voxels (one patch row, dx = -2..2) with two 16-byte loads
// and one 8-byte load.  The pointer is only 8-byte aligned and the type says
// so: the compiler picks the widest loads that alignment allows.
typedef uint32_t u32x4_a8 __attribute__((ext_vector_type(4), aligned(8)));
typedef uint32_t u32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));

struct Row5 {
  uint2 v[5];
};

__device__ __forceinline__ Row5 load_row5(const uint2* __restrict__ r) {
  const u32x4_a8 v01 = *reinterpret_cast<const u32x4_a8*>(r);
  const u32x4_a8 v23 = *reinterpret_cast<const u32x4_a8*>(r + 2);
  Row5 o;
  o.v[0] = make_uint2(v01.x, v01.y);
  o.v[1] = make_uint2(v01.z, v01.w);
  o.v[2] = make_uint2(v23.x, v23.y);
  o.v[3] = make_uint2(v23.z, v23.w);
  o.v[4] = r[4];
  return o;
}

// one row (dt, dy) of the patch pair; FULL: every target voxel is in the
// volume and compared (no masks)
template <bool FULL, bool MASKED>
__device__ __forceinline__ void ssd_row(const DevLevel& L, const uint8_t* __restrict__ excl,
                                        int32_t p, int32_t px, int32_t py, int32_t pt, int32_t c,
                                        int dt, int dy, SsdAcc& q) {
  const uint2* __restrict__ vox = L.vox;
  const int32_t row = dt * L.WH + dy * L.W;
  // the candidate patch lies inside the volume: its row is one span
  const Row5 b = load_row5(vox + (c + row - 2));
  if (FULL) {
    const Row5 a = load_row5(vox + (p + row - 2));
#pragma unroll
    for (int k = 0; k < 5; ++k) acc_voxel(q, a.v[k], b.v[k]);
  } else if (MASKED) {
    // the target row with one row load as well (the voxel array holds two
    // entries of padding on both sides) and its five exclusion bytes with
    // one 8-byte load (the mask holds 16 bytes of padding on both sides);
    // entries outside the volume or excluded are masked
    const int32_t tt = pt + dt, yy = py + dy;
    const bool rok = tt >= 0 && tt < L.T && yy >= 0 && yy < L.H;
    const int32_t base = (rok ? p + row : p) - 2;
    const Row5 a = load_row5(vox + base);
    const int klo = px < 2 ? 2 - px : 0;
    const int khi = px + 2 >= L.W ? L.W + 1 - px : 4;
    uint32_t okm = rok ? ((0x1fu << klo) & (0x1fu >> (4 - khi))) : 0u;
    const int32_t al = base & ~3;
    const u32x2_a4 e = *reinterpret_cast<const u32x2_a4*>(excl + al);
    const uint64_t e64 = ((uint64_t)e[1] << 32 | e[0]) >> (8 * (base - al));
#pragma unroll
    for (int k = 0; k < 5; ++k)
      if ((e64 >> (8 * k)) & 0xffu) okm &= ~(1u << k);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const bool ok = (okm >> k) & 1u;
      q.n += ok ? 1 : 0;
      acc_voxel(q, ok ? a.v[k] : make_uint2(0, 0), ok ? b.v[k] : make_uint2(0, 0));
    }
  } else {
    // voxel by voxel: fewer registers than a masked row (the unmasked pass
    // keeps its occupancy)
    const int32_t tt = pt + dt, yy = py + dy;
    const bool rok = tt >= 0 && tt < L.T && yy >= 0 && yy < L.H;
#pragma unroll
    for (int dx = -2; dx <= 2; ++dx) {
      const int32_t xx = px + dx;
      const bool ok = rok && xx >= 0 && xx < L.W;
      const int32_t ai = ok ? p + row + dx : p;
      uint2 a = vox[ai];
      uint2 bb = b.v[dx + 2];
      if (!ok) {
        a = make_uint2(0, 0);
        bb = make_uint2(0, 0);
      }
      q.n += ok ? 1 : 0;
      acc_voxel(q, a, bb);
    }
  }
}

// The centre row, then twelve groups of two rows in a loop that is not
// unrolled: the two rows of a group are fetched together, and the code stays
// small enough for the instruction cache although the kernels inline it at
// several call sites.
template <bool FULL, bool MASKED, bool ABORT>
__device__ __forceinline__ uint32_t ssd_groups(const DevLevel& L, const uint8_t* excl, int32_t p,
                                               int32_t px, int32_t py, int32_t pt, int32_t c,
                                               uint32_t abort_above, int32_t& nvox) {
  SsdAcc q{0u, 0u, 0};
  const uint32_t lam = (uint32_t)L.lambda;
  // 25 rows (dt, dy) of a video patch, or the 5 rows of an image patch; the
  // row counts after the centre (24, 4) are multiples of both group sizes
  const bool vid = L.ht != 0;
  const int nrows = vid ? 25 : 5;
  const int8_t* rdt = vid ? kRowDt : kRowDt2;
  const int8_t* rdy = vid ? kRowDy : kRowDy2;
  ssd_row<FULL, MASKED>(L, excl, p, px, py, pt, c, 0, 0, q);
  if (ABORT) {
#pragma unroll 1
    for (int r = 1; r < nrows; r += 2) {
      if (q.sc + lam * q.st > abort_above) break;
      ssd_row<FULL, MASKED>(L, excl, p, px, py, pt, c, rdt[r], rdy[r], q);
      ssd_row<FULL, MASKED>(L, excl, p, px, py, pt, c, rdt[r + 1], rdy[r + 1], q);
    }
  } else {
    // without early exit nothing orders the rows: four in flight at a time
#pragma unroll 1
    for (int r = 1; r < nrows; r += 4) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        ssd_row<FULL, MASKED>(L, excl, p, px, py, pt, c, rdt[r + j], rdy[r + j], q);
    }
  }
  nvox = FULL ? (vid ? 125 : 25) : q.n;
  return q.sc + lam * q.st;
}

template <bool MASKED, bool ABORT>
__device__ __forceinline__ uint32_t patch_ssd(const DevLevel& L, const uint8_t* __restrict__ excl,
                                              int32_t p, int32_t px, int32_t py, int32_t pt,
                                              int32_t c, uint32_t abort_above, int32_t& nvox) {
  const bool interior = !MASKED && px >= 2 && py >= 2 && pt >= L.ht && px < L.W - 2 &&
                        py < L.H - 2 && pt < L.T - L.ht;
  // wave-uniform choice: a whole wave of interior targets needs no masks
  if (__all(interior))
    return ssd_groups<true, MASKED, ABORT>(L, excl, p, px, py, pt, c, abort_above, nvox);
  return ssd_groups<false, MASKED, ABORT>(L, excl, p, px, py, pt, c, abort_above, nvox);
}

// Reduced distance of the dimensionality-reduced patch space: the sum over
// the level's rd features (a multiple of four, zero padded) of
// (f(p) - f(c))^2, saturated at 2^31 - 1.  Features are below 2^23 in
// magnitude, so a difference fits in 32 bits and a square at or above 2^31
// saturates at once.
__device__ __forceinline__ uint32_t red_dist(const DevLevel& L, int32_t p, int32_t c) {
  const int4* a = reinterpret_cast<const int4*>(L.feat + (size_t)p * L.rd);
  const int4* b = reinterpret_cast<const int4*>(L.feat + (size_t)c * L.rd);
  uint32_t s = 0;
  for (int k = 0; k < L.rd / 4; ++k) {
    const int4 u = a[k], v = b[k];
    const int32_t e[4] = {u.x - v.x, u.y - v.y, u.z - v.z, u.w - v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t m = (uint32_t)abs(e[j]);
      const uint32_t sq = m >= 46341u ? 0x7fffffffu : m * m;
      s = min(s + sq, 0x7fffffffu);
    }
  }
  return s;
}

// Wave-wide reductions with DPP row operations instead of LDS permutes:
// adjacent lanes, quads, half rows and rows of 16 by swizzles within a row,
// then the four rows through row_bcast:15 (rows 1 and 3) and row_bcast:31
// (rows 2 and 3), which leaves the total in lane 63; it is read back as a
// wave-uniform value.  Lanes outside a broadcast's rows receive the neutral
// element.  Every lane of the wave must be active.
template <typename Op>
__device__ __forceinline__ uint32_t dpp_reduce(uint32_t v, Op op) {
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // half mirror
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // mirror
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));  // bcast 15
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));  // bcast 31
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// float sum over the wave (the order of the additions is fixed: sums of
// integers below 2^24 are exact)
__device__ __forceinline__ float wave_sum_f32(float x) {
  return __uint_as_float(dpp_reduce(__float_as_uint(x), [](uint32_t a, uint32_t b) {
    return __float_as_uint(__uint_as_float(a) + __uint_as_float(b));
  }));
}

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t x) {
  return dpp_reduce(x, [](uint32_t a, uint32_t b) { return a | b; });
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// adds the wave's sum of v to the spread counter at base (every lane calls)
__device__ __forceinline__ void add_spread(unsigned long long* base, unsigned long long v) {
  const unsigned long long s = wave_sum_u64(v);
  if ((threadIdx.x & 63) == 0 && s) {
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    atomicAdd(base + (wave & (kCntSlots - 1)) * kCntStride, s);
  }
}

__device__ __forceinline__ void count_evals(unsigned long long* evals, int n) {
  if (!evals) return;
  add_spread(evals, (unsigned long long)n);
}

// ------------------------------------------------------------------------
// Step 0 of the search: random initialisation of targets whose match is
// missing or not a source (Philox purpose 1), then the distance of every
// target's match on the current video.
// ------------------------------------------------------------------------
template <bool MASKED, bool RED = false>
__device__ __forceinline__ int s0_target(const DevLevel& L, const PassArgs& A, int32_t i) {
  if (i >= A.nS) return 0;
  const int32_t p = A.tlist[i];
  int32_t px, py, pt;
  unlin(L, p, px, py, pt);
  int2* nnf = const_cast<int2*>(A.nin);
  const int2 old = nnf[p];
  const uint8_t n_old = L.nvox[p];
  int32_t c = old.x;
  if (c < 0 || c >= L.V || !L.dsrc[c]) {
    uint64_t w[4];
    philox4x64_10((uint64_t)p, A.step, 0, ((uint64_t)L.level << 8) | 1u, L.seed, 0, w);
    c = L.dlist[draw_below(w[0], (uint32_t)L.nD)];
  }
  if (RED) {
    // the reduced distance; the exact one (and the count and the marks) is
    // written after the search, which compares it with the entry kept here
    L.prev[p] = old;
    nnf[p] = make_int2(c, (int32_t)red_dist(L, p, c));
    L.chg[p] = 0;
    return 1;
  }
  int32_t n;
  const uint32_t d = patch_ssd<MASKED, false>(L, A.excl, p, px, py, pt, c, 0xffffffffu, n);
  nnf[p] = make_int2(c, (int32_t)d);
  L.nvox[p] = (uint8_t)n;
  L.chg[p] = 0;
  if (c != old.x || (int32_t)d != old.y || (uint8_t)n != n_old) L.rmark[p] = (uint8_t)L.repoch;
  return 1;
}

template <bool MASKED, bool RED>
__global__ __launch_bounds__(kBlock) void k_s0(DevLevel L, PassArgs A) {
  const int ne = s0_target<MASKED, RED>(L, A, blockIdx.x * kBlock + threadIdx.x);
  count_evals(A.evals, ne);
}

// After a search with the reduced distance: every target's match evaluated
// with the exact patch distance, which the reconstruction weights use; a
// target whose (match, distance, count) differs from before the search is
// marked for the next reconstruction, as step 0 of an exact search marks.
__global__ __launch_bounds__(kBlock) void k_rerank(DevLevel L, const int32_t* __restrict__ tlist,
                                                   int32_t nS) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nS) return;
  const int32_t p = tlist[i];
  int32_t px, py, pt;
  unlin(L, p, px, py, pt);
  const int32_t c = L.nnf0[p].x;
  int32_t n;
  const uint32_t d = patch_ssd<false, false>(L, nullptr, p, px, py, pt, c, 0xffffffffu, n);
  const int2 old = L.prev[p];
  const uint8_t n_old = L.nvox[p];
  L.nnf0[p] = make_int2(c, (int32_t)d);
  L.nvox[p] = (uint8_t)n;
  if (c != old.x || (int32_t)d != old.y || (uint8_t)n != n_old) L.rmark[p] = (uint8_t)L.repoch;
}

// Block index -> logical block such that the workgroups that land on one XCD
// (dispatch is round-robin over the 8 XCDs) process one contiguous range of
// targets, which share candidate voxels and neighbour entries in that XCD's L2.
__device__ __forceinline__ int32_t xcd_block(int32_t b, int32_t nb) {
  constexpr int32_t kXcd = 8;
  const int32_t x = b % kXcd, y = b / kXcd;
  const int32_t q = nb / kXcd, r = nb % kXcd;
  return x * q + (x < r ? x : r) + y;
}

__device__ __forceinline__ int lane_prefix(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ------------------------------------------------------------------------
// One Jacobi propagation pass at stride s (candidate i = 1..6 is the shift of
// the neighbour p -/+ s along x, y, t, applied at p), followed, when rs_k > 0,
// by the random search of iteration rs_k (Eq. (3.1)).  The new match
// minimises (distance, candidate index); a candidate equal to the incumbent
// or to an earlier candidate cannot win and is not evaluated.
//
// The candidate of neighbour q = p + d is c = cand(q) - d.  cand(q) is a
// source, so its coordinates lie in [2, dim-3]; for |d| <= 4 a shifted
// coordinate outside the volume wraps, in linear order, onto a coordinate in
// {0, 1, dim-2, dim-1} of an adjacent row or frame, or out of [0, V), none of
// which is a source: the linear test 0 <= c < V && dsrc[c] is therefore the
// exact vector test.
//
// A workgroup of 256 targets works in three phases: (1) each thread gathers
// its target's candidates and appends (target, direction) entries to an LDS
// queue, grouped per wave and direction so that neighbouring entries point
// at neighbouring voxels; (2) all threads evaluate the queue densely (one
// lane per entry; in the GQ instantiation a short queue takes one group of
// kGrp lanes per entry) and fold (distance << 3 | index) into the target's
// LDS minimum with a 64-bit atomic min, which is exactly the lexicographic
// (distance, index) order; (3) each thread takes its target's winner and
// runs the random search.
// ------------------------------------------------------------------------
template <int BLK>
struct PassShared {
  int32_t p[BLK];
  int32_t xy[BLK];
  int32_t t[BLK];
  unsigned long long best[BLK];
  int32_t cand[BLK * 6];
  uint16_t q[BLK * 6];
  int32_t nq;
};

// Propagation candidates of one target (phase 1): candidate j (0..5) goes to
// s_cand[slot * 6 + j], and the candidates that can win are appended to the
// LDS queue as (slot | j << 8), grouped per wave and direction.  Reports
// whether the target is stable and its own change mark.  Every lane of the
// calling waves must call it together (wave ballots).
template <bool MASKED>
__device__ __forceinline__ void gather_candidates(const DevLevel& L, const PassArgs& A,
                                                  bool active, int32_t p, int32_t px, int32_t py,
                                                  int32_t pt, int2 inc, int slot,
                                                  int32_t* s_cand, uint16_t* s_q, int32_t& s_nq,
                                                  bool& stable, uint16_t& cp) {
  const int32_t s = A.s;
  int32_t c[6];
  bool v[6];
  int32_t qi[6];
  bool qok[6];
  // the gathers are unconditional (clamped to p), so the six neighbours'
  // marks, then their entries, then the six source flags, are fetched
  // together
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int axis = j >> 1;
    const int32_t sgn = (j & 1) ? 1 : -1;
    const int32_t coord = axis == 0 ? px : (axis == 1 ? py : pt);
    const int32_t dim = axis == 0 ? L.W : (axis == 1 ? L.H : L.T);
    const int32_t stride = axis == 0 ? 1 : (axis == 1 ? L.W : L.WH);
    const int32_t qc = coord + sgn * s;
    // nothing beats a perfect incumbent: (0, index 0) is the minimum
    qok[j] = active && inc.y != 0 && qc >= 0 && qc < dim;
    qi[j] = qok[j] ? p + sgn * s * stride : p;
  }
  uint16_t cg[6];
  if (A.since > 0) {
    cp = active ? L.chg[p] : (uint16_t)0;
#pragma unroll
    for (int j = 0; j < 6; ++j) cg[j] = L.chg[qi[j]];
  }
  if (MASKED) {
#pragma unroll
    for (int j = 0; j < 6; ++j) qok[j] = qok[j] && A.smask[qi[j]] != 0;
  }
  // Within a search the video is fixed, so distances are.  A target whose
  // match is unchanged since its previous pass at this stride, and whose
  // neighbours in the target set are unchanged since before that pass,
  // sees exactly the candidates that lost to its match then: it keeps it.
  // A neighbour's mark read while it is being rewritten only holds this
  // pass (no skip).  Neighbours outside the target set give no candidate.
  stable = A.since > 0 && active && cp <= A.since;
  if (A.since > 0) {
#pragma unroll
    for (int j = 0; j < 6; ++j) stable = stable && (!qok[j] || cg[j] < A.since);
  }
  // a stable target needs neither its neighbours' matches nor the source
  // flags of their candidates
  int32_t cq[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    qok[j] = qok[j] && !stable;
    cq[j] = -1;
  }
  if (!stable) {
#pragma unroll
    for (int j = 0; j < 6; ++j) cq[j] = A.nin[qi[j]].x;
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int axis = j >> 1;
    const int32_t sgn = (j & 1) ? 1 : -1;
    const int32_t stride = axis == 0 ? 1 : (axis == 1 ? L.W : L.WH);
    // unmasked search: the target set is H~, where every entry holds a
    // match after step 0 and every other entry holds -1 in both buffers
    if (!MASKED) qok[j] = qok[j] && cq[j] >= 0;
    c[j] = cq[j] - sgn * s * stride;
    qok[j] = qok[j] && c[j] >= 0 && c[j] < L.V;
  }
  uint8_t ds[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) ds[j] = 0;
  if (!stable) {
#pragma unroll
    for (int j = 0; j < 6; ++j) ds[j] = L.dsrc[qok[j] ? c[j] : 0];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    bool ok = qok[j] && ds[j] && c[j] != inc.x;
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (k < j) ok = ok && !(v[k] && c[k] == c[j]);
    v[j] = ok;
    s_cand[slot * 6 + j] = c[j];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const uint64_t bal = __ballot(v[j]);
    const int cnt = __popcll(bal);
    int base = 0;
    if ((threadIdx.x & 63) == 0 && cnt) base = atomicAdd(&s_nq, cnt);
    base = __builtin_amdgcn_readlane(base, 0);
    if (v[j]) s_q[base + lane_prefix(bal)] = (uint16_t)(slot | (j << 8));
  }
}

// The random-search candidate of iteration A.rs_k around best_c (Eq. (3.1)):
// a uniform draw per axis over the window of radius A.R clipped to the
// centres whose patch lies inside the volume (Philox purpose 0).
__device__ __forceinline__ int32_t random_candidate(const DevLevel& L, const PassArgs& A,
                                                    int32_t p, int32_t best_c) {
  int32_t cx, cy, ct;
  unlin(L, best_c, cx, cy, ct);
  const int32_t R = A.R;
  const int32_t lox = max(2, cx - R), hix = min(L.W - 3, cx + R);
  const int32_t loy = max(2, cy - R), hiy = min(L.H - 3, cy + R);
  const int32_t lot = max(L.ht, ct - R), hit = min(L.T - 1 - L.ht, ct + R);
  uint64_t w[4];
  philox4x64_10((uint64_t)p, A.step, (uint64_t)A.rs_k, ((uint64_t)L.level << 8) | 0u, L.seed, 0,
                w);
  const int32_t rx = lox + draw_below(w[0], (uint32_t)(hix - lox + 1));
  const int32_t ry = loy + draw_below(w[1], (uint32_t)(hiy - loy + 1));
  const int32_t rt = lot + draw_below(w[2], (uint32_t)(hit - lot + 1));
  return (rt * L.H + ry) * L.W + rx;
}

// The pass's result for one target: its entry in the output state and, when
// its match changed, its marks.
__device__ __forceinline__ void store_match(const DevLevel& L, const PassArgs& A, int32_t p,
                                            bool stable, uint16_t cp, int2 inc, int32_t best_c,
                                            uint32_t best_d) {
  // A stable target unchanged for two passes already holds this entry in
  // both buffers: the write is skipped.
  if (!(stable && (int32_t)cp + 2 <= A.t && best_c == inc.x))
    A.nout[p] = make_int2(best_c, (int32_t)best_d);
  if (best_c != inc.x) {
    L.chg[p] = (uint16_t)A.t;
    L.rmark[p] = (uint8_t)L.repoch;
  }
}

// Target lists up to this size take the wide pass (kWideTargets targets per
// workgroup of kBlock lanes).  Larger ones take the one-lane pass: with its
// 76 registers six of its workgroups (1536 targets) are resident per compute
// unit against five of the wide pass's (320 targets, 83 registers), and its
// early exit costs fewer loads, so once the targets fill the device it is
// faster (measured crossover between 72 k and 220 k targets).
constexpr int32_t kWideMaxTargets = 131072;
constexpr int kWideTargets = 64;
// Step 0's target lists up to this size take the group form as well.
constexpr int32_t kWideS0MaxTargets = 131072;

constexpr int kGrp = 8;
// Unmasked exact passes without random search over the larger lists: a
// workgroup of 256 targets whose queue holds at most this many candidates
// (in proportion for smaller workgroups) evaluates them with lane groups
// (two round trips at most) instead of one lane each (up to 13 with early
// exit); a longer queue keeps one lane each.
constexpr int32_t kGroupQueueMax = 64;

// Rows of a video patch for the lanes of a group: slot k of lane g holds the
// row with index 8k + g in the centre-out order of the one-lane distance,
// coded (dt + 2) | (dy + 2) << 3 in six bits per lane; 63 marks no row.
constexpr int8_t kCoDt[25] = {0, 0, 0, -1, 1, 0, 0, -1, -1, 1, 1, -2, 2,
                              -1, -1, 1, 1, -2, -2, 2, 2, -2, -2, 2, 2};
constexpr int8_t kCoDy[25] = {0, -1, 1, 0, 0, -2, 2, -1, 1, -1, 1, 0, 0,
                              -2, 2, -2, 2, -1, 1, -1, 1, -2, 2, -2, 2};
constexpr uint64_t slot_rows(int k) {
  uint64_t v = 0;
  for (int g = 0; g < 8; ++g) {
    const int r = 8 * k + g;
    const uint64_t code = r < 25 ? (uint64_t)((kCoDt[r] + 2) | ((kCoDy[r] + 2) << 3)) : 63u;
    v |= code << (6 * g);
  }
  return v;
}
constexpr uint64_t kSlotRows[4] = {slot_rows(0), slot_rows(1), slot_rows(2), slot_rows(3)};

// Patch distance computed by the kGrp lanes of a group (target voxels
// outside the volume, or flagged in excl when MASKED, are not compared; the
// candidate patch is a source, inside the volume).  A video patch: first
// the eight rows nearest the centre, one per lane, and the 25th row on lane
// 0; when the group's partial sum already exceeds abort_above the
// evaluation stops there (the full distance could only be larger, as in the
// one-lane form), otherwise the 16 other rows follow, two per lane, all
// loads in flight at once.  An image patch: its five rows on lanes 0-4.  The
// lanes' sums are added with DPP within each group of eight lanes (quad
// swaps, then the half-row mirror), modulo 2^32 like the one-lane sum, so
// the full distance is the same.  Returns the full distance when it is
// <= abort_above, otherwise some value above it.  Every lane of the group
// must call it together with the same arguments.
__device__ __forceinline__ uint32_t group_sum8(uint32_t d) {
  d += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)d, 0xB1, 0xF, 0xF, false);   // [1,0,3,2]
  d += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)d, 0x4E, 0xF, 0xF, false);   // [2,3,0,1]
  d += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)d, 0x141, 0xF, 0xF, false);  // half mirror
  return d;
}

// the group's sum over the rows of slots SA and SB (SB < 0: none) of lane lg;
// a slot without a row on this lane loads nothing and adds nothing
template <int SA, int SB, bool MASKED>
__device__ __forceinline__ uint32_t group_rows(const DevLevel& L, const uint8_t* __restrict__ excl,
                                               int32_t p, int32_t py, int32_t pt, int32_t c,
                                               int lg, uint32_t xm, bool vid,
                                               uint32_t* nvox = nullptr) {
  constexpr int NS = SB < 0 ? 1 : 2;
  const uint2* __restrict__ vox = L.vox;
  Row5 a[NS], b[NS];
  uint32_t okm[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int k = i == 0 ? SA : SB;
    int dt, dy;
    bool rv;
    if (vid) {
      const uint32_t code = (uint32_t)(kSlotRows[k] >> (6 * lg)) & 63u;
      rv = code != 63u;
      dt = rv ? (int)(code & 7u) - 2 : 0;
      dy = rv ? (int)(code >> 3) - 2 : 0;
    } else {
      rv = k == 0 && lg < 5;
      dt = 0;
      dy = rv ? lg - 2 : 0;
    }
    const int32_t tt = pt + dt, yy = py + dy;
    const bool rok = rv && tt >= 0 && tt < L.T && yy >= 0 && yy < L.H;
    const int32_t row = dt * L.WH + dy * L.W;
    okm[i] = rok ? xm : 0u;
    if (rv) {
      // the video holds two voxels of padding on both sides; a target row
      // outside the volume reads the centre row and is masked
      const int32_t base = (rok ? p + row : p) - 2;
      b[i] = load_row5(vox + (c + row - 2));
      a[i] = load_row5(vox + base);
      if (MASKED) {
        // the row's five exclusion bytes with one 8-byte load (the masks
        // hold 16 bytes of padding on both sides)
        const int32_t al = base & ~3;
        const u32x2_a4 e = *reinterpret_cast<const u32x2_a4*>(excl + al);
        const uint64_t e64 = ((uint64_t)e[1] << 32 | e[0]) >> (8 * (base - al));
#pragma unroll
        for (int x = 0; x < 5; ++x)
          if ((e64 >> (8 * x)) & 0xffu) okm[i] &= ~(1u << x);
      }
    } else {
#pragma unroll
      for (int x = 0; x < 5; ++x) a[i].v[x] = b[i].v[x] = make_uint2(0, 0);
    }
  }
  SsdAcc q{0u, 0u, 0};
#pragma unroll
  for (int i = 0; i < NS; ++i) {
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      const bool ok = (okm[i] >> x) & 1u;
      acc_voxel(q, ok ? a[i].v[x] : make_uint2(0, 0), ok ? b[i].v[x] : make_uint2(0, 0));
    }
  }
  // the voxels compared, summed over the group
  if (nvox) {
    uint32_t n = 0;
#pragma unroll
    for (int i = 0; i < NS; ++i) n += __builtin_popcount(okm[i]);
    *nvox = group_sum8(n);
  }
  return group_sum8(q.sc + (uint32_t)L.lambda * q.st);
}

template <bool MASKED>
__device__ __forceinline__ uint32_t group_ssd(const DevLevel& L, const uint8_t* excl, int32_t p,
                                              int32_t px, int32_t py, int32_t pt, int32_t c,
                                              int lg, uint32_t abort_above) {
  const bool vid = L.ht != 0;
  const int klo = px < 2 ? 2 - px : 0;
  const int khi = px + 2 >= L.W ? L.W + 1 - px : 4;
  const uint32_t xm = (0x1fu << klo) & (0x1fu >> (4 - khi));
  const uint32_t d0 = group_rows<0, 3, MASKED>(L, excl, p, py, pt, c, lg, xm, vid);
  if (!vid || d0 > abort_above) return d0;
  return d0 + group_rows<1, 2, MASKED>(L, excl, p, py, pt, c, lg, xm, true);
}

// The full distance (no early exit) and the number of voxels compared, by
// the kGrp lanes of a group, every row load of a video patch in flight at
// once.
template <bool MASKED>
__device__ __forceinline__ uint32_t group_full(const DevLevel& L, const uint8_t* excl, int32_t p,
                                               int32_t px, int32_t py, int32_t pt, int32_t c,
                                               int lg, uint32_t& nvox) {
  const bool vid = L.ht != 0;
  const int klo = px < 2 ? 2 - px : 0;
  const int khi = px + 2 >= L.W ? L.W + 1 - px : 4;
  const uint32_t xm = (0x1fu << klo) & (0x1fu >> (4 - khi));
  uint32_t n0, n1 = 0;
  uint32_t d = group_rows<0, 3, MASKED>(L, excl, p, py, pt, c, lg, xm, vid, &n0);
  if (vid) d += group_rows<1, 2, MASKED>(L, excl, p, py, pt, c, lg, xm, true, &n1);
  nvox = n0 + n1;
  return d;
}

// One block of BLK consecutive targets (block index blk of the target list);
// returns the evaluations this thread accounts for.  All threads of the
// workgroup must call it together.
template <int BLK, bool MASKED, bool RED = false, bool GQ = false>
__device__ __forceinline__ int pass_block(const DevLevel& L, const PassArgs& A, int32_t blk,
                                          PassShared<BLK>& sh) {
  static_assert(!GQ || (!MASKED && !RED), "group evaluation: unmasked exact distances");
  int32_t* s_p = sh.p;
  int32_t* s_xy = sh.xy;
  int32_t* s_t = sh.t;
  unsigned long long* s_best = sh.best;
  int32_t* s_cand = sh.cand;
  uint16_t* s_q = sh.q;
  int32_t& s_nq = sh.nq;
  const int tid = threadIdx.x;
  const int32_t i = blk * BLK + tid;
  __syncthreads();  // the previous block's readers are done with the LDS
  const bool active = i < A.nS;
  int32_t p = 0, px = 0, py = 0, pt = 0;
  int2 inc = make_int2(0, 0);
  if (tid == 0) s_nq = 0;
  if (active) {
    p = A.tlist[i];
    unlin(L, p, px, py, pt);
    inc = A.nin[p];
    s_best[tid] = (unsigned long long)(uint32_t)inc.y << 3;
  }
  s_p[tid] = p;
  s_xy[tid] = px | (py << 16);
  s_t[tid] = pt;
  __syncthreads();
  int ne = 0;
  bool stable = false;
  uint16_t cp = 0;
  if (A.s > 0) {
    gather_candidates<MASKED>(L, A, active, p, px, py, pt, inc, tid, s_cand, s_q, s_nq, stable,
                              cp);
    __syncthreads();
    const int32_t nq = s_nq;
    if (GQ && nq <= kGroupQueueMax * BLK / kBlock) {
      // a short queue: one group of kGrp lanes per candidate
      const int g = tid / kGrp, lg = tid % kGrp;
      for (int32_t e = g; e < nq; e += BLK / kGrp) {
        const uint32_t ent = s_q[e];
        const int lt = ent & 255, j = ent >> 8;
        const int32_t xy = s_xy[lt];
        const uint32_t bound = (uint32_t)(s_best[lt] >> 3);
        const uint32_t d = group_ssd<false>(L, nullptr, s_p[lt], xy & 0xFFFF, xy >> 16,
                                            s_t[lt], s_cand[lt * 6 + j], lg, bound);
        if (lg == 0 && d <= bound)
          atomicMin(&s_best[lt], ((unsigned long long)d << 3) | (unsigned long long)(j + 1));
      }
    } else {
      // one lane per candidate, with early exit
      for (int32_t e = tid; e < nq; e += BLK) {
        const uint32_t ent = s_q[e];
        const int lt = ent & 255, j = ent >> 8;
        const int32_t xy = s_xy[lt];
        // a candidate whose partial distance exceeds the current best cannot win
        const uint32_t bound = (uint32_t)(s_best[lt] >> 3);
        int32_t n;
        const uint32_t d =
            RED ? red_dist(L, s_p[lt], s_cand[lt * 6 + j])
                : patch_ssd<MASKED, true>(L, A.excl, s_p[lt], xy & 0xFFFF, xy >> 16, s_t[lt],
                                          s_cand[lt * 6 + j], bound, n);
        if (d <= bound)
          atomicMin(&s_best[lt], ((unsigned long long)d << 3) | (unsigned long long)(j + 1));
      }
    }
    if (tid == 0) ne += nq;
    __syncthreads();
  }
  if (active) {
    const unsigned long long key = s_best[tid];
    const int slot = (int)(key & 7);
    uint32_t best_d = (uint32_t)(key >> 3);
    int32_t best_c = slot ? s_cand[tid * 6 + slot - 1] : inc.x;
    // best_c >= 0 for every target once step 0 has run; a target without a
    // match (cand -1) is left to step 0 rather than searched around
    if (A.rs_k > 0 && best_c >= 0) {
      const int32_t rc = random_candidate(L, A, p, best_c);
      // strictly better only: nothing beats distance 0.  The window keeps the
      // whole candidate patch inside the volume, so the distance can be
      // computed before the source test, which is only needed (and its
      // random byte fetched) when the candidate would win.
      const int nr = (best_d != 0 && rc != best_c) ? 1 : 0;
      if (nr) {
        int32_t n;
        const uint32_t d = RED ? red_dist(L, p, rc)
                               : patch_ssd<MASKED, true>(L, A.excl, p, px, py, pt, rc,
                                                         best_d - 1u, n);
        if (d < best_d && L.dsrc[rc]) {
          best_d = d;
          best_c = rc;
        }
      }
      ne += nr;
    }
    store_match(L, A, p, stable, cp, inc, best_c, best_d);
  }
  return ne;
}

// ------------------------------------------------------------------------
// The same pass for levels with few targets, where one workgroup per 256
// targets leaves most compute units idle and a pass takes as long as the
// longest chain of dependent fetches in a wave: a queued candidate with early
// exit is up to 13 round trips, its random-search candidate 13 more.  Here a
// group of kGrp lanes computes one candidate's distance (group_ssd: two
// round trips at most), for the queued candidates and then for the
// random-search candidates, and a workgroup of 256 lanes serves TB targets.
// The same candidates win with the same distances, and the same evaluations
// are counted.  MASKED: the onion peel's passes (target set and exclusions
// as in the one-lane form).
// ------------------------------------------------------------------------
template <int TB>
struct WideShared {
  PassShared<TB> s;
  int32_t rc[TB];   // random-search candidate of the target, or -1
  uint32_t rd[TB];  // its distance
};

// One block of TB consecutive targets with NT = kBlock lanes (exact
// distance); returns the evaluations this thread accounts for.
template <int TB, bool MASKED>
__device__ __forceinline__ int pass_block_wide(const DevLevel& L, const PassArgs& A, int32_t blk,
                                               WideShared<TB>& wsh) {
  static_assert(TB % 64 == 0 && TB <= kBlock, "targets per workgroup: whole waves");
  PassShared<TB>& sh = wsh.s;
  const int tid = threadIdx.x;
  const bool tgt = tid < TB;  // wave-uniform
  const int32_t i = blk * TB + tid;
  const bool active = tgt && i < A.nS;
  int32_t p = 0, px = 0, py = 0, pt = 0;
  int2 inc = make_int2(0, 0);
  if (tid == 0) sh.nq = 0;
  if (active) {
    p = A.tlist[i];
    unlin(L, p, px, py, pt);
    inc = A.nin[p];
    sh.best[tid] = (unsigned long long)(uint32_t)inc.y << 3;
  }
  if (tgt) {
    sh.p[tid] = p;
    sh.xy[tid] = px | (py << 16);
    sh.t[tid] = pt;
  }
  __syncthreads();
  const int g = tid / kGrp, lg = tid % kGrp;
  constexpr int kGroups = kBlock / kGrp;
  int ne = 0;
  bool stable = false;
  uint16_t cp = 0;
  if (A.s > 0) {
    if (tgt)
      gather_candidates<MASKED>(L, A, active, p, px, py, pt, inc, tid, sh.cand, sh.q, sh.nq,
                                stable, cp);
    __syncthreads();
    const int32_t nq = sh.nq;
    for (int32_t e = g; e < nq; e += kGroups) {
      const uint32_t ent = sh.q[e];
      const int lt = ent & 255, j = ent >> 8;
      const int32_t xy = sh.xy[lt];
      // a candidate whose partial distance exceeds the current best cannot win
      const uint32_t bound = (uint32_t)(sh.best[lt] >> 3);
      const uint32_t d = group_ssd<MASKED>(L, A.excl, sh.p[lt], xy & 0xFFFF, xy >> 16,
                                           sh.t[lt], sh.cand[lt * 6 + j], lg, bound);
      if (lg == 0 && d <= bound)
        atomicMin(&sh.best[lt], ((unsigned long long)d << 3) | (unsigned long long)(j + 1));
    }
    if (tid == 0) ne += nq;
    __syncthreads();
  }
  uint32_t best_d = 0;
  int32_t best_c = -1;
  int32_t rc = -1;
  if (active) {
    const unsigned long long key = sh.best[tid];
    const int slot = (int)(key & 7);
    best_d = (uint32_t)(key >> 3);
    best_c = slot ? sh.cand[tid * 6 + slot - 1] : inc.x;
    // as in the one-lane pass: no search around a missing match, and
    // nothing beats distance 0
    if (A.rs_k > 0 && best_c >= 0) {
      const int32_t r = random_candidate(L, A, p, best_c);
      if (best_d != 0 && r != best_c) rc = r;
    }
  }
  if (A.rs_k > 0) {
    if (tgt) {
      wsh.rc[tid] = rc;
      wsh.rd[tid] = best_d - 1u;  // strictly better only (best_d > 0 when rc >= 0)
    }
    __syncthreads();
    for (int e = g; e < TB; e += kGroups) {
      const int32_t c = wsh.rc[e];
      if (c >= 0) {
        const int32_t xy = sh.xy[e];
        const uint32_t d =
            group_ssd<MASKED>(L, A.excl, sh.p[e], xy & 0xFFFF, xy >> 16, sh.t[e], c, lg,
                              wsh.rd[e]);
        if (lg == 0) wsh.rd[e] = d;
      }
    }
    __syncthreads();
    if (rc >= 0) {
      const uint32_t d = wsh.rd[tid];
      if (d < best_d && L.dsrc[rc]) {
        best_d = d;
        best_c = rc;
      }
      ne += 1;
    }
  }
  if (active) store_match(L, A, p, stable, cp, inc, best_c, best_d);
  return ne;
}

// GQ: short queues evaluated by lane groups (the unmasked exact passes
// without random search; a separate instantiation, so that the passes with
// random search keep the one-lane form's 76 registers and six waves per SIMD)
template <bool MASKED, bool RED, bool GQ>
__global__ __launch_bounds__(kBlock) void k_pass(DevLevel L, PassArgs A) {
  __shared__ PassShared<kBlock> sh;
  const int ne = pass_block<kBlock, MASKED, RED, GQ>(L, A, xcd_block(blockIdx.x, gridDim.x), sh);
  count_evals(A.evals, ne);
}

template <int TB, bool MASKED>
__global__ __launch_bounds__(kBlock) void k_pass_wide(DevLevel L, PassArgs A) {
  __shared__ WideShared<TB> sh;
  const int ne = pass_block_wide<TB, MASKED>(L, A, xcd_block(blockIdx.x, gridDim.x), sh);
  count_evals(A.evals, ne);
}

// Step 0 for small target lists: kWideTargets targets per workgroup of
// kBlock lanes, each target's distance by a group of kGrp lanes (the same
// random initialisation, distance, count and marks as s0_target).
template <bool MASKED>
__global__ __launch_bounds__(kBlock) void k_s0_wide(DevLevel L, PassArgs A) {
  constexpr int TB = kWideTargets;
  __shared__ int32_t s_p[TB], s_xy[TB], s_t[TB], s_c[TB];
  __shared__ uint32_t s_d[TB], s_n[TB];
  const int tid = threadIdx.x;
  const bool tgt = tid < TB;  // wave-uniform
  const int32_t i = xcd_block(blockIdx.x, gridDim.x) * TB + tid;
  const bool active = tgt && i < A.nS;
  int2* nnf = const_cast<int2*>(A.nin);
  int32_t p = 0, px = 0, py = 0, pt = 0, c = -1;
  int2 old = make_int2(0, 0);
  uint8_t n_old = 0;
  if (active) {
    p = A.tlist[i];
    unlin(L, p, px, py, pt);
    old = nnf[p];
    n_old = L.nvox[p];
    c = old.x;
    if (c < 0 || c >= L.V || !L.dsrc[c]) {
      uint64_t w[4];
      philox4x64_10((uint64_t)p, A.step, 0, ((uint64_t)L.level << 8) | 1u, L.seed, 0, w);
      c = L.dlist[draw_below(w[0], (uint32_t)L.nD)];
    }
  }
  if (tgt) {
    s_p[tid] = p;
    s_xy[tid] = px | (py << 16);
    s_t[tid] = pt;
    s_c[tid] = active ? c : -1;
  }
  __syncthreads();
  const int g = tid / kGrp, lg = tid % kGrp;
  for (int e = g; e < TB; e += kBlock / kGrp) {
    const int32_t ce = s_c[e];
    if (ce >= 0) {
      const int32_t xy = s_xy[e];
      uint32_t n;
      const uint32_t d =
          group_full<MASKED>(L, A.excl, s_p[e], xy & 0xFFFF, xy >> 16, s_t[e], ce, lg, n);
      if (lg == 0) {
        s_d[e] = d;
        s_n[e] = n;
      }
    }
  }
  __syncthreads();
  if (active) {
    const uint32_t d = s_d[tid];
    const uint8_t n = (uint8_t)s_n[tid];
    nnf[p] = make_int2(c, (int32_t)d);
    L.nvox[p] = n;
    L.chg[p] = 0;
    if (c != old.x || (int32_t)d != old.y || n != n_old) L.rmark[p] = (uint8_t)L.repoch;
  }
  count_evals(A.evals, active ? 1 : 0);
}

__global__ void k_copy_targets(const int32_t* tlist, int32_t nS, const int2* src, int2* dst) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < nS) dst[tlist[i]] = src[tlist[i]];
}

// ------------------------------------------------------------------------
// Reconstruction, one wavefront per hole pixel p (Sec. 3.2).  Lane l holds
// the contributors with offset index l and l + 64 (offsets enumerated
// dt-major, then dy, then dx): q = p - o votes u(cand(q) + o).
// delta_q = dist(q) / nvox(q) is ordered through its correctly rounded
// double, which is exact for ordering: distinct such fractions (numerators
// < 2^31, denominators <= 125) differ by more than the double spacing.
// WEIGHTED: sigma^2 is the ceil(3m/4)-th smallest delta (nearest rank),
// selected by a radix walk with wave ballots over the integer distances when
// all contributors share one voxel count, else over float32 keys and then
// the exact keys when a float value is shared by different deltas; weights
// exp(-delta_q / (2 sigma^2)) with the ratio formed as one double division of
// exact integer products, then float32.  BEST: (delta, offset index) argmin.
// ------------------------------------------------------------------------
// One wavefront reconstructs hole pixel number w of plist; lane 0 adds the
// pixel's |change| over the colour channels to my_abs.
template <int MODE, bool FILT>
__device__ __forceinline__ void recon_pixel(const DevLevel& L, const int32_t* __restrict__ plist,
                                            int32_t w, const uint8_t* __restrict__ excl,
                                            float* __restrict__ out_f,
                                            unsigned long long& my_abs) {
  const int lane = threadIdx.x & 63;
  {
    const int32_t p = plist[w];
    int32_t px, py, pt;
    unlin(L, p, px, py, pt);
    bool valid[2];
    int32_t dist[2], nv[2], oi[2];
    uint64_t key[2];
    uint2 v[2];
    // unconditional loads (an invalid contributor reads the pixel itself and
    // is masked), so both contributors' entries, then both votes, are
    // fetched together
    int32_t qq[2], off[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int32_t o = lane + 64 * k;
      oi[k] = o;
      const int32_t dx = o % 5 - 2, dy = (o / 5) % 5 - 2, dt = o / 25 - 2;
      const int32_t qx = px - dx, qy = py - dy, qt = pt - dt;
      valid[k] = o < 125 && qx >= 0 && qy >= 0 && qt >= 0 && qx < L.W && qy < L.H && qt < L.T;
      qq[k] = valid[k] ? (qt * L.H + qy) * L.W + qx : p;
      off[k] = (dt * L.H + dy) * L.W + dx;
    }
    int2 nn[2];
    uint8_t nb[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      nn[k] = L.nnf0[qq[k]];
      nb[k] = L.nvox[qq[k]];
      if (FILT) valid[k] = valid[k] && !excl[qq[k]];
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      // a masked contributor still needs an in-volume address for its vote
      const int32_t src = valid[k] ? nn[k].x + off[k] : p;
      v[k] = L.vox[src];
      dist[k] = valid[k] ? nn[k].y : 0;
      nv[k] = valid[k] ? (int32_t)nb[k] : 1;
      if (MODE == 2)
        key[k] = valid[k] ? (uint64_t)__double_as_longlong((double)dist[k] / (double)nv[k])
                          : ~0ull;
      if (!valid[k]) v[k] = make_uint2(0, 0);
    }
    float s[2] = {0.f, 0.f};
    int best_lane = 0, best_k = 0;
    if (MODE == 2) {
      // argmin of (delta, offset index): keys are exact, indices unique
      uint64_t bk = key[0];
      int32_t bo = oi[0];
      int bkk = 0;
      if (valid[1] && (key[1] < bk || !valid[0])) {
        bk = key[1];
        bo = oi[1];
        bkk = 1;
      }
      if (!valid[0] && !valid[1]) bo = 1 << 20;
      uint64_t gk = bk;
      int32_t go = bo;
      for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t ok2 = __shfl_xor(gk, off);
        const int32_t oo = __shfl_xor(go, off);
        if (ok2 < gk || (ok2 == gk && oo < go)) {
          gk = ok2;
          go = oo;
        }
      }
      // every lane holds the minimum: one wave-uniform copy
      const int32_t gu = __builtin_amdgcn_readfirstlane(go);
      best_lane = gu & 63;
      best_k = gu >> 6;
      (void)bkk;
    } else if (MODE == 1) {
      s[0] = valid[0] ? 1.f : 0.f;
      s[1] = valid[1] ? 1.f : 0.f;
    } else {
      // candidate sets as wave masks (slot 0 and slot 1 of every lane): the
      // selection runs on scalar registers, one ballot per slot and bit
      uint64_t a0 = __ballot(valid[0]), a1 = __ballot(valid[1]);
      const int m = __popcll(a0) + __popcll(a1);
      int rr = (3 * m + 3) >> 2;  // 1-based rank
      // When every valid contributor compared the same number of voxels (all
      // pixels away from the borders of the volume and of the onion's known
      // region), delta is ordered as the integer distance: the walk runs on
      // the distances themselves and no tie needs an exact second look.
      const int fs = a0 ? (int)__ffsll((unsigned long long)a0) - 1
                        : (int)__ffsll((unsigned long long)a1) - 1;
      const int32_t n_first = __builtin_amdgcn_readlane(a0 ? nv[0] : nv[1], fs);
      const bool uni =
          (__ballot(valid[0] && nv[0] != n_first) | __ballot(valid[1] && nv[1] != n_first)) == 0;
      uint32_t uk[2];
      if (uni) {
        uk[0] = (uint32_t)dist[0];
        uk[1] = (uint32_t)dist[1];
      } else {
        // float32 rounding of the exact double key: monotone, so the walk
        // selects the float group that holds the rr-th smallest delta
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          key[k] = valid[k] ? (uint64_t)__double_as_longlong((double)dist[k] / (double)nv[k])
                            : ~0ull;
          uk[k] = valid[k] ? __float_as_uint((float)__longlong_as_double((long long)key[k])) : 0u;
        }
      }
      // keys are below 2^31 (distances) or non-negative floats; the walk
      // starts at the highest bit any key has set
      uint32_t any = (valid[0] ? uk[0] : 0u) | (valid[1] ? uk[1] : 0u);
      any = wave_or_u32(any);
      const int top = any ? 31 - __builtin_clz(any) : -1;
      for (int b = top; b >= 0; --b) {
        const uint64_t t0 = __ballot((uk[0] >> b) & 1u), t1 = __ballot((uk[1] >> b) & 1u);
        const uint64_t z0 = a0 & ~t0, z1 = a1 & ~t1;
        const int cnt = __popcll(z0) + __popcll(z1);
        if (rr > cnt) {
          rr -= cnt;
          a0 &= t0;
          a1 &= t1;
        } else {
          a0 = z0;
          a1 = z1;
        }
        // one candidate left: it is the selected one
        if (__popcll(a0) + __popcll(a1) == 1) break;
      }
      // (a0, a1) now holds the contributors whose key equals the selected
      // one (or the one contributor left) and rr the rank among them; float
      // keys can merge distinct
      // deltas, which a walk over the exact keys of the group separates
      if (!uni) {
        const int gl = a0 ? (int)__ffsll((unsigned long long)a0) - 1
                          : (int)__ffsll((unsigned long long)a1) - 1;
        const uint64_t kl = a0 ? key[0] : key[1];
        const uint64_t kf =
            (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)kl, gl) |
            (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(kl >> 32), gl) << 32;
        const bool in0 = (a0 >> lane) & 1ull, in1 = (a1 >> lane) & 1ull;
        if ((__ballot(in0 && key[0] != kf) | __ballot(in1 && key[1] != kf)) != 0) {
          for (int b = 63; b >= 0; --b) {
            const uint64_t t0 = __ballot((key[0] >> b) & 1ull), t1 = __ballot((key[1] >> b) & 1ull);
            const uint64_t z0 = a0 & ~t0, z1 = a1 & ~t1;
            const int cnt = __popcll(z0) + __popcll(z1);
            if (rr > cnt) {
              rr -= cnt;
              a0 &= t0;
              a1 &= t1;
            } else {
              a0 = z0;
              a1 = z1;
            }
          }
        }
      }
      // a contributor holding the selected delta provides (dist_r, n_r)
      const int src_lane = a0 ? (int)__ffsll((unsigned long long)a0) - 1
                              : (int)__ffsll((unsigned long long)a1) - 1;
      const int src_k = a0 ? 0 : 1;
      const int32_t dr = __builtin_amdgcn_readlane(src_k == 0 ? dist[0] : dist[1], src_lane);
      const int32_t nr = __builtin_amdgcn_readlane(src_k == 0 ? nv[0] : nv[1], src_lane);
      // with one voxel count for all, delta_q / (2 sigma^2) = dist_q / (2 dist_r):
      // one reciprocal per pixel instead of a division per contributor
      const double inv2dr = uni && dr > 0 ? 1.0 / (2.0 * (double)dr) : 0.0;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (!valid[k]) continue;
        if (dr > 0) {
          float tq;
          if (uni) {
            tq = (float)((double)dist[k] * inv2dr);
          } else {
            const double num = (double)((int64_t)dist[k] * (int64_t)nr);
            const double den = (double)(2 * (int64_t)dr * (int64_t)nv[k]);
            tq = (float)(num / den);
          }
          // hardware exponential: the ceil(3m/4) contributors at or below the
          // percentile weigh at least e^-1/2, so underflow of the others is
          // immaterial
          s[k] = __expf(-tq);
        } else {
          s[k] = dist[k] == 0 ? 1.f : 0.f;
        }
      }
    }
    uint2 oldv = make_uint2(0, 0);
    if (lane == 0) oldv = L.vox[p];
    uint32_t nx, ny;
    if (MODE == 2) {
      const uint32_t vx0 = (uint32_t)__builtin_amdgcn_readlane((int)(best_k ? v[1].x : v[0].x), best_lane);
      const uint32_t vy0 = (uint32_t)__builtin_amdgcn_readlane((int)(best_k ? v[1].y : v[0].y), best_lane);
      nx = vx0;
      ny = vy0;
      if (lane == 0 && out_f) {
        float* o = out_f + 5 * (size_t)w;
        o[0] = (float)(nx & 255) / 255.f;
        o[1] = (float)((nx >> 8) & 255) / 255.f;
        o[2] = (float)((nx >> 16) & 255) / 255.f;
        o[3] = (float)(ny & 255) / 255.f;
        o[4] = (float)((ny >> 8) & 255) / 255.f;
      }
    } else {
      float acc[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[c] = 0.f;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const float sk = s[k];
        acc[0] = fmaf(sk, (float)(v[k].x & 255), acc[0]);
        acc[1] = fmaf(sk, (float)((v[k].x >> 8) & 255), acc[1]);
        acc[2] = fmaf(sk, (float)((v[k].x >> 16) & 255), acc[2]);
        acc[3] = fmaf(sk, (float)(v[k].y & 255), acc[3]);
        acc[4] = fmaf(sk, (float)((v[k].y >> 8) & 255), acc[4]);
        acc[5] += sk;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[c] = wave_sum_f32(acc[c]);
      uint32_t q8[5];
      // the weighted mean multiplies by one reciprocal; the plain mean (exact
      // parity) divides
      const float inv = 1.f / acc[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const float o = MODE == 0 ? acc[c] * inv : acc[c] / acc[5];
        const int qi = (int)floorf(o + 0.5f);
        q8[c] = (uint32_t)(qi > 255 ? 255 : qi);
        if (lane == 0 && out_f) out_f[5 * (size_t)w + c] = o / 255.f;
      }
      nx = q8[0] | (q8[1] << 8) | (q8[2] << 16);
      ny = q8[3] | (q8[4] << 8);
    }
    if (lane == 0) {
      L.vox[p] = make_uint2(nx, ny);
      int a = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int nvv = (int)((nx >> (8 * c)) & 255), ov = (int)((oldv.x >> (8 * c)) & 255);
        a += nvv > ov ? nvv - ov : ov - nvv;
      }
      my_abs += (unsigned long long)a;
    }
  }
}

// The hole pixels w0 + i*stride (i < 64, below end) that a reconstruction of
// epoch L.repoch has to recompute, as a wave mask (bit i): those with a
// contributor (a target of the 5x5x5 box around the pixel) whose mark is the
// epoch.  Lane i checks pixel i: the five marks of each of the 25 rows come
// with one 8-byte load from the multiple of 4 at or below the row's first
// entry (the mark array holds 16 entries of padding on both sides); a byte
// equal to the epoch sets the top bit of its flag byte (exact, no carry
// crosses bytes), and entries outside the volume are masked.  With skip
// false every pixel below end is returned.
__device__ __forceinline__ uint64_t recon_todo(const DevLevel& L,
                                               const int32_t* __restrict__ plist, int32_t w0,
                                               int32_t stride, int32_t end, bool skip) {
  const int lane = threadIdx.x & 63;
  const int32_t w = w0 + lane * stride;
  bool todo = w < end;
  if (skip && todo) {
    const int32_t p = plist[w];
    int32_t px, py, pt;
    unlin(L, p, px, py, pt);
    const uint32_t ee = (uint32_t)L.repoch * 0x01010101u;
    // flag bytes k = 0..4 (x offsets -2..2) inside the volume
    const int klo = px < 2 ? 2 - px : 0;
    const int khi = px + 2 >= L.W ? L.W + 1 - px : 4;
    uint64_t km = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k)
      if (k >= klo && k <= khi) km |= 0x80ull << (8 * k);
    uint64_t acc = 0;
#pragma unroll
    for (int dt = -2; dt <= 2; ++dt) {
      const int32_t qt = pt + dt;
#pragma unroll
      for (int dy = -2; dy <= 2; ++dy) {
        const int32_t qy = py + dy;
        if (qt < 0 || qt >= L.T || qy < 0 || qy >= L.H) continue;
        const int32_t qb = (qt * L.H + qy) * L.W + px - 2;  // >= -2
        const int32_t a = qb & ~3;
        const u32x2_a4 m = *reinterpret_cast<const u32x2_a4*>(L.rmark + a);
        uint32_t z[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const uint32_t x = m[j] ^ ee;
          z[j] = ~(((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x | 0x7f7f7f7fu);
        }
        acc |= ((uint64_t)z[1] << 32 | z[0]) >> (8 * (qb - a));
      }
    }
    todo = (acc & km) != 0;
  }
  return __ballot(todo);
}

template <int MODE, bool FILT>
// Eight waves per SIMD: the code fits in 64 VGPRs without spilling vector
// registers, and a reconstruction is bound by each wave's chain of fetches.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8)))
void k_recon(DevLevel L, const int32_t* __restrict__ plist, int32_t nP,
             const uint8_t* __restrict__ excl, float* __restrict__ out_f,
             unsigned long long* __restrict__ absdiff, int32_t skip) {
  const int32_t nwaves = gridDim.x * (kBlock / 64);
  unsigned long long my_abs = 0;
  // the wave's pixels w, w + nwaves, ... in groups of 64
  for (int32_t w0 = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); w0 < nP;
       w0 += 64 * nwaves) {
    uint64_t todo = recon_todo(L, plist, w0, nwaves, nP, skip != 0);
    while (todo) {
      const int i = __builtin_ctzll(todo);
      todo &= todo - 1;
      recon_pixel<MODE, FILT>(L, plist, w0 + i * nwaves, excl, out_f, my_abs);
    }
  }
  if (absdiff) add_spread(absdiff, (threadIdx.x & 63) == 0 ? my_abs : 0ull);
}


// ------------------------------------------------------------------------
// Batched, persistent launches: one launch covers the chunks of every job
// (clip) in the batch.  A job's chunks are consecutive in the flat list.
// Workgroups take chunks from a shared counter in increasing order (chunks
// of different jobs and levels cost very different amounts, so a static
// split would leave the launch waiting for its slowest workgroup) and run
// exactly the per-target / per-pixel code of the single-clip kernels, so a
// clip's results do not depend on the batch it runs in or on which
// workgroup takes which chunk.  Chunk counts are read from device memory, so
// a captured graph of these launches stays valid when jobs come and go.
// ------------------------------------------------------------------------
// Chunk scheduler.  Direct launches (grid = number of chunks) map workgroup
// b to chunk xcd_block(b), like the single-clip kernels.  Persistent
// launches (a fixed grid, as captured in a graph) take chunks from one
// counter per launch in increasing order: chunks of different jobs and
// levels cost very different amounts, so a static split would leave the
// launch waiting for its slowest workgroup.
struct ChunkCursor {
  int32_t c;
  bool first;
};

__device__ __forceinline__ bool next_chunk(int32_t* counter, int32_t n, bool direct,
                                           ChunkCursor& cur, int32_t* s_c) {
  if (direct) {
    // block b takes chunks xcd_block(b) + k * grid: every chunk is covered
    // whatever the grid (one chunk per workgroup when grid = n)
    cur.c = cur.first ? xcd_block(blockIdx.x, gridDim.x) : cur.c + (int32_t)gridDim.x;
    cur.first = false;
    return cur.c < n;
  }
  __syncthreads();  // every thread has read the previous chunk index
  if (threadIdx.x == 0) *s_c = atomicAdd(counter, 1);
  __syncthreads();
  // the same value in every lane: scalar registers address the job
  cur.c = __builtin_amdgcn_readfirstlane(*s_c);
  return cur.c < n;
}

#define FOR_EACH_CHUNK(counter, n, direct, c)                   \
  __shared__ int32_t s_cur_;                                    \
  ChunkCursor cur_{0, true};                                    \
  for (int32_t c = 0; next_chunk(counter, n, direct, cur_, &s_cur_) && ((c = cur_.c), true);)

__global__ void kb_zero(BatchArgs B) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < B.counts[2] * kCntSlots)
    B.jobs[j / kCntSlots].absdiff[(j % kCntSlots) * kCntStride] = 0;
  if (j < kQueueSlots) B.queue[j] = 0;
}

__global__ void kb_sum_abs(BatchArgs B, unsigned long long* out) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= B.counts[2]) return;
  const unsigned long long* a = B.jobs[j].absdiff;
  unsigned long long s = 0;
  for (int k = 0; k < kCntSlots; ++k) s += a[k * kCntStride];
  out[j] = s;
}

__global__ void k_sum_spread(const unsigned long long* base, int32_t n, unsigned long long* out) {
  const int32_t i = blockIdx.x;
  if (i >= n) return;
  const int lane = threadIdx.x;  // one wave per counter, one slot per lane
  unsigned long long v = base[(size_t)i * kCntWords + lane * kCntStride];
  v = wave_sum_u64(v);
  if (lane == 0) out[i] = v;
}

// A field of the job descriptor, read word by word into scalar registers:
// the job index is the same in every lane, but the compiler cannot prove that
// the table is not written during the kernel and would otherwise keep the
// descriptor in vector registers.
template <typename T>
__device__ __forceinline__ T uniform(const T& src) {
  static_assert(sizeof(T) % 4 == 0, "word-sized fields");
  uint32_t w[sizeof(T) / 4];
  __builtin_memcpy(w, &src, sizeof(T));
#pragma unroll
  for (size_t i = 0; i < sizeof(T) / 4; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  T out;
  __builtin_memcpy(&out, w, sizeof(T));
  return out;
}

template <int BLK, bool MASKED>
__global__ __launch_bounds__(BLK) void kb_s0(BatchArgs B, int32_t slot) {
  const int32_t n = B.counts[0];
  FOR_EACH_CHUNK(B.queue + slot, n, B.direct, c) {
    const JobDesc& J = B.jobs[__builtin_amdgcn_readfirstlane(B.tchunk_job[c])];
    const DevLevel L = uniform(J.L);
    PassArgs A{};
    A.tlist = uniform(J.tlist);
    A.nS = uniform(J.nS);
    A.excl = uniform(J.excl);
    A.nin = L.nnf0;
    A.step = uniform(J.step);
    const int ne = s0_target<MASKED>(L, A, (c - uniform(J.tchunk0)) * BLK + (int32_t)threadIdx.x);
    count_evals(uniform(J.evals_init), ne);
  }
}

// one chunk of a batched pass (every thread of the workgroup calls it)
template <int BLK, bool MASKED, bool GQ>
__device__ __forceinline__ void kb_pass_chunk(const BatchArgs& B, PassShared<BLK>& sh, int32_t c,
                                              int32_t s, int32_t k, int32_t parity, int32_t t,
                                              int32_t since) {
  const JobDesc& J = B.jobs[__builtin_amdgcn_readfirstlane(B.tchunk_job[c])];
  const DevLevel L = uniform(J.L);
  PassArgs A{};
  A.tlist = uniform(J.tlist);
  A.nS = uniform(J.nS);
  A.smask = MASKED ? uniform(J.smask) : L.htil;
  A.excl = uniform(J.excl);
  A.nin = parity ? L.nnf1 : L.nnf0;
  A.nout = parity ? L.nnf0 : L.nnf1;
  A.s = s;
  A.R = uniform(J.R[k]);
  A.rs_k = (k > 0 && A.R >= 1) ? k : 0;
  A.t = t;
  A.since = since;
  A.step = uniform(J.step);
  const int ne = pass_block<BLK, MASKED, false, GQ>(L, A, c - uniform(J.tchunk0), sh);
  count_evals(uniform(J.evals), ne);
}

// PERSIST: workgroups take chunks from the launch's counter.  Otherwise
// (direct launches, grid = the chunk count) workgroup b takes chunk
// xcd_block(b) and nothing else: without a loop around the pass the kernel
// keeps the register count, and so the occupancy, of the single-clip pass.
// GQ: the passes without random search (k = 0), short queues evaluated by
// lane groups, as the single-clip pass does
template <int BLK, bool MASKED, bool PERSIST, bool GQ>
__global__ __launch_bounds__(BLK) void kb_pass(BatchArgs B, int32_t s, int32_t k, int32_t parity,
                                               int32_t slot, int32_t t, int32_t since) {
  __shared__ PassShared<BLK> sh;
  const int32_t n = B.counts[0];
  if (PERSIST) {
    FOR_EACH_CHUNK(B.queue + slot, n, false, c)
        kb_pass_chunk<BLK, MASKED, GQ>(B, sh, c, s, k, parity, t, since);
  } else {
    const int32_t c = xcd_block(blockIdx.x, gridDim.x);
    if (c < n) kb_pass_chunk<BLK, MASKED, GQ>(B, sh, c, s, k, parity, t, since);
  }
}

template <int BLK>
__global__ __launch_bounds__(BLK) void kb_copy(BatchArgs B, int32_t slot) {
  const int32_t n = B.counts[0];
  FOR_EACH_CHUNK(B.queue + slot, n, B.direct, c) {
    const JobDesc& J = B.jobs[__builtin_amdgcn_readfirstlane(B.tchunk_job[c])];
    const DevLevel L = uniform(J.L);
    const int32_t* tlist = uniform(J.tlist);
    const int32_t i = (c - uniform(J.tchunk0)) * BLK + (int32_t)threadIdx.x;
    if (i < uniform(J.nS)) L.nnf0[tlist[i]] = L.nnf1[tlist[i]];
  }
}

template <bool FILT>
// eight waves per SIMD, as k_recon
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8)))
void kb_recon(BatchArgs B, int32_t slot) {
  constexpr int kWaves = kBlock / 64;
  const int32_t n = B.counts[1];
  FOR_EACH_CHUNK(B.queue + slot, n, B.direct, c) {
    const JobDesc& J = B.jobs[__builtin_amdgcn_readfirstlane(B.pchunk_job[c])];
    const DevLevel L = uniform(J.L);
    const int32_t* hlist = uniform(J.hlist);
    const uint8_t* excl = uniform(J.excl);
    const int32_t base = (c - uniform(J.pchunk0)) * kPixChunk;
    const int32_t end = min(uniform(J.nH), base + kPixChunk);
    const int32_t mode = uniform(J.recon_mode);
    const bool skip = !FILT && uniform(J.recon_skip) != 0;
    unsigned long long my_abs = 0;
    // kPixChunk / kWaves (<= 64) pixels per wave
    const int32_t w0 = base + (int32_t)(threadIdx.x >> 6);
    uint64_t todo = recon_todo(L, hlist, w0, kWaves, end, skip);
    while (todo) {
      const int i = __builtin_ctzll(todo);
      todo &= todo - 1;
      if (mode == 1)
        recon_pixel<1, FILT>(L, hlist, w0 + i * kWaves, excl, nullptr, my_abs);
      else
        recon_pixel<0, FILT>(L, hlist, w0 + i * kWaves, excl, nullptr, my_abs);
    }
    add_spread(uniform(J.absdiff), (threadIdx.x & 63) == 0 ? my_abs : 0ull);
  }
}

// ------------------------------------------------------------------------
// Level transition (Sec. 3.6): fine target p takes its parent's shift with
// the spatial components doubled and the parent's distance and count.
// ------------------------------------------------------------------------
__global__ void k_upsample(DevLevel F, DevLevel C, const int32_t* __restrict__ ftlist,
                           int32_t nS) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nS) return;
  const int32_t p = ftlist[i];
  int32_t x, y, t;
  unlin(F, p, x, y, t);
  // with temporal subsampling (the coarser level holds fewer frames) the
  // parent and the doubled shift cover time as well
  const bool ts = C.T != F.T;
  const int32_t Pt = ts ? t >> 1 : t;
  const int32_t P = (Pt * C.H + (y >> 1)) * C.W + (x >> 1);
  const int2 pc = C.nnf0[P];
  int32_t cx, cy, ct;
  unlin(C, pc.x, cx, cy, ct);
  const int32_t fx = x + 2 * (cx - (x >> 1));
  const int32_t fy = y + 2 * (cy - (y >> 1));
  const int32_t ft = ts ? t + 2 * (ct - Pt) : ct;
  F.nnf0[p] = make_int2((ft * F.H + fy) * F.W + fx, pc.y);
  F.nvox[p] = C.nvox[P];
}

// ------------------------------------------------------------------------
// Pyramids and texture features.
// ------------------------------------------------------------------------
__global__ void k_init_level0(const uint8_t* __restrict__ rgb, const uint8_t* __restrict__ mask,
                              DevLevel L) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.V) return;
  const bool h = mask[i] != 0;
  L.hole[i] = h ? 1 : 0;
  uint32_t x = 0;
  if (!h) x = (uint32_t)rgb[3 * (size_t)i] | ((uint32_t)rgb[3 * (size_t)i + 1] << 8) |
              ((uint32_t)rgb[3 * (size_t)i + 2] << 16);
  L.vox[i] = make_uint2(x, 0);
}

// 2x2 spatial box mean rounded half up (no temporal subsampling), OR-pooled hole
__global__ void k_pyr_down(DevLevel F, DevLevel C) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= C.V) return;
  int32_t x, y, t;
  unlin(C, i, x, y, t);
  int any = 0, cnt = 0;
  uint32_t sr = 0, sg = 0, sb = 0;
  // 2x2 blocks, or 2x2x2 when the coarser level holds fewer frames
  const int nbt = C.T != F.T ? 2 : 1;
  for (int bt = 0; bt < nbt; ++bt)
    for (int by = 0; by < 2; ++by)
      for (int bx = 0; bx < 2; ++bx) {
        const int32_t fx = 2 * x + bx, fy = 2 * y + by, ft = nbt == 2 ? 2 * t + bt : t;
        if (fx >= F.W || fy >= F.H || ft >= F.T) continue;
        const int32_t j = (ft * F.H + fy) * F.W + fx;
        any |= F.hole[j];
        ++cnt;
        const uint32_t v = F.vox[j].x;
        sr += v & 255;
        sg += (v >> 8) & 255;
        sb += (v >> 16) & 255;
      }
  C.hole[i] = (uint8_t)any;
  uint32_t out = 0;
  if (!any) {
    const uint32_t h = (uint32_t)cnt / 2;
    out = ((sr + h) / cnt) | (((sg + h) / cnt) << 8) | (((sb + h) / cnt) << 16);
  }
  C.vox[i] = make_uint2(out, 0);
}

// |grey(x+1) - grey(x-1)| (times 3) over known pixels, packed:
// bits 0-9 gx, bit 10 gx defined, bits 11-20 gy, bit 21 gy defined
__global__ void k_grad(const uint8_t* __restrict__ rgb, DevLevel L, uint32_t* __restrict__ gpk) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.V) return;
  int32_t x, y, t;
  unlin(L, i, x, y, t);
  auto g = [&](int32_t j) -> int {
    return (int)rgb[3 * (size_t)j] + (int)rgb[3 * (size_t)j + 1] + (int)rgb[3 * (size_t)j + 2];
  };
  uint32_t out = 0;
  if (x >= 1 && x + 1 < L.W && !L.hole[i - 1] && !L.hole[i + 1]) {
    const int d = g(i + 1) - g(i - 1);
    out |= (uint32_t)(d < 0 ? -d : d) | (1u << 10);
  }
  if (y >= 1 && y + 1 < L.H && !L.hole[i - L.W] && !L.hole[i + L.W]) {
    const int d = g(i + L.W) - g(i - L.W);
    out |= ((uint32_t)(d < 0 ? -d : d) << 11) | (1u << 21);
  }
  gpk[i] = out;
}

// sums over [x, x+s) of the defined derivatives: .x = gx sum | count << 20.
// A workgroup takes kBlock consecutive x of one row (y, t) and stages the
// row's entries [x0, x0 + kBlock + s - 1) in LDS (entries past the row read
// 0: no defined derivative), so each entry is fetched once instead of s
// times.  s <= kMaxBox (2^(levels - 1), levels <= 8).
constexpr int32_t kMaxBox = 128;
__global__ __launch_bounds__(kBlock) void k_box_h(const uint32_t* __restrict__ gpk, DevLevel L,
                                                  int32_t s, uint2* __restrict__ hsum) {
  __shared__ uint32_t seg[kBlock + kMaxBox];
  const int32_t nseg = (L.W + kBlock - 1) / kBlock;
  const int32_t row = blockIdx.x / nseg, x0 = (blockIdx.x % nseg) * kBlock;
  const uint32_t* __restrict__ src = gpk + (size_t)row * L.W;
  for (int32_t k = threadIdx.x; k < kBlock + s - 1; k += kBlock)
    seg[k] = x0 + k < L.W ? src[x0 + k] : 0u;
  __syncthreads();
  const int32_t x = x0 + (int32_t)threadIdx.x;
  if (x >= L.W) return;
  uint32_t sx = 0, cx = 0, sy = 0, cy = 0;
  for (int32_t k = 0; k < s; ++k) {
    const uint32_t g = seg[threadIdx.x + k];
    if (g & (1u << 10)) {
      sx += g & 1023u;
      ++cx;
    }
    if (g & (1u << 21)) {
      sy += (g >> 11) & 1023u;
      ++cy;
    }
  }
  hsum[(size_t)row * L.W + x] = make_uint2(sx | (cx << 20), sy | (cy << 20));
}

// texture of level l: T(2^l X, 2^l Y, t) of the finest level (or 2^l t as
// well when the pyramid subsamples time), rounded half up mean of |grey
// difference| = S / (3c) over the sums of the finest level's rows
// [2^l Y, min(H, 2^l Y + s)) at column 2^l X; zero inside the level's hole.
// A thread takes kTexRun consecutive rows Y of one column (X, t) and slides
// the window: consecutive windows are 2^l rows apart, so while 2^l < s it
// drops 2^l rows and adds 2^l (4 loads per output at level 1 instead of s =
// 16), and from 2^l >= s on it sums each window afresh.  Thread order: X
// fastest.  The sums stay below 2^25 (s <= 128 rows of at most 128 x 1023),
// so 32-bit arithmetic is exact.
constexpr int32_t kTexRun = 32;

struct TexSums {
  uint32_t sx = 0, cx = 0, sy = 0, cy = 0;
  __device__ __forceinline__ void add(uint2 h) {
    sx += h.x & 0xFFFFFu;
    cx += h.x >> 20;
    sy += h.y & 0xFFFFFu;
    cy += h.y >> 20;
  }
  __device__ __forceinline__ void sub(uint2 h) {
    sx -= h.x & 0xFFFFFu;
    cx -= h.x >> 20;
    sy -= h.y & 0xFFFFFu;
    cy -= h.y >> 20;
  }
};

__global__ void k_tex_level(const uint2* __restrict__ hsum, DevLevel L0, DevLevel Ll, int32_t l,
                            int32_t s) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int32_t runs = (Ll.H + kTexRun - 1) / kTexRun;
  const int32_t X = (int32_t)(gid % Ll.W);
  const int64_t rt = gid / Ll.W;
  const int32_t run = (int32_t)(rt % runs), tl = (int32_t)(rt / runs);
  if (tl >= Ll.T) return;
  const int32_t H0 = L0.H, step = 1 << l;
  const int32_t t = Ll.T != L0.T ? tl << l : tl;
  const uint2* __restrict__ col = hsum + (size_t)t * H0 * L0.W + ((size_t)X << l);
  const int32_t Y0 = run * kTexRun, Y1 = min(Ll.H, Y0 + kTexRun);
  TexSums w;
  for (int32_t yy = Y0 * step; yy < min(H0, Y0 * step + s); ++yy) w.add(col[(size_t)yy * L0.W]);
  for (int32_t Y = Y0; Y < Y1; ++Y) {
    const int32_t i = (tl * Ll.H + Y) * Ll.W + X;
    uint32_t tx = 0, ty = 0;
    if (!Ll.hole[i]) {
      tx = w.cx ? (2 * w.sx + 3 * w.cx) / (6 * w.cx) : 0;
      ty = w.cy ? (2 * w.sy + 3 * w.cy) / (6 * w.cy) : 0;
    }
    Ll.vox[i].y = tx | (ty << 8);
    if (Y + 1 == Y1) break;
    // the window of Y + 1: [y + step, min(H0, y + step + s))
    const int32_t y = Y * step;
    if (step < s) {
      for (int32_t yy = y; yy < y + step; ++yy)
        if (yy < H0) w.sub(col[(size_t)yy * L0.W]);
      for (int32_t yy = y + s; yy < y + s + step; ++yy)
        if (yy < H0) w.add(col[(size_t)yy * L0.W]);
    } else {
      w = TexSums();
      for (int32_t yy = y + step; yy < min(H0, y + step + s); ++yy)
        w.add(col[(size_t)yy * L0.W]);
    }
  }
}

// ------------------------------------------------------------------------
// Morphology.
// ------------------------------------------------------------------------
// 1-D OR over [-2, 2] along an axis (stride, coordinate extent)
__global__ void k_dil_axis(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, int32_t W,
                           int32_t H, int32_t T, int axis, const uint8_t* __restrict__ and_not) {
  const int32_t V = W * H * T;
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= V) return;
  const int32_t x = i % W, y = (i / W) % H, t = i / (W * H);
  const int32_t c = axis == 0 ? x : (axis == 1 ? y : t);
  const int32_t dim = axis == 0 ? W : (axis == 1 ? H : T);
  const int32_t stride = axis == 0 ? 1 : (axis == 1 ? W : W * H);
  uint8_t r = 0;
  for (int d = -2; d <= 2; ++d) {
    const int32_t cc = c + d;
    if (cc < 0 || cc >= dim) continue;
    r |= src[i + d * stride];
  }
  if (and_not) r = (uint8_t)(r && !and_not[i]);
  dst[i] = r ? 1 : 0;
}

// D~: patch inside the volume and no hole voxel in it
__global__ void k_sources(DevLevel L) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.V) return;
  int32_t x, y, t;
  unlin(L, i, x, y, t);
  const bool inner =
      x >= 2 && y >= 2 && t >= L.ht && x < L.W - 2 && y < L.H - 2 && t < L.T - L.ht;
  L.dsrc[i] = (uint8_t)(inner && !L.htil[i]);
}

// E = H' minus voxels with an in-volume 3x3x3 neighbour outside H'
// (outside the volume counts as occluded); bd = H' \ E.
__global__ void k_erode3(const uint8_t* __restrict__ Hp, uint8_t* __restrict__ E,
                         uint8_t* __restrict__ bd, int32_t W, int32_t H, int32_t T) {
  const int32_t V = W * H * T;
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= V) return;
  const int32_t x = i % W, y = (i / W) % H, t = i / (W * H);
  uint8_t e = 0;
  if (Hp[i]) {
    e = 1;
    for (int dt = -1; dt <= 1; ++dt)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int32_t xx = x + dx, yy = y + dy, tt = t + dt;
          if (xx < 0 || yy < 0 || tt < 0 || xx >= W || yy >= H || tt >= T) continue;
          if (!Hp[(tt * H + yy) * W + xx]) e = 0;
        }
  }
  E[i] = e;
  bd[i] = (uint8_t)(Hp[i] && !e);
}

// ------------------------------------------------------------------------
// State transfer and fills.
// ------------------------------------------------------------------------
__global__ void k_fill_nnf(int2* nnf, uint8_t* nvox, int32_t V) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= V) return;
  nnf[i] = make_int2(-1, -1);
  if (nvox) nvox[i] = 0;
}

__global__ void k_fill_u64(unsigned long long* p, int32_t n) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ void k_get_state(DevLevel L, uint8_t* rgbt, int32_t* cand, int32_t* dist,
                            uint8_t* nvox) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.V) return;
  if (rgbt) {
    const uint2 v = L.vox[i];
    uint8_t* o = rgbt + 5 * (size_t)i;
    o[0] = v.x & 255;
    o[1] = (v.x >> 8) & 255;
    o[2] = (v.x >> 16) & 255;
    o[3] = v.y & 255;
    o[4] = (v.y >> 8) & 255;
  }
  const bool tg = L.htil[i] != 0;
  const int2 nn = L.nnf0[i];
  if (cand) cand[i] = tg ? nn.x : -1;
  if (dist) dist[i] = tg ? nn.y : -1;
  if (nvox) nvox[i] = tg ? L.nvox[i] : 0;
}

// bad[0]: cand outside [-1, V); bad[1]: target without a source match or
// with a zero voxel count
// write = 0 only counts the entries vi_set_state rejects (bad[0]: a match
// outside [-1, V)) and those that leave the map incomplete (bad[1]); write = 1
// also stores the state.  The host validates before writing, so a rejected
// call leaves the level as it was.
__global__ void k_set_state(DevLevel L, const uint8_t* rgbt, const int32_t* cand,
                            const int32_t* dist, const uint8_t* nvox, unsigned long long* bad,
                            int write) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  int b0 = 0, b1 = 0;
  if (i < L.V && !write) {
    const bool tg = L.htil[i] != 0;
    if (cand) {
      const int32_t c = cand[i];
      if (c < -1 || c >= L.V) b0 = 1;
      else if (tg && (c < 0 || !L.dsrc[c])) b1 = 1;
    }
    if (nvox && tg && nvox[i] == 0) b1 = 1;
  } else if (i < L.V) {
    if (rgbt && L.hole[i]) {
      const uint8_t* s = rgbt + 5 * (size_t)i;
      L.vox[i] = make_uint2((uint32_t)s[0] | ((uint32_t)s[1] << 8) | ((uint32_t)s[2] << 16),
                            (uint32_t)s[3] | ((uint32_t)s[4] << 8));
    }
    const bool tg = L.htil[i] != 0;
    int2 nn = L.nnf0[i];
    if (cand) nn.x = tg ? cand[i] : -1;
    if (dist) nn.y = tg ? dist[i] : -1;
    L.nnf0[i] = nn;
    if (nvox) L.nvox[i] = tg ? nvox[i] : 0;
  }
  unsigned long long s0 = wave_sum_u64((unsigned long long)b0);
  unsigned long long s1 = wave_sum_u64((unsigned long long)b1);
  if ((threadIdx.x & 63) == 0) {
    if (s0) atomicAdd(&bad[0], s0);
    if (s1) atomicAdd(&bad[1], s1);
  }
}

__global__ void k_out_rgb(DevLevel L, uint8_t* out) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.V) return;
  const uint32_t v = L.vox[i].x;
  out[3 * (size_t)i] = v & 255;
  out[3 * (size_t)i + 1] = (v >> 8) & 255;
  out[3 * (size_t)i + 2] = (v >> 16) & 255;
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------

static inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

void launch_init_level0(hipStream_t st, const uint8_t* rgb, const uint8_t* mask, DevLevel L0) {
  k_init_level0<<<grid_for(L0.V), kBlock, 0, st>>>(rgb, mask, L0);
}

void launch_pyr_down(hipStream_t st, DevLevel F, DevLevel C) {
  k_pyr_down<<<grid_for(C.V), kBlock, 0, st>>>(F, C);
}

void launch_texture(hipStream_t st, const uint8_t* rgb, DevLevel L0, int32_t s, uint32_t* gpk,
                    uint2* hsum) {
  k_grad<<<grid_for(L0.V), kBlock, 0, st>>>(rgb, L0, gpk);
  const int64_t nseg = (L0.W + kBlock - 1) / kBlock;
  k_box_h<<<(unsigned)(nseg * L0.H * L0.T), kBlock, 0, st>>>(gpk, L0, s, hsum);
}

void launch_texture_level(hipStream_t st, const uint2* hsum, DevLevel L0, DevLevel Ll, int32_t l,
                          int32_t s) {
  const int64_t n = (int64_t)Ll.W * ((Ll.H + kTexRun - 1) / kTexRun) * Ll.T;
  k_tex_level<<<grid_for(n), kBlock, 0, st>>>(hsum, L0, Ll, l, s);
}

void launch_dilate5(hipStream_t st, const uint8_t* src, uint8_t* dst, uint8_t* tmp1,
                    uint8_t* tmp2, int32_t W, int32_t H, int32_t T, const uint8_t* and_not) {
  const int64_t V = (int64_t)W * H * T;
  k_dil_axis<<<grid_for(V), kBlock, 0, st>>>(src, tmp1, W, H, T, 0, nullptr);
  k_dil_axis<<<grid_for(V), kBlock, 0, st>>>(tmp1, tmp2, W, H, T, 1, nullptr);
  k_dil_axis<<<grid_for(V), kBlock, 0, st>>>(tmp2, dst, W, H, T, 2, and_not);
}

void launch_sources(hipStream_t st, DevLevel L) { k_sources<<<grid_for(L.V), kBlock, 0, st>>>(L); }


void launch_fill_nnf(hipStream_t st, int2* nnf, uint8_t* nvox, int32_t V) {
  k_fill_nnf<<<grid_for(V), kBlock, 0, st>>>(nnf, nvox, V);
}

void launch_fill_u64(hipStream_t st, unsigned long long* p, int32_t n) {
  k_fill_u64<<<grid_for(n), kBlock, 0, st>>>(p, n);
}

void launch_s0(hipStream_t st, DevLevel L, const PassArgs& A, bool red, int32_t wide_max) {
  if (A.nS <= 0) return;
  const bool wide = !red && A.nS <= (wide_max < 0 ? kWideS0MaxTargets : wide_max);
  const unsigned wide_grid = (unsigned)((A.nS + kWideTargets - 1) / kWideTargets);
  if (wide && A.excl)
    k_s0_wide<true><<<wide_grid, kBlock, 0, st>>>(L, A);
  else if (wide)
    k_s0_wide<false><<<wide_grid, kBlock, 0, st>>>(L, A);
  else if (A.excl)
    k_s0<true, false><<<grid_for(A.nS), kBlock, 0, st>>>(L, A);
  else if (red)
    k_s0<false, true><<<grid_for(A.nS), kBlock, 0, st>>>(L, A);
  else
    k_s0<false, false><<<grid_for(A.nS), kBlock, 0, st>>>(L, A);
}

bool pass_is_wide(int32_t nS, bool red, int32_t wide_max) {
  return !red && nS <= (wide_max < 0 ? kWideMaxTargets : wide_max);
}

void launch_pass(hipStream_t st, DevLevel L, const PassArgs& A, bool red, int32_t wide_max) {
  if (A.nS <= 0) return;
  const unsigned wide_grid = (unsigned)((A.nS + kWideTargets - 1) / kWideTargets);
  if (A.excl && pass_is_wide(A.nS, false, wide_max))
    k_pass_wide<kWideTargets, true><<<wide_grid, kBlock, 0, st>>>(L, A);
  else if (A.excl)
    k_pass<true, false, false><<<grid_for(A.nS), kBlock, 0, st>>>(L, A);
  else if (red)
    k_pass<false, true, false><<<grid_for(A.nS), kBlock, 0, st>>>(L, A);
  else if (pass_is_wide(A.nS, false, wide_max))
    k_pass_wide<kWideTargets, false><<<wide_grid, kBlock, 0, st>>>(L, A);
  else if (A.rs_k == 0)
    k_pass<false, false, true><<<grid_for(A.nS), kBlock, 0, st>>>(L, A);
  else
    k_pass<false, false, false><<<grid_for(A.nS), kBlock, 0, st>>>(L, A);
}

void launch_rerank(hipStream_t st, DevLevel L, const int32_t* tlist, int32_t nS) {
  if (nS <= 0) return;
  k_rerank<<<grid_for(nS), kBlock, 0, st>>>(L, tlist, nS);
}

void launch_copy_targets(hipStream_t st, const int32_t* tlist, int32_t nS, const int2* src,
                         int2* dst) {
  if (nS <= 0) return;
  k_copy_targets<<<grid_for(nS), kBlock, 0, st>>>(tlist, nS, src, dst);
}

void launch_recon(hipStream_t st, DevLevel L, const int32_t* plist, int32_t nP,
                  const uint8_t* filt_excl, int mode, float* out_f, unsigned long long* absdiff,
                  bool skip) {
  if (nP <= 0) return;
  const int wpb = kBlock / 64;
  int64_t blocks = (nP + wpb - 1) / wpb;
  if (blocks > 8192) blocks = 8192;
  const dim3 g((unsigned)blocks);
  // only unmasked weighted or plain means may keep unchanged pixels
  const int32_t sk = skip && !filt_excl && mode != 2 ? 1 : 0;
  if (filt_excl) {
    if (mode == 0)
      k_recon<0, true><<<g, kBlock, 0, st>>>(L, plist, nP, filt_excl, out_f, absdiff, 0);
    else if (mode == 1)
      k_recon<1, true><<<g, kBlock, 0, st>>>(L, plist, nP, filt_excl, out_f, absdiff, 0);
    else
      k_recon<2, true><<<g, kBlock, 0, st>>>(L, plist, nP, filt_excl, out_f, absdiff, 0);
  } else {
    if (mode == 0)
      k_recon<0, false><<<g, kBlock, 0, st>>>(L, plist, nP, nullptr, out_f, absdiff, sk);
    else if (mode == 1)
      k_recon<1, false><<<g, kBlock, 0, st>>>(L, plist, nP, nullptr, out_f, absdiff, sk);
    else
      k_recon<2, false><<<g, kBlock, 0, st>>>(L, plist, nP, nullptr, out_f, absdiff, 0);
  }
}

void launch_upsample(hipStream_t st, DevLevel F, DevLevel C, const int32_t* ftlist, int32_t nS) {
  if (nS <= 0) return;
  k_upsample<<<grid_for(nS), kBlock, 0, st>>>(F, C, ftlist, nS);
}

void launch_erode3(hipStream_t st, const uint8_t* Hp, uint8_t* E, uint8_t* bd, int32_t W,
                   int32_t H, int32_t T) {
  k_erode3<<<grid_for((int64_t)W * H * T), kBlock, 0, st>>>(Hp, E, bd, W, H, T);
}

void launch_get_state(hipStream_t st, DevLevel L, uint8_t* rgbt, int32_t* cand, int32_t* dist,
                      uint8_t* nvox) {
  k_get_state<<<grid_for(L.V), kBlock, 0, st>>>(L, rgbt, cand, dist, nvox);
}

void launch_set_state(hipStream_t st, DevLevel L, const uint8_t* rgbt, const int32_t* cand,
                      const int32_t* dist, const uint8_t* nvox, unsigned long long* bad,
                      int write) {
  k_set_state<<<grid_for(L.V), kBlock, 0, st>>>(L, rgbt, cand, dist, nvox, bad, write);
}

void launch_out_rgb(hipStream_t st, DevLevel L0, uint8_t* out) {
  k_out_rgb<<<grid_for(L0.V), kBlock, 0, st>>>(L0, out);
}

// Stable stream compaction: out[k] = i for the k-th i with flags[i] != 0,
// *d_count = their number.  Three launches over tiles of kCmpTile flags
// (16 per thread, one 16-byte load): per-tile counts, one workgroup's
// exclusive scan of the tile counts, then every tile writes its indices in
// order from its offset (a wave prefix of the per-thread counts by
// shuffles, the waves' totals through LDS).
constexpr int kCmpPer = 16;
constexpr int kCmpTile = kBlock * kCmpPer;

__device__ __forceinline__ uint32_t flags16(const uint8_t* __restrict__ flags, int32_t n,
                                            int64_t i0, uint32_t bits[1]) {
  // bit k of the result: flag i0 + k is set
  uint32_t m = 0;
  if (i0 + kCmpPer <= n) {
    const uint4 v = *reinterpret_cast<const uint4*>(flags + i0);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if ((w[q] >> (8 * b)) & 255u) m |= 1u << (4 * q + b);
  } else {
    for (int k = 0; k < kCmpPer; ++k)
      if (i0 + k < n && flags[i0 + k]) m |= 1u << k;
  }
  bits[0] = m;
  return (uint32_t)__popc(m);
}

__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* wsum, uint32_t* total) {
  // inclusive prefix within the wave
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    before += k < w ? wsum[k] : 0u;
    all += wsum[k];
  }
  *total = all;
  return before + x - v;
}

__global__ __launch_bounds__(kBlock) void k_cmp_count(const uint8_t* __restrict__ flags, int32_t n,
                                                      uint32_t* __restrict__ tile_count) {
  __shared__ uint32_t wsum[kBlock / 64];
  uint32_t bits[1];
  const int64_t i0 = (int64_t)blockIdx.x * kCmpTile + (int64_t)threadIdx.x * kCmpPer;
  const uint32_t c = flags16(flags, n, i0, bits);
  uint32_t total;
  (void)block_exclusive(c, wsum, &total);
  if (threadIdx.x == 0) tile_count[blockIdx.x] = total;
}

// one workgroup: tile_off[t] = sum of tile_count[0..t), *d_count = the total
__global__ __launch_bounds__(1024) void k_cmp_scan(const uint32_t* __restrict__ tile_count,
                                                   int32_t nt, uint32_t* __restrict__ tile_off,
                                                   int32_t* d_count) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  const int32_t per = (nt + 1023) / 1024;
  const int32_t a = t * per, b = min(nt, a + per);
  uint32_t s = 0;
  for (int32_t k = a; k < b; ++k) s += tile_count[k];
  part[t] = s;
  __syncthreads();
  // exclusive scan of the 1024 partial sums (Hillis-Steele in LDS)
  for (int o = 1; o < 1024; o <<= 1) {
    const uint32_t y = t >= o ? part[t - o] : 0u;
    __syncthreads();
    part[t] += y;
    __syncthreads();
  }
  uint32_t off = part[t] - s;
  for (int32_t k = a; k < b; ++k) {
    tile_off[k] = off;
    off += tile_count[k];
  }
  if (t == 1023) *d_count = (int32_t)part[1023];
}

__global__ __launch_bounds__(kBlock) void k_cmp_write(const uint8_t* __restrict__ flags, int32_t n,
                                                      const uint32_t* __restrict__ tile_off,
                                                      int32_t* __restrict__ out) {
  __shared__ uint32_t wsum[kBlock / 64];
  uint32_t bits[1];
  const int64_t i0 = (int64_t)blockIdx.x * kCmpTile + (int64_t)threadIdx.x * kCmpPer;
  const uint32_t c = flags16(flags, n, i0, bits);
  uint32_t total;
  uint32_t pos = tile_off[blockIdx.x] + block_exclusive(c, wsum, &total);
  for (uint32_t m = bits[0]; m != 0; m &= m - 1) out[pos++] = (int32_t)(i0 + __ffs(m) - 1);
}

size_t compact_temp_bytes(int32_t n) {
  const size_t nt = ((size_t)(n > 0 ? n : 1) + kCmpTile - 1) / kCmpTile;
  return 2 * sizeof(uint32_t) * nt + 256;
}

hipError_t compact(hipStream_t st, const uint8_t* flags, int32_t n, int32_t* out, int32_t* d_count,
                   void* temp, size_t temp_bytes) {
  const int32_t nt = (int32_t)(((size_t)(n > 0 ? n : 1) + kCmpTile - 1) / kCmpTile);
  if (temp_bytes < compact_temp_bytes(n)) return hipErrorInvalidValue;
  uint32_t* tile_count = static_cast<uint32_t*>(temp);
  uint32_t* tile_off = tile_count + nt;
  k_cmp_count<<<nt, kBlock, 0, st>>>(flags, n, tile_count);
  k_cmp_scan<<<1, 1024, 0, st>>>(tile_count, nt, tile_off, d_count);
  k_cmp_write<<<nt, kBlock, 0, st>>>(flags, n, tile_off, out);
  return hipGetLastError();
}

}  // namespace vi

namespace vi {

void launch_batch_zero(hipStream_t st, const BatchArgs& B, int32_t max_jobs) {
  const int32_t nz = max_jobs * kCntSlots;
  const int32_t n = nz > kQueueSlots ? nz : kQueueSlots;
  kb_zero<<<dim3((unsigned)((n + 255) / 256)), 256, 0, st>>>(B);
}

void launch_batch_sum_abs(hipStream_t st, const BatchArgs& B, int32_t max_jobs,
                          unsigned long long* out) {
  const int32_t n = max_jobs > 0 ? max_jobs : 1;
  kb_sum_abs<<<dim3((unsigned)((n + 255) / 256)), 256, 0, st>>>(B, out);
}

void launch_sum_spread(hipStream_t st, const unsigned long long* base, int32_t n,
                       unsigned long long* out) {
  static_assert(kCntSlots == 64, "one lane per slot");
  if (n <= 0) return;
  k_sum_spread<<<dim3((unsigned)n), 64, 0, st>>>(base, n, out);
}

template <bool M>
static void batch_s0(hipStream_t st, const BatchArgs& B, int blk, int32_t grid, int32_t slot) {
  if (blk == 64)
    kb_s0<64, M><<<grid, 64, 0, st>>>(B, slot);
  else if (blk == 128)
    kb_s0<128, M><<<grid, 128, 0, st>>>(B, slot);
  else
    kb_s0<256, M><<<grid, 256, 0, st>>>(B, slot);
}

void launch_batch_s0(hipStream_t st, const BatchArgs& B, int blk, int32_t grid, int32_t slot,
                     bool masked) {
  if (masked)
    batch_s0<true>(st, B, blk, grid, slot);
  else
    batch_s0<false>(st, B, blk, grid, slot);
}

template <bool M, bool P>
static void batch_pass_shape(hipStream_t st, const BatchArgs& B, int blk, int32_t grid,
                             int32_t s, int32_t k, int32_t parity, int32_t slot, int32_t t,
                             int32_t since) {
  // unmasked passes without random search: the group-queue form
  constexpr bool G = !M;
  if (G && k == 0) {
    if (blk == 64)
      kb_pass<64, M, P, G><<<grid, 64, 0, st>>>(B, s, k, parity, slot, t, since);
    else if (blk == 128)
      kb_pass<128, M, P, G><<<grid, 128, 0, st>>>(B, s, k, parity, slot, t, since);
    else
      kb_pass<256, M, P, G><<<grid, 256, 0, st>>>(B, s, k, parity, slot, t, since);
  } else if (blk == 64) {
    kb_pass<64, M, P, false><<<grid, 64, 0, st>>>(B, s, k, parity, slot, t, since);
  } else if (blk == 128) {
    kb_pass<128, M, P, false><<<grid, 128, 0, st>>>(B, s, k, parity, slot, t, since);
  } else {
    kb_pass<256, M, P, false><<<grid, 256, 0, st>>>(B, s, k, parity, slot, t, since);
  }
}

template <bool M>
static void batch_pass(hipStream_t st, const BatchArgs& B, int blk, int32_t grid, int32_t s,
                       int32_t k, int32_t parity, int32_t slot, int32_t t, int32_t since) {
  if (B.direct)
    batch_pass_shape<M, false>(st, B, blk, grid, s, k, parity, slot, t, since);
  else
    batch_pass_shape<M, true>(st, B, blk, grid, s, k, parity, slot, t, since);
}

void launch_batch_pass(hipStream_t st, const BatchArgs& B, int blk, int32_t grid, int32_t s,
                       int32_t k, int32_t parity, int32_t slot, int32_t t, int32_t since,
                       bool masked) {
  if (masked)
    batch_pass<true>(st, B, blk, grid, s, k, parity, slot, t, since);
  else
    batch_pass<false>(st, B, blk, grid, s, k, parity, slot, t, since);
}

void launch_batch_copy(hipStream_t st, const BatchArgs& B, int blk, int32_t grid, int32_t slot) {
  if (blk == 64)
    kb_copy<64><<<grid, 64, 0, st>>>(B, slot);
  else if (blk == 128)
    kb_copy<128><<<grid, 128, 0, st>>>(B, slot);
  else
    kb_copy<256><<<grid, 256, 0, st>>>(B, slot);
}

void launch_batch_recon(hipStream_t st, const BatchArgs& B, int32_t grid, int32_t slot,
                        bool masked) {
  if (masked)
    kb_recon<true><<<grid, kBlock, 0, st>>>(B, slot);
  else
    kb_recon<false><<<grid, kBlock, 0, st>>>(B, slot);
}

}  // namespace vi
