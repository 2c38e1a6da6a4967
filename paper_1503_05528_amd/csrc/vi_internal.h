// vi_internal.h -- device-side data layout and kernel launchers of libvi.
//
// Per pyramid level the context keeps, in HBM:
//   vox    uint2 [V]  .x = R | G<<8 | B<<16, .y = Tx | Ty<<8 (one 8-byte load
//                     per voxel feeds two v_dot4_u32_u8 operations); two
//                     entries of padding on both sides (row loads of patches
//                     that cross the volume's first or last row)
//   hole   u8 [V]     H^l
//   dsrc   u8 [V]     D~^l (centres of hole-free, in-volume patches)
//   htil   u8 [V]     H~^l (targets of the shift map)
//   dlist  i32 [nD]   D~ in ascending linear order (uniform random init)
//   tlist  i32 [nS]   H~ in ascending linear order (one thread per target)
//   hlist  i32 [nH]   H  in ascending linear order (one wave per hole pixel)
//   nnf0/1 int2 [V]   (cand, dist) double buffer of the Jacobi passes; entries
//                     outside the current target set are never read
//   nvox   u8 [V]     number of voxels the stored distance compared
//   chg    u16 [V]    pass of the current search that last changed the match
//                     (0 after step 0; 0 outside the target set)
//   rmark  u8 [V]     reconstruction epoch at which the target's (match,
//                     distance, count) last changed; a reconstruction of
//                     epoch e may skip a hole pixel whose 125 contributors
//                     all hold marks other than e (16 zero entries of padding
//                     on both sides, for the 8-byte row loads); epochs run
//                     1..255 and wrap, so an old mark can only cause a
//                     recomputation
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "vi.h"

namespace vi {

// Division by a run-time invariant divisor (Granlund & Montgomery, "Division
// by invariant integers using multiplication", PLDI 1994): q = (mulhi(m, n) +
// n) >> l, exact for 0 <= n < 2^31 and 1 <= d < 2^31.
struct FastDiv {
  uint32_t d, m, l;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  f.l = l;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (__umulhi(n, f.m) + n) >> f.l;
}

struct DevLevel {
  int32_t W, H, T, V, WH, level;
  FastDiv fdW, fdWH;
  uint2* vox;
  uint8_t* hole;
  uint8_t* dsrc;
  uint8_t* htil;
  int32_t* dlist;
  int32_t nD;
  int2* nnf0;
  int2* nnf1;
  uint8_t* nvox;
  uint16_t* chg;
  uint8_t* rmark;
  int32_t repoch;  // epoch of the next reconstruction of the level (from 1)
  int32_t ht;      // temporal half-size of a patch: 2 (5x5x5 video patches) or 0
                   // (5x5x1 patches of single images, T = 1)
  int32_t lambda;
  uint64_t seed;
  // dimensionality-reduced patch space: rd features per voxel (a multiple of
  // four; 0 = the exact distance) in feat [V][rd]
  const int32_t* feat;
  int32_t rd;
  int2* prev;  // [V] a reduced search's targets' entries before it
};

constexpr int kPatchDimMax = 625;  // coordinates of a 5x5x5 patch vector (5 channels)
constexpr int kMaxRed = 32;        // features of the reduced patch space, at most

// One synchronous pass of the search over a target list.
struct PassArgs {
  const int32_t* tlist;
  int32_t nS;
  const uint8_t* smask;    // target-set membership (q in S)
  const uint8_t* excl;     // voxels excluded from comparisons (onion: H'), or null
  const int2* nin;         // state before the pass
  int2* nout;              // state after the pass
  int32_t s;               // propagation stride, 0 = no propagation
  int32_t rs_k;            // PatchMatch iteration of the random search, 0 = none
  int32_t R;               // random-search radius floor(r_max rho^k)
  int32_t t;               // index of the pass in the search, from 1
  int32_t since;           // previous pass at the same stride, or 0: no skipping
  uint64_t step;           // Philox counter word 1
  unsigned long long* evals;  // effective-evaluation counter (spread), or null
};

// One clip's EM iteration inside a batched launch (device memory).
constexpr int kMaxPmIters = 64;
struct JobDesc {
  DevLevel L;
  const int32_t* tlist;
  const int32_t* hlist;
  int32_t nS, nH;
  int32_t tchunk0;  // first target chunk of this job in the flat chunk list
  int32_t pchunk0;  // first pixel chunk
  int32_t recon_mode;
  int32_t recon_skip;  // the reconstruction may skip pixels with unchanged contributors
  const uint8_t* smask;  // target-set membership (masked launches: onion layer)
  const uint8_t* excl;   // voxels excluded from comparisons and votes (onion: H')
  uint64_t step;    // EM index at the level (Philox counter word 1)
  unsigned long long* absdiff;     // spread counters (kCntWords words each)
  unsigned long long* evals;       // distances computed by the passes
  unsigned long long* evals_init;  // distances computed by step 0
  int32_t R[kMaxPmIters + 1];  // random-search radius of iteration k
};

constexpr int kPixChunk = 256;  // hole pixels per chunk of a batched reconstruction
constexpr size_t kMarkPad = 16;  // zero entries before and after the marks of a level
// (and the onion's exclusion masks)
constexpr size_t kVoxPad = 2;    // voxel entries before and after a level's video

constexpr int kQueueSlots = 1024;  // chunk counters, one per launch of a batched iteration

// Counters that every wave adds to (evaluation counts, |change| sums) are
// spread over kCntSlots slots, one 128-byte line each: a wave adds its sum to
// the slot of its wave index, and a reader sums the slots.  Tens of thousands
// of device-scope atomics on one address per launch serialise in the memory
// system and cost more than the work they count.
constexpr int kCntSlots = 64;
constexpr int kCntStride = 16;  // 64-bit words per slot
constexpr int kCntWords = kCntSlots * kCntStride;

struct BatchArgs {
  const JobDesc* jobs;
  const int32_t* tchunk_job;  // job of every target chunk
  const int32_t* pchunk_job;  // job of every pixel chunk
  const int32_t* counts;      // [0] target chunks, [1] pixel chunks, [2] jobs
  int32_t* queue;             // [kQueueSlots] next chunk of each persistent launch
  int32_t direct;             // 1: one workgroup per chunk (grid = chunk count)
};

// out[i] = sum of the slots of the spread counter base + i * kCntWords, i < n
void launch_sum_spread(hipStream_t st, const unsigned long long* base, int32_t n,
                       unsigned long long* out);

// ---------------------------------------------------------------- launchers
// All launch on `st`; none synchronises.
void launch_init_level0(hipStream_t st, const uint8_t* rgb, const uint8_t* mask, DevLevel L0);
void launch_pyr_down(hipStream_t st, DevLevel F, DevLevel C);
void launch_texture(hipStream_t st, const uint8_t* rgb, DevLevel L0, int32_t s,
                    uint32_t* gpk, uint2* hsum);
void launch_texture_level(hipStream_t st, const uint2* hsum, DevLevel L0, DevLevel Ll,
                          int32_t l, int32_t s);
// separable 5x5x5 box dilation of src into dst (tmp: two scratch volumes)
void launch_dilate5(hipStream_t st, const uint8_t* src, uint8_t* dst, uint8_t* tmp1,
                    uint8_t* tmp2, int32_t W, int32_t H, int32_t T, const uint8_t* and_not);
void launch_sources(hipStream_t st, DevLevel L);
void launch_fill_nnf(hipStream_t st, int2* nnf, uint8_t* nvox, int32_t V);
void launch_fill_u64(hipStream_t st, unsigned long long* p, int32_t n);

// red: compare the reduced distance (unmasked searches of a level with
// features); launch_rerank then evaluates every target's match exactly
// wide_max as for launch_pass: step 0 of lists up to that size takes the group
// form
void launch_s0(hipStream_t st, DevLevel L, const PassArgs& A, bool red = false,
               int32_t wide_max = -1);
// Whether launch_pass takes the wide form for a target list of nS targets:
// exact passes (also the onion peel's masked ones) over at most wide_max
// targets (-1: the library's limit).
bool pass_is_wide(int32_t nS, bool red, int32_t wide_max);
void launch_pass(hipStream_t st, DevLevel L, const PassArgs& A, bool red = false,
                 int32_t wide_max = -1);
void launch_rerank(hipStream_t st, DevLevel L, const int32_t* tlist, int32_t nS);
void launch_copy_targets(hipStream_t st, const int32_t* tlist, int32_t nS, const int2* src,
                         int2* dst);

// skip: the previous reconstruction of the level was a full unmasked one of
// the same mode and nothing but searches changed the state since
void launch_recon(hipStream_t st, DevLevel L, const int32_t* plist, int32_t nP,
                  const uint8_t* filt_excl, int mode, float* out_f, unsigned long long* absdiff,
                  bool skip = false);
void launch_upsample(hipStream_t st, DevLevel F, DevLevel C, const int32_t* ftlist,
                     int32_t nS);

void launch_erode3(hipStream_t st, const uint8_t* Hp, uint8_t* E, uint8_t* bd, int32_t W,
                   int32_t H, int32_t T);

void launch_get_state(hipStream_t st, DevLevel L, uint8_t* rgbt, int32_t* cand, int32_t* dist,
                      uint8_t* nvox);
void launch_set_state(hipStream_t st, DevLevel L, const uint8_t* rgbt, const int32_t* cand,
                      const int32_t* dist, const uint8_t* nvox, unsigned long long* bad,
                      int write);
void launch_out_rgb(hipStream_t st, DevLevel L0, uint8_t* out);

// batched launches over every job's chunks: persistent (grid = `grid`
// workgroups taking chunks from a counter) or direct (B.direct: grid must be
// the chunk count; the pass kernel then takes exactly one chunk per
// workgroup); blk = targets per workgroup, 64, 128 or 256
// `slot` selects the chunk counter of the launch; launch_batch_zero clears
// the counters and the per-job outputs at the start of an iteration
void launch_batch_zero(hipStream_t st, const BatchArgs& B, int32_t max_jobs);
// masked: the onion peel's partial distance (J.excl) and target sets (J.smask)
void launch_batch_s0(hipStream_t st, const BatchArgs& B, int blk, int32_t grid, int32_t slot,
                     bool masked = false);
// t: index of the pass in the search (from 1); since: t - n_jf when a
// previous pass at the same stride exists, else 0 (no skipping)
void launch_batch_pass(hipStream_t st, const BatchArgs& B, int blk, int32_t grid, int32_t s,
                       int32_t k, int32_t parity, int32_t slot, int32_t t, int32_t since,
                       bool masked = false);
void launch_batch_copy(hipStream_t st, const BatchArgs& B, int blk, int32_t grid, int32_t slot);
void launch_batch_recon(hipStream_t st, const BatchArgs& B, int32_t grid, int32_t slot,
                        bool masked = false);
// out[j] = |change| sum of job j (the slots of its spread counter J.absdiff)
void launch_batch_sum_abs(hipStream_t st, const BatchArgs& B, int32_t max_jobs,
                          unsigned long long* out);

// Device memory and timing events reused across contexts (vi_pool.cpp).
// pool_alloc: a block of at least `bytes` on device `dev`, or nullptr;
// pool_free: returns a block that no queued work uses any more.
void* pool_alloc(int dev, size_t bytes);
void pool_free(int dev, void* p);
size_t pool_trim(int dev);
hipEvent_t event_get(int dev);
void event_put(int dev, hipEvent_t e);

// Realignment (vi_align.hip): the C ABI's checks are done by the caller;
// err receives a message on failure.  d_minv / d_m: device space for 6 T
// doubles.
vi_status align_estimate(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H, int32_t T,
                         const vi_align_params* prm, double* theta, hipStream_t st,
                         std::string* err);
vi_status align_compose(const double* theta, int32_t T, double* M);
vi_status align_warp(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H, int32_t T,
                     const double* M, double* d_minv, uint8_t* out_rgb, uint8_t* out_mask,
                     hipStream_t st);
vi_status align_unwarp(const uint8_t* aligned, const uint8_t* rgb, const uint8_t* mask, int32_t W,
                       int32_t H, int32_t T, const double* M, double* d_m, uint8_t* out,
                       hipStream_t st);

// The textured-patch count of App. B (vi_appb.hip); arguments checked by
// the caller; work: closer_work_bytes(n_ref) bytes of device memory for the
// packed references.
size_t closer_work_bytes(int32_t n_ref);
vi_status closer_than_constant(const uint8_t* ref, int32_t n_ref, const uint8_t* vol, int32_t W,
                               int32_t H, int32_t T, int32_t pw, int32_t ph, int32_t pt,
                               int32_t mu, unsigned long long* counts, void* work,
                               hipStream_t st);

// Dimensionality-reduced patch space (vi_reduce.hip).  A basis on the
// device: Qp [rows][kPairs][dp] int32 (rows = dim / 25 patch rows (dt, dy);
// each row's 25 coordinates in 13 pairs, the low 16 bits coordinate 2m,
// the high 16 bits 2m + 1; dp = features rounded up to a multiple of 4,
// zero beyond them).  Features of the voxels of list (all voxels when null)
// into feat [V][dp].
constexpr int kPairs = 13;
void launch_features(hipStream_t st, const DevLevel& L, const int32_t* Qp, int32_t dim,
                     int32_t dp, const int32_t* list, int32_t n, int32_t* feat);
// bytes of device work space the PCA of one level needs
size_t pca_work_bytes(int32_t dim, int32_t n_max);
// exact moments of every k-th source's patch vector (k = ceil(nD / n_max));
// returns the sample count and points S1 [dim], S2 [dim][dim] into work
int64_t pca_moments(hipStream_t st, const DevLevel& L, int32_t dim, int32_t n_max, void* work,
                    unsigned long long** S1, unsigned long long** S2);
// the d leading principal directions of the weighted patch vectors (iters
// steps of orthogonal iteration), quantised: dQ [d][dim] and the device
// layout dQp; rq points into work at the captured variances [dp]
vi_status pca_basis(hipStream_t st, const DevLevel& L, int32_t dim, int32_t d, int32_t n_max,
                    int32_t iters, double wtex, void* work, int16_t* dQ, int32_t* dQp,
                    double** rq);

// stream compaction (stable): out[k] = i for the k-th i with flags[i] != 0
size_t compact_temp_bytes(int32_t n);
hipError_t compact(hipStream_t st, const uint8_t* flags, int32_t n, int32_t* out,
                   int32_t* d_count, void* temp, size_t temp_bytes);

}  // namespace vi
