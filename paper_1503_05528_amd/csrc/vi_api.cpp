// vi_api.cpp -- host orchestration and C ABI of libvi (see include/vi.h).
//
// Every step of the method runs in the kernels of vi_kernels.hip; this file
// validates arguments, owns device memory, sequences launches on the
// context's stream and implements the control flow of Alg. 4 (onion peel,
// EM loop with its stopping test, level transitions, final reconstruction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "vi.h"
#include "vi_internal.h"

namespace {

thread_local std::string g_err = "no error";

vi_status fail(vi_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define VI_HIP(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(VI_E_HIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

#define VI_TRY(expr)               \
  do {                             \
    vi_status s_ = (expr);         \
    if (s_ != VI_OK) return s_;    \
  } while (0)

constexpr int kMaxLevels = 8;

struct Level {
  vi::DevLevel d{};
  int32_t nH = 0, nS = 0;
  int32_t* hlist = nullptr;
  int32_t* tlist = nullptr;
  bool complete = false;
  // the last reconstruction of the level was a full unmasked one of mode
  // recon_last (weighted or mean), and since then only searches (which keep
  // the reconstruction marks) changed the state: the next one may skip
  bool recon_ok = false;
  int32_t recon_last = -1;
  // dimensionality-reduced patch space: basis in the feature kernel's layout
  // ([rows][kPairs][d.rd] int32), features [V][d.rd], entries before a
  // search, number of features in use
  int32_t* redQp = nullptr;
  int32_t* feat = nullptr;
  int2* prev = nullptr;
  int32_t red_n = 0;
};

}  // namespace

struct vi_ctx {
  vi_params prm{};
  int32_t L = 0;
  int32_t W = 0, H = 0, T = 0;
  hipStream_t st = nullptr;
  Level lv[kMaxLevels];
  int dev = 0;                                   // device of the context
  std::vector<std::pair<void*, size_t>> allocs;  // pooled blocks, requested sizes
  size_t bytes = 0;
  void* ctemp = nullptr;  // compaction scratch
  size_t ctemp_bytes = 0;
  int32_t* d_count = nullptr;             // [2]
  unsigned long long* d_u64 = nullptr;    // [0] |change| sum, [1..2] set_state checks,
                                          // [3..6] evaluation sums: one-lane passes, step
                                          // 0, onion, wide passes
  unsigned long long* d_cnt = nullptr;    // spread counters (kCntWords words each):
                                          // [0] |change|, [1..4] evaluations as d_u64[3..6]
  // onion-peel scratch (coarsest level)
  uint8_t *o_Hp = nullptr, *o_E = nullptr, *o_bd = nullptr, *o_S = nullptr;
  uint8_t *o_t1 = nullptr, *o_t2 = nullptr;
  int32_t *o_tl = nullptr, *o_pl = nullptr;
  // work counters (host side; effective evaluations live in d_cnt[1..4])
  int64_t n_nominal = 0, n_searches = 0, n_em = 0, n_recon = 0;
  // kernel timing with events on the context's stream
  uint32_t prof_mask = 0;  // kernel kinds timed (bit 1 << vi_kernel_kind)
  int32_t kind_override = -1;  // every launch of the onion peel is VI_K_ONION
  struct Rec {
    int32_t kind, level;
    int64_t units;
    int ev;
    int32_t launches;
  };
  std::vector<hipEvent_t> events;  // pairs (start, stop)
  std::vector<Rec> recs;
  // position in Alg. 4 when driven step by step (batches): phase 0 = not
  // started, 1 = EM loop of cur_level at iteration em_k, 2 = finished
  int32_t phase = 0;
  int32_t cur_level = -1;
  int32_t em_k = 0;
  // batch membership: the batch the clip belongs to and the clip's own
  // stream, given back when it leaves the batch
  vi_batch* batch = nullptr;
  hipStream_t own_st = nullptr;
};

namespace {

// removes a clip from its batch (defined with the batches below)
void batch_detach(vi_batch* b, vi_ctx* c);

template <typename T>
vi_status dalloc(vi_ctx* c, T** p, size_t n) {
  const size_t b = n * sizeof(T) > 0 ? n * sizeof(T) : 16;
  void* q = vi::pool_alloc(c->dev, b);
  if (!q) return fail(VI_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
  c->allocs.push_back({q, b});
  c->bytes += b;
  *p = static_cast<T*>(q);
  return VI_OK;
}

void dfree(vi_ctx* c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c->allocs.size(); ++i)
    if (c->allocs[i].first == p) {
      c->bytes -= c->allocs[i].second;
      vi::pool_free(c->dev, p);
      c->allocs.erase(c->allocs.begin() + (long)i);
      return;
    }
}

vi_status launched(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(VI_E_HIP, std::string("launch of ") + what + " failed: " + hipGetErrorString(e));
  return VI_OK;
}

// event pair around a launch of this kind while it is timed; returns the
// record index or -1
int prof_begin(vi_ctx* c, int32_t kind) {
  const int32_t k = c->kind_override >= 0 ? c->kind_override : kind;
  if (!(c->prof_mask & (1u << k))) return -1;
  const size_t need = 2 * (c->recs.size() + 1);
  while (c->events.size() < need) {
    hipEvent_t e = vi::event_get(c->dev);
    if (!e) return -1;
    c->events.push_back(e);
  }
  const int ev = (int)(2 * c->recs.size());
  if (hipEventRecord(c->events[ev], c->st) != hipSuccess) return -1;
  c->recs.push_back({0, 0, 0, ev, 0});
  return (int)c->recs.size() - 1;
}

void prof_end(vi_ctx* c, int r, int32_t kind, int32_t level, int64_t units,
              int32_t launches = 1) {
  if (r < 0) return;
  vi_ctx::Rec& rec = c->recs[(size_t)r];
  rec.kind = c->kind_override >= 0 ? c->kind_override : kind;
  rec.level = level;
  rec.units = units;
  rec.launches = launches;
  (void)hipEventRecord(c->events[(size_t)rec.ev + 1], c->st);
}

int64_t per_target_evals(const vi_params& p, int32_t rmax);

// coordinates of a patch vector: 5 channels per voxel
int32_t patch_dim(const vi_params& p) { return 5 * p.patch[0] * p.patch[1] * p.patch[2]; }

vi_status check_params(const vi_params* p) {
  if (!p) return fail(VI_E_INVAL, "null params");
  if (p->abi_version != 1) return fail(VI_E_INVAL, "abi_version must be 1");
  if (p->patch[0] != 5 || p->patch[1] != 5 || (p->patch[2] != 5 && p->patch[2] != 1))
    return fail(VI_E_INVAL, "patches are 5x5x5 (videos) or 5x5x1 (single images)");
  if (p->patch[2] == 1 && p->temporal_subsample)
    return fail(VI_E_INVAL, "5x5x1 patches are for single images: no temporal subsampling");
  if (p->levels < 1 || p->levels > kMaxLevels) return fail(VI_E_INVAL, "levels must be in [1, 8]");
  if (p->lambda < 0 || p->lambda > 130) return fail(VI_E_INVAL, "lambda must be in [0, 130]");
  if (p->pm_iters < 0 || p->pm_iters > 64) return fail(VI_E_INVAL, "pm_iters must be in [0, 64]");
  if (p->n_jf < 0 || p->n_jf > 8) return fail(VI_E_INVAL, "n_jf must be in [0, 8]");
  for (int i = 0; i < p->n_jf; ++i)
    if (p->jf_steps[i] < 1 || p->jf_steps[i] > 4)
      return fail(VI_E_INVAL, "jump-flood steps must be in [1, 4]");
  if (!(p->rho > 0.0 && p->rho <= 1.0)) return fail(VI_E_INVAL, "rho must be in (0, 1]");
  if (p->em_max_iters < 1) return fail(VI_E_INVAL, "em_max_iters must be >= 1");
  if (p->recon_mode != VI_RECON_WEIGHTED && p->recon_mode != VI_RECON_MEAN)
    return fail(VI_E_INVAL, "recon_mode must be WEIGHTED or MEAN");
  if (p->temporal_subsample != 0 && p->temporal_subsample != 1)
    return fail(VI_E_INVAL, "temporal_subsample must be 0 or 1");
  if (p->reduce_dims < 0 || p->reduce_dims > vi::kMaxRed)
    return fail(VI_E_INVAL, "reduce_dims must be in [0, 32]");
  if (p->wide_pass_max < -1) return fail(VI_E_INVAL, "wide_pass_max must be >= -1");
  return VI_OK;
}

// frames of the next coarser level
int32_t coarser_T(const vi_params* p, int32_t T) { return p->temporal_subsample ? (T + 1) / 2 : T; }

vi_status check_dims(const vi_params* p, int32_t W, int32_t H, int32_t T) {
  if (p->patch[2] == 1 && T != 1) return fail(VI_E_INVAL, "5x5x1 patches need T = 1 (one image)");
  if (W < 5 || H < 5 || T < p->patch[2] || W >= 32768 || H >= 32768 || T >= 32768)
    return fail(VI_E_INVAL, "W, H must be in [5, 32768), T in [patch depth, 32768)");
  if ((int64_t)W * H * T >= (int64_t(1) << 31)) return fail(VI_E_INVAL, "W*H*T must be < 2^31");
  int32_t w = W, h = H, t = T;
  for (int l = 1; l < p->levels; ++l) {
    w = (w + 1) / 2;
    h = (h + 1) / 2;
    t = coarser_T(p, t);
  }
  if (w < 5 || h < 5 || t < p->patch[2])
    return fail(VI_E_INVAL, "the coarsest level is smaller than a patch");
  return VI_OK;
}

vi_status sync(vi_ctx* c) {
  VI_HIP(hipStreamSynchronize(c->st));
  return VI_OK;
}

// stable compaction of flags into a fresh exact-size list
vi_status compact_to(vi_ctx* c, const uint8_t* flags, int32_t n, int32_t* tmp_list,
                     int32_t** out, int32_t* count) {
  VI_HIP(vi::compact(c->st, flags, n, tmp_list, c->d_count, c->ctemp, c->ctemp_bytes));
  int32_t h = 0;
  VI_HIP(hipMemcpyAsync(&h, c->d_count, sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
  VI_TRY(sync(c));
  VI_TRY(dalloc(c, out, (size_t)h));
  if (h > 0)
    VI_HIP(hipMemcpyAsync(*out, tmp_list, sizeof(int32_t) * (size_t)h, hipMemcpyDeviceToDevice,
                          c->st));
  *count = h;
  return VI_OK;
}

int32_t r_max(const vi::DevLevel& d) {
  int32_t r = d.W > d.H ? d.W : d.H;
  return r > d.T ? r : d.T;
}

int32_t rs_radius(const vi_params& p, int32_t rmax, int k) {
  double r = (double)rmax;
  for (int i = 0; i < k; ++i) r *= p.rho;
  return (int32_t)std::floor(r);
}

// nominal evaluations per target of one search: the initial evaluation, six
// neighbour candidates per propagation pass, one random candidate per
// iteration with a radius of at least one
int64_t per_target_evals(const vi_params& p, int32_t rmax) {
  int64_t per = 1;
  for (int k = 1; k <= p.pm_iters; ++k)
    per += 6 * p.n_jf + (rs_radius(p, rmax, k) >= 1 ? 1 : 0);
  return per;
}

// ANN search over a target list (Sec. 3.1, Alg. 1): step 0, then K
// iterations of propagation passes with the random search fused into the
// last pass.  The result always ends in nnf0.
vi_status search(vi_ctx* c, int32_t level, const int32_t* tlist, int32_t nS,
                 const uint8_t* smask, const uint8_t* excl, uint64_t step) {
  Level& lv = c->lv[level];
  const vi::DevLevel& d = lv.d;
  if (nS <= 0) return VI_OK;
  const int32_t rmax = r_max(d);
  c->n_nominal += per_target_evals(c->prm, rmax) * (int64_t)nS;
  c->n_searches += 1;
  vi::PassArgs A{};
  A.tlist = tlist;
  A.nS = nS;
  A.smask = smask;
  A.excl = excl;
  A.step = step;
  // the reduced distance (unmasked searches of a level with a basis): the
  // targets' features on the current video first
  const bool red = d.rd > 0 && !excl;
  // onion searches (masked) count apart from the EM loop's, and the EM
  // loop's passes of the wide form apart from the one-lane form's
  const bool wide = vi::pass_is_wide(nS, red, c->prm.wide_pass_max);
  unsigned long long* ev_pass = c->d_cnt + (size_t)(excl ? 3 : (wide ? 4 : 1)) * vi::kCntWords;
  unsigned long long* ev_init = c->d_cnt + (size_t)(excl ? 3 : 2) * vi::kCntWords;
  A.evals = ev_init;
  A.nin = d.nnf0;
  A.nout = d.nnf0;
  int r;
  if (red) {
    r = prof_begin(c, VI_K_OTHER);
    vi::launch_features(c->st, d, lv.redQp, patch_dim(c->prm), d.rd, tlist, nS, lv.feat);
    prof_end(c, r, VI_K_OTHER, level, nS);
    VI_TRY(launched("features"));
  }
  r = prof_begin(c, VI_K_INIT);
  vi::launch_s0(c->st, d, A, red, c->prm.wide_pass_max);
  A.evals = ev_pass;
  prof_end(c, r, VI_K_INIT, level, nS);
  VI_TRY(launched("s0"));
  int2* buf[2] = {d.nnf0, d.nnf1};
  int cur = 0;
  // the passes run back to back: one event pair covers all of them
  const int32_t pass_kind = wide ? VI_K_PASS_WIDE : VI_K_PASS;
  r = prof_begin(c, pass_kind);
  int64_t pass_units = 0;
  int32_t n_pass = 0;
  int32_t t = 0;
  for (int k = 1; k <= c->prm.pm_iters; ++k) {
    const int32_t R = rs_radius(c->prm, rmax, k);
    const bool rs = R >= 1;
    const int np = c->prm.n_jf > 0 ? c->prm.n_jf : 1;
    if (c->prm.n_jf == 0 && !rs) continue;
    for (int js = 0; js < np; ++js) {
      A.nin = buf[cur];
      A.nout = buf[cur ^ 1];
      A.s = c->prm.n_jf > 0 ? c->prm.jf_steps[js] : 0;
      A.rs_k = (js == np - 1 && rs) ? k : 0;
      A.R = R;
      // passes are numbered from 1 within the search; a target may keep its
      // match without evaluating when nothing around it changed since the
      // previous pass at the same stride
      A.t = ++t;
      A.since = (c->prm.n_jf > 0 && t > np) ? t - np : 0;
      vi::launch_pass(c->st, d, A, red, c->prm.wide_pass_max);
      pass_units += (int64_t)nS;
      ++n_pass;
      VI_TRY(launched("pass"));
      cur ^= 1;
    }
  }
  if (n_pass > 0)
    prof_end(c, r, pass_kind, level, pass_units, n_pass);
  else if (r >= 0)
    c->recs.pop_back();
  if (cur == 1) {
    r = prof_begin(c, VI_K_OTHER);
    vi::launch_copy_targets(c->st, tlist, nS, d.nnf1, d.nnf0);
    prof_end(c, r, VI_K_OTHER, level, nS);
    VI_TRY(launched("copy"));
  }
  if (red) {
    // the reconstruction weighs the matches by their exact distances
    r = prof_begin(c, VI_K_OTHER);
    vi::launch_rerank(c->st, d, tlist, nS);
    prof_end(c, r, VI_K_OTHER, level, nS);
    VI_TRY(launched("rerank"));
  }
  return VI_OK;
}

// the next reconstruction epoch of a level (marks are 8-bit, 0 = never)
void next_epoch(Level& lv) {
  lv.d.repoch = lv.d.repoch >= 0xFF ? 1 : lv.d.repoch + 1;
}

// absdiff (optional, one word of device memory) receives the pixels' |change|
// sum, gathered in the spread counter d_cnt[0].  A full unmasked weighted or
// plain reconstruction without float output may keep the pixels whose
// contributors did not change since the previous one of the same mode.
vi_status recon(vi_ctx* c, int32_t level, const int32_t* plist, int32_t nP, const uint8_t* excl,
                int mode, float* out_f, unsigned long long* absdiff) {
  Level& lv = c->lv[level];
  const bool full = !excl && plist == lv.hlist && nP == lv.nH && mode != VI_RECON_BEST;
  const bool skip = full && !out_f && lv.recon_ok && lv.recon_last == mode;
  unsigned long long* spread = absdiff ? c->d_cnt : nullptr;
  if (spread) vi::launch_fill_u64(c->st, spread, vi::kCntWords);
  c->n_recon += nP;
  const int r = prof_begin(c, VI_K_RECON);
  vi::launch_recon(c->st, lv.d, plist, nP, excl, mode, out_f, spread, skip);
  prof_end(c, r, VI_K_RECON, level, nP);
  next_epoch(lv);
  lv.recon_ok = full;
  lv.recon_last = mode;
  if (spread) vi::launch_sum_spread(c->st, spread, 1, absdiff);
  return launched("recon");
}

vi_status level_ok(const vi_ctx* c, int32_t level) {
  if (!c) return fail(VI_E_INVAL, "null context");
  if (level < 0 || level >= c->L) return fail(VI_E_INVAL, "level out of range");
  return VI_OK;
}

vi_status inpaint_level(vi_ctx* c, int32_t level, int32_t* iters) {
  Level& lv = c->lv[level];
  int32_t k = 0;
  if (lv.nH > 0) {
    double e;
    do {
      VI_TRY(search(c, level, lv.tlist, lv.nS, lv.d.htil, nullptr, (uint64_t)k));
      VI_TRY(recon(c, level, lv.hlist, lv.nH, nullptr, c->prm.recon_mode, nullptr, c->d_u64));
      ++k;
      ++c->n_em;
      if (c->prm.em_tol < 0) {
        e = INFINITY;
      } else {
        unsigned long long s = 0;
        VI_HIP(hipMemcpyAsync(&s, c->d_u64, sizeof(s), hipMemcpyDeviceToHost, c->st));
        VI_TRY(sync(c));
        e = (double)s / (3.0 * (double)lv.nH);
      }
    } while (e > c->prm.em_tol && k < c->prm.em_max_iters);
  }
  lv.complete = true;
  if (iters) *iters = k;
  return VI_OK;
}

// scratch of the onion peel (allocated once per context)
vi_status onion_buffers(vi_ctx* c) {
  if (c->o_Hp) return VI_OK;
  const size_t V = (size_t)c->lv[c->L - 1].d.V;
  // exclusion masks: padded for the 8-byte row loads of the distance
  VI_TRY(dalloc(c, &c->o_Hp, V + 2 * vi::kMarkPad));
  VI_TRY(dalloc(c, &c->o_E, V + 2 * vi::kMarkPad));
  c->o_Hp += vi::kMarkPad;
  c->o_E += vi::kMarkPad;
  VI_TRY(dalloc(c, &c->o_bd, V));
  VI_TRY(dalloc(c, &c->o_S, V));
  VI_TRY(dalloc(c, &c->o_t1, V));
  VI_TRY(dalloc(c, &c->o_t2, V));
  VI_TRY(dalloc(c, &c->o_tl, V));
  VI_TRY(dalloc(c, &c->o_pl, V));
  return VI_OK;
}

// the peel starts from empty shift maps at the coarsest level
vi_status onion_empty_maps(vi_ctx* c) {
  Level& lv = c->lv[c->L - 1];
  lv.recon_ok = false;
  vi::launch_fill_nnf(c->st, lv.d.nnf0, lv.d.nvox, lv.d.V);
  vi::launch_fill_nnf(c->st, lv.d.nnf1, nullptr, lv.d.V);
  return launched("onion set-up");
}

// work buffers of one onion layer: H' and its erosion (both with
// kMarkPad bytes before and after: the masked distance reads H' in 8-byte
// rows), the layer and target flags, two dilation temporaries, and the
// compact layer and target lists
struct OnionBufs {
  uint8_t *Hp, *E, *bd, *S, *t1, *t2;
  int32_t *tl, *pl;
};

OnionBufs ctx_onion_bufs(vi_ctx* c) {
  return OnionBufs{c->o_Hp, c->o_E, c->o_bd, c->o_S, c->o_t1, c->o_t2, c->o_tl, c->o_pl};
}

// One layer of Alg. 3 at the coarsest level: E = erosion of H' (B.Hp), the
// layer bd = H' \ E and its targets S = dilate(bd) \ H'; search of S with
// the distance over voxels outside H', reconstruction of bd from the
// contributors outside H'.  *nb receives |bd| (0: H' is empty, nothing
// searched).  Syncs.
vi_status onion_step(vi_ctx* c, const OnionBufs& B, int32_t layer, float* out_f, int32_t* nb) {
  const int32_t level = c->L - 1;
  const vi::DevLevel& d = c->lv[level].d;
  const int r = prof_begin(c, VI_K_OTHER);
  vi::launch_erode3(c->st, B.Hp, B.E, B.bd, d.W, d.H, d.T);
  vi::launch_dilate5(c->st, B.bd, B.S, B.t1, B.t2, d.W, d.H, d.T, B.Hp);
  prof_end(c, r, VI_K_OTHER, level, d.V);
  VI_TRY(launched("onion layer"));
  VI_HIP(vi::compact(c->st, B.bd, d.V, B.pl, c->d_count, c->ctemp, c->ctemp_bytes));
  VI_HIP(vi::compact(c->st, B.S, d.V, B.tl, c->d_count + 1, c->ctemp, c->ctemp_bytes));
  int32_t cnt[2] = {0, 0};
  VI_HIP(hipMemcpyAsync(cnt, c->d_count, sizeof(cnt), hipMemcpyDeviceToHost, c->st));
  VI_TRY(sync(c));
  *nb = cnt[0];
  if (cnt[0] == 0) return VI_OK;
  VI_TRY(search(c, level, B.tl, cnt[1], B.S, B.Hp, (uint64_t(1) << 32) + (uint64_t)layer));
  return recon(c, level, B.pl, cnt[0], B.Hp, c->prm.recon_mode, out_f, nullptr);
}

// the start of a peel: scratch, empty shift maps, H' = the coarsest hole
vi_status onion_prepare(vi_ctx* c) {
  const vi::DevLevel& d = c->lv[c->L - 1].d;
  VI_TRY(onion_buffers(c));
  VI_TRY(onion_empty_maps(c));
  VI_HIP(hipMemcpyAsync(c->o_Hp, d.hole, (size_t)d.V, hipMemcpyDeviceToDevice, c->st));
  return VI_OK;
}

vi_status onion(vi_ctx* c, int32_t* layers_run) {
  const int32_t level = c->L - 1;
  Level& lv = c->lv[level];
  VI_TRY(onion_prepare(c));
  OnionBufs B = ctx_onion_bufs(c);
  int32_t layer = 0;
  struct Kind {
    vi_ctx* c;
    ~Kind() { c->kind_override = -1; }
  } kind_guard{c};
  c->kind_override = VI_K_ONION;
  for (;;) {
    int32_t nb = 0;
    VI_TRY(onion_step(c, B, layer, nullptr, &nb));
    if (nb == 0) break;  // no layer left: H' is empty
    std::swap(B.Hp, B.E);
    ++layer;
  }
  lv.complete = false;  // the innermost layer's targets may be unmatched
  if (layers_run) *layers_run = layer;
  return VI_OK;
}

vi_status transition(vi_ctx* c, int32_t level) {
  Level& F = c->lv[level];
  Level& C = c->lv[level + 1];
  if (!C.complete) return fail(VI_E_STATE, "the coarser level has no complete shift map");
  const int r = prof_begin(c, VI_K_OTHER);
  vi::launch_upsample(c->st, F.d, C.d, F.tlist, F.nS);
  prof_end(c, r, VI_K_OTHER, level, F.nS);
  VI_TRY(launched("upsample"));
  F.complete = true;
  F.recon_ok = false;  // the upsampling sets no reconstruction marks
  return recon(c, level, F.hlist, F.nH, nullptr, c->prm.recon_mode, nullptr, nullptr);
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed scratch of vi_onion_layer_noalloc: one array per GPU, resolved once
// per device with hipGetSymbolAddress; host code uses only the resolved
// device address, never the array's name.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocBytes = size_t(16) << 20;
constexpr int kNoAllocDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kNoAllocDevices] = {};

// bytes of one 256-aligned segment
size_t seg(size_t b) { return (b + 255) & ~size_t(255); }

// scratch bytes one onion layer needs for a level of V voxels
size_t noalloc_bytes(size_t V) {
  return 2 * seg(V + 2 * vi::kMarkPad) + 4 * seg(V) + 2 * seg(4 * V);
}

// the largest V with noalloc_bytes(V) <= kNoAllocBytes (1 198 336)
int64_t noalloc_max_voxels() {
  int64_t lo = 0, hi = (int64_t)kNoAllocBytes;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (noalloc_bytes((size_t)mid) <= kNoAllocBytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

OnionBufs noalloc_bufs(unsigned char* base, size_t V) {
  OnionBufs B{};
  size_t o = 0;
  B.Hp = base + o + vi::kMarkPad;
  o += seg(V + 2 * vi::kMarkPad);
  B.E = base + o + vi::kMarkPad;
  o += seg(V + 2 * vi::kMarkPad);
  uint8_t** flags[4] = {&B.bd, &B.S, &B.t1, &B.t2};
  for (uint8_t** f : flags) {
    *f = base + o;
    o += seg(V);
  }
  B.tl = reinterpret_cast<int32_t*>(base + o);
  o += seg(4 * V);
  B.pl = reinterpret_cast<int32_t*>(base + o);
  return B;
}

// the device address of this device's scratch array (set up once per device,
// with that device current)
vi_status noalloc_scratch(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kNoAllocDevices) return fail(VI_E_INVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    VI_HIP(hipGetDevice(&cur));
    if (cur != dev) VI_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(VI_E_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return VI_OK;
}

}  // namespace

namespace {

// device work space for the PCA of a level, released when it goes out of
// scope (after the caller's synchronisation)
struct PcaBuf {
  int dev = 0;
  void* p = nullptr;
  vi_status get(int d, size_t bytes) {
    dev = d;
    p = vi::pool_alloc(dev, bytes);
    return p ? VI_OK : fail(VI_E_NOMEM, "device allocation of the PCA work space failed");
  }
  ~PcaBuf() {
    if (p) vi::pool_free(dev, p);
  }
};

// Installs the basis already in lv.redQp (n features, dp columns) and
// computes the features of every voxel of the level on the current video.
vi_status install_reduction(vi_ctx* c, int32_t level, int32_t n) {
  Level& lv = c->lv[level];
  const int32_t dp = (n + 3) & ~3;
  if (lv.feat && lv.d.rd != dp) {
    dfree(c, lv.feat);
    lv.feat = nullptr;
  }
  if (!lv.feat) VI_TRY(dalloc(c, &lv.feat, (size_t)lv.d.V * dp));
  if (!lv.prev) VI_TRY(dalloc(c, &lv.prev, (size_t)lv.d.V));
  lv.d.feat = lv.feat;
  lv.d.prev = lv.prev;
  lv.d.rd = dp;
  lv.red_n = n;
  vi::launch_features(c->st, lv.d, lv.redQp, patch_dim(c->prm), dp, nullptr, lv.d.V, lv.feat);
  return launched("features");
}

// The PCA basis of a level's source patches (d features, n_max samples,
// iters steps) into lv.redQp; Q (host [d][dim]) and var (host [d]) optional.
vi_status level_pca(vi_ctx* c, int32_t level, int32_t d, int32_t n_max, int32_t iters,
                    int16_t* Q, double* var) {
  Level& lv = c->lv[level];
  const int32_t dim = patch_dim(c->prm);
  if (!lv.redQp) VI_TRY(dalloc(c, &lv.redQp, (size_t)(dim / 25) * vi::kPairs * vi::kMaxRed));
  PcaBuf work, qbuf;
  VI_TRY(work.get(c->dev, vi::pca_work_bytes(dim, n_max)));
  VI_TRY(qbuf.get(c->dev, sizeof(int16_t) * (size_t)dim * vi::kMaxRed));
  double* rq = nullptr;
  const vi_status st =
      vi::pca_basis(c->st, lv.d, dim, d, n_max, iters, std::sqrt((double)c->prm.lambda),
                    work.p, static_cast<int16_t*>(qbuf.p), lv.redQp, &rq);
  if (st != VI_OK) return fail(st, "PCA launch failed");
  if (Q)
    VI_HIP(hipMemcpyAsync(Q, qbuf.p, sizeof(int16_t) * (size_t)d * dim, hipMemcpyDeviceToHost,
                          c->st));
  if (var) VI_HIP(hipMemcpyAsync(var, rq, sizeof(double) * d, hipMemcpyDeviceToHost, c->st));
  return sync(c);
}

}  // namespace

extern "C" {

vi_status vi_params_default(vi_params* o) {
  if (!o) return fail(VI_E_INVAL, "null params");
  std::memset(o, 0, sizeof(*o));
  o->abi_version = 1;
  o->patch[0] = o->patch[1] = o->patch[2] = 5;
  o->levels = 1;
  o->lambda = 50;
  o->pm_iters = 10;
  o->n_jf = 3;
  o->jf_steps[0] = 4;
  o->jf_steps[1] = 2;
  o->jf_steps[2] = 1;
  o->rho = 0.5;
  o->em_max_iters = 20;
  o->em_tol = 0.1;
  o->recon_mode = VI_RECON_WEIGHTED;
  o->seed = 0;
  o->temporal_subsample = 0;
  o->reduce_dims = 0;
  o->wide_pass_max = -1;
  return VI_OK;
}

const char* vi_last_error(void) { return g_err.c_str(); }

size_t vi_footprint_bytes(const vi_params* prm, int32_t W, int32_t H, int32_t T,
                          double hole_fraction) {
  if (check_params(prm) != VI_OK || check_dims(prm, W, H, T) != VI_OK) return 0;
  if (!(hole_fraction >= 0.0 && hole_fraction <= 1.0)) return 0;
  size_t total = 0;
  int64_t w = W, h = H, t = T;
  const int64_t V0 = (int64_t)W * H * T;
  for (int l = 0; l < prm->levels; ++l) {
    const int64_t V = w * h * t;
    // vox 8, hole/dsrc/htil 3, nnf 16, nvox 1, change marks 3, source list 4
    total += (size_t)V * 35;
    // target and hole lists: the dilated hole is at most 125x the hole
    const double fr = hole_fraction * 125.0 < 1.0 ? hole_fraction * 125.0 : 1.0;
    total += (size_t)((double)V * (fr + hole_fraction) * 4.0) + 4096;
    // reduced patch space: features and basis
    if (prm->reduce_dims > 0)
      total += (size_t)V * (4 * (size_t)((prm->reduce_dims + 3) & ~3) + 8) +
               2 * vi::kPatchDimMax * vi::kMaxRed;
    w = (w + 1) / 2;
    h = (h + 1) / 2;
    t = coarser_T(prm, (int32_t)t);
  }
  // creation temporaries at the finest level: gradients 4, box sums 8,
  // dilation scratch 2, compaction list 4
  total += (size_t)V0 * 18;
  if (prm->reduce_dims > 0) total += vi::pca_work_bytes(patch_dim(*prm), 65536);
  return total + (size_t)(64u << 20);
}

vi_status vi_create(vi_ctx** out, const vi_params* prm, int32_t W, int32_t H, int32_t T,
                    const uint8_t* video_rgb, const uint8_t* mask, void* hip_stream) {
  if (!out) return fail(VI_E_INVAL, "null output handle");
  *out = nullptr;
  VI_TRY(check_params(prm));
  VI_TRY(check_dims(prm, W, H, T));
  if (!video_rgb || !mask) return fail(VI_E_INVAL, "null input pointer");
  vi_ctx* c = new (std::nothrow) vi_ctx();
  if (!c) return fail(VI_E_NOMEM, "host allocation failed");
  if (hipGetDevice(&c->dev) != hipSuccess) {
    delete c;
    return fail(VI_E_HIP, "no current device");
  }
  c->prm = *prm;
  c->L = prm->levels;
  c->W = W;
  c->H = H;
  c->T = T;
  c->st = static_cast<hipStream_t>(hip_stream);
  vi_status st = VI_OK;
  auto bail = [&](vi_status s) {
    vi_destroy(c);
    return s;
  };
  // level geometry and buffers
  int32_t w = W, h = H, tl = T;
  for (int l = 0; l < c->L; ++l) {
    vi::DevLevel& d = c->lv[l].d;
    d.W = w;
    d.H = h;
    d.T = tl;
    d.WH = w * h;
    d.V = w * h * tl;
    d.level = l;
    d.fdW = vi::make_fastdiv((uint32_t)w);
    d.fdWH = vi::make_fastdiv((uint32_t)(w * h));
    d.lambda = prm->lambda;
    d.seed = prm->seed;
    d.ht = prm->patch[2] / 2;
    const size_t V = (size_t)d.V;
    if ((st = dalloc(c, &d.vox, V + 2 * vi::kVoxPad)) || (st = dalloc(c, &d.hole, V)) ||
        (st = dalloc(c, &d.dsrc, V)) || (st = dalloc(c, &d.htil, V)) ||
        (st = dalloc(c, &d.nnf0, V)) ||
        (st = dalloc(c, &d.nnf1, V)) || (st = dalloc(c, &d.nvox, V)) ||
        (st = dalloc(c, &d.chg, V)) || (st = dalloc(c, &d.rmark, V + 2 * vi::kMarkPad)))
      return bail(st);
    if (hipMemsetAsync(d.chg, 0, sizeof(uint16_t) * (size_t)V, c->st) != hipSuccess ||
        hipMemsetAsync(d.rmark, 0, V + 2 * vi::kMarkPad, c->st) !=
            hipSuccess)
      return bail(fail(VI_E_HIP, "clearing the change marks failed"));
    // the blocks are released through the context's list
    d.rmark += vi::kMarkPad;
    d.vox += vi::kVoxPad;
    d.repoch = 1;
    w = (w + 1) / 2;
    h = (h + 1) / 2;
    tl = coarser_T(prm, tl);
  }
  const vi::DevLevel& L0 = c->lv[0].d;
  const size_t V0 = (size_t)L0.V;
  if ((st = dalloc(c, &c->d_count, 4)) || (st = dalloc(c, &c->d_u64, 8)) ||
      (st = dalloc(c, &c->d_cnt, 5 * (size_t)vi::kCntWords)))
    return bail(st);
  vi::launch_fill_u64(c->st, c->d_u64, 8);
  vi::launch_fill_u64(c->st, c->d_cnt, 5 * vi::kCntWords);
  c->ctemp_bytes = vi::compact_temp_bytes(L0.V);
  if ((st = dalloc(c, reinterpret_cast<uint8_t**>(&c->ctemp), c->ctemp_bytes))) return bail(st);
  // creation temporaries
  uint32_t* gpk = nullptr;
  uint2* hsum = nullptr;
  uint8_t *t1 = nullptr, *t2 = nullptr;
  int32_t* tmp_list = nullptr;
  if ((st = dalloc(c, &gpk, V0)) || (st = dalloc(c, &hsum, V0)) || (st = dalloc(c, &t1, V0)) ||
      (st = dalloc(c, &t2, V0)) || (st = dalloc(c, &tmp_list, V0)))
    return bail(st);
  // pyramids (Alg. 4) and texture features (Sec. 3.3)
  vi::launch_init_level0(c->st, video_rgb, mask, L0);
  for (int l = 1; l < c->L; ++l) vi::launch_pyr_down(c->st, c->lv[l - 1].d, c->lv[l].d);
  const int32_t s = 1 << (c->L - 1);
  vi::launch_texture(c->st, video_rgb, L0, s, gpk, hsum);
  for (int l = 0; l < c->L; ++l) vi::launch_texture_level(c->st, hsum, L0, c->lv[l].d, l, s);
  if ((st = launched("pyramids"))) return bail(st);
  // sets (Sec. 2), empty shift maps
  for (int l = 0; l < c->L; ++l) {
    Level& lv = c->lv[l];
    vi::DevLevel& d = lv.d;
    vi::launch_dilate5(c->st, d.hole, d.htil, t1, t2, d.W, d.H, d.T, nullptr);
    vi::launch_sources(c->st, d);
    vi::launch_fill_nnf(c->st, d.nnf0, d.nvox, d.V);
    vi::launch_fill_nnf(c->st, d.nnf1, nullptr, d.V);
    if ((st = launched("sets"))) return bail(st);
    if ((st = compact_to(c, d.dsrc, d.V, tmp_list, &d.dlist, &d.nD))) return bail(st);
    if ((st = compact_to(c, d.htil, d.V, tmp_list, &lv.tlist, &lv.nS))) return bail(st);
    if ((st = compact_to(c, d.hole, d.V, tmp_list, &lv.hlist, &lv.nH))) return bail(st);
    if (d.nD == 0) return bail(fail(VI_E_EMPTY_SOURCE, "level " + std::to_string(l) +
                                                           " has no hole-free patch"));
  }
  if ((st = sync(c))) return bail(st);
  dfree(c, gpk);
  dfree(c, hsum);
  dfree(c, t1);
  dfree(c, t2);
  dfree(c, tmp_list);
  // the reduced patch space of every level: PCA of its own sources
  for (int l = 0; l < c->L && prm->reduce_dims > 0; ++l) {
    if ((st = level_pca(c, l, prm->reduce_dims, 65536, 32, nullptr, nullptr))) return bail(st);
    if ((st = install_reduction(c, l, prm->reduce_dims))) return bail(st);
  }
  if (prm->reduce_dims > 0 && (st = sync(c))) return bail(st);
  *out = c;
  return VI_OK;
}

void vi_destroy(vi_ctx* c) {
  if (!c) return;
  if (c->batch) batch_detach(c->batch, c);
  // nothing queued uses the blocks after this: they may serve any stream
  (void)hipStreamSynchronize(c->st);
  for (const auto& a : c->allocs) vi::pool_free(c->dev, a.first);
  for (hipEvent_t e : c->events) vi::event_put(c->dev, e);
  delete c;
}

vi_status vi_set_stream(vi_ctx* c, void* hip_stream) {
  if (!c) return fail(VI_E_INVAL, "null context");
  if (c->batch) return fail(VI_E_STATE, "the clip is in a batch: its work runs on the batch's stream");
  c->st = static_cast<hipStream_t>(hip_stream);
  return VI_OK;
}

size_t vi_ctx_bytes(const vi_ctx* c) { return c ? c->bytes : 0; }

vi_status vi_level_info(const vi_ctx* c, int32_t level, int32_t dims[3], int64_t counts[3]) {
  VI_TRY(level_ok(c, level));
  const Level& lv = c->lv[level];
  if (dims) {
    dims[0] = lv.d.W;
    dims[1] = lv.d.H;
    dims[2] = lv.d.T;
  }
  if (counts) {
    counts[0] = lv.nH;
    counts[1] = lv.nS;
    counts[2] = lv.d.nD;
  }
  return VI_OK;
}

vi_status vi_level_sets(const vi_ctx* c, int32_t level, uint8_t* hole, uint8_t* dsrc,
                        uint8_t* htil) {
  VI_TRY(level_ok(c, level));
  const vi::DevLevel& d = c->lv[level].d;
  const size_t V = (size_t)d.V;
  if (hole) VI_HIP(hipMemcpyAsync(hole, d.hole, V, hipMemcpyDeviceToDevice, c->st));
  if (dsrc) VI_HIP(hipMemcpyAsync(dsrc, d.dsrc, V, hipMemcpyDeviceToDevice, c->st));
  if (htil) VI_HIP(hipMemcpyAsync(htil, d.htil, V, hipMemcpyDeviceToDevice, c->st));
  return VI_OK;
}

vi_status vi_nnf_search(vi_ctx* c, int32_t level, int32_t em_iter) {
  VI_TRY(level_ok(c, level));
  if (em_iter < 0) return fail(VI_E_INVAL, "em_iter must be >= 0");
  Level& lv = c->lv[level];
  VI_TRY(search(c, level, lv.tlist, lv.nS, lv.d.htil, nullptr, (uint64_t)em_iter));
  lv.complete = true;
  return VI_OK;
}

vi_status vi_reconstruct(vi_ctx* c, int32_t level, int32_t mode, float* out_f,
                         uint64_t* absdiff) {
  VI_TRY(level_ok(c, level));
  if (mode != VI_RECON_WEIGHTED && mode != VI_RECON_MEAN && mode != VI_RECON_BEST)
    return fail(VI_E_INVAL, "bad reconstruction mode");
  Level& lv = c->lv[level];
  if (!lv.complete) return fail(VI_E_STATE, "no complete shift map at this level");
  return recon(c, level, lv.hlist, lv.nH, nullptr, mode, out_f,
               reinterpret_cast<unsigned long long*>(absdiff));
}

vi_status vi_inpaint_level(vi_ctx* c, int32_t level, int32_t* em_iters_run) {
  VI_TRY(level_ok(c, level));
  return inpaint_level(c, level, em_iters_run);
}

vi_status vi_onion_init(vi_ctx* c, int32_t* layers_run) {
  if (!c) return fail(VI_E_INVAL, "null context");
  return onion(c, layers_run);
}

vi_status vi_onion_layer(vi_ctx* c, uint8_t* Hp, int32_t layer, float* out_f,
                         int64_t* n_layer) {
  if (!c || !Hp) return fail(VI_E_INVAL, "null argument");
  if (layer < 0) return fail(VI_E_INVAL, "layer must be >= 0");
  if (c->batch) return fail(VI_E_STATE, "the clip is in a batch");
  Level& lv = c->lv[c->L - 1];
  const size_t V = (size_t)lv.d.V;
  VI_TRY(onion_buffers(c));
  if (layer == 0) VI_TRY(onion_empty_maps(c));
  lv.recon_ok = false;
  VI_HIP(hipMemcpyAsync(c->o_Hp, Hp, V, hipMemcpyDeviceToDevice, c->st));
  struct Kind {
    vi_ctx* c;
    ~Kind() { c->kind_override = -1; }
  } kind_guard{c};
  c->kind_override = VI_K_ONION;
  int32_t nb = 0;
  VI_TRY(onion_step(c, ctx_onion_bufs(c), layer, out_f, &nb));
  VI_HIP(hipMemcpyAsync(Hp, c->o_E, V, hipMemcpyDeviceToDevice, c->st));
  lv.complete = false;  // the inner layers' targets may be unmatched
  if (n_layer) *n_layer = nb;
  return sync(c);
}

vi_status vi_onion_layer_noalloc(vi_ctx* c, uint8_t* Hp, int32_t layer, float* out_f,
                                 int64_t* n_layer) {
  if (!c || !Hp) return fail(VI_E_INVAL, "null argument");
  if (layer < 0) return fail(VI_E_INVAL, "layer must be >= 0");
  if (c->batch) return fail(VI_E_STATE, "the clip is in a batch");
  Level& lv = c->lv[c->L - 1];
  const size_t V = (size_t)lv.d.V;
  if (noalloc_bytes(V) > kNoAllocBytes)
    return fail(VI_E_BUDGET, "the coarsest level has more voxels than the fixed scratch of "
                             "vi_onion_layer_noalloc holds (" +
                                 std::to_string(noalloc_max_voxels()) + ")");
  unsigned char* base = nullptr;
  VI_TRY(noalloc_scratch(c->dev, &base));
  const OnionBufs B = noalloc_bufs(base, V);
  // no timing events either: they may be created on first use
  struct Prof {
    vi_ctx* c;
    uint32_t mask;
    ~Prof() {
      c->prof_mask = mask;
      c->kind_override = -1;
    }
  } prof_guard{c, c->prof_mask};
  c->prof_mask = 0;
  c->kind_override = VI_K_ONION;
  if (layer == 0) VI_TRY(onion_empty_maps(c));
  lv.recon_ok = false;
  VI_HIP(hipMemcpyAsync(B.Hp, Hp, V, hipMemcpyDeviceToDevice, c->st));
  int32_t nb = 0;
  VI_TRY(onion_step(c, B, layer, out_f, &nb));
  VI_HIP(hipMemcpyAsync(Hp, B.E, V, hipMemcpyDeviceToDevice, c->st));
  lv.complete = false;  // the inner layers' targets may be unmatched
  if (n_layer) *n_layer = nb;
  return sync(c);
}

vi_status vi_align_params_default(vi_align_params* o) {
  if (!o) return fail(VI_E_INVAL, "null params");
  o->levels = 3;
  o->iters = 8;
  o->tukey_c = 20.0;
  return VI_OK;
}

vi_status vi_align_estimate(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H,
                            int32_t T, const vi_align_params* prm, double* theta,
                            void* hip_stream) {
  if (!rgb || !mask || !prm || !theta) return fail(VI_E_INVAL, "null argument");
  if (T < 2) return fail(VI_E_INVAL, "the motion estimation needs at least two frames");
  if (prm->levels < 1 || prm->levels > 8 || prm->iters < 0 || prm->iters > 100 ||
      !(prm->tukey_c > 0.0))
    return fail(VI_E_INVAL, "levels in [1, 8], iters in [0, 100], tukey_c > 0");
  if (W < 8 || H < 8 || W >= 32768 || H >= 32768 || (int64_t)W * H * T >= (int64_t(1) << 31))
    return fail(VI_E_INVAL, "W, H in [8, 32768) and W*H*T < 2^31");
  int32_t w = W, h = H;
  for (int l = 1; l < prm->levels; ++l) {
    w = (w + 1) / 2;
    h = (h + 1) / 2;
  }
  if (w < 8 || h < 8) return fail(VI_E_INVAL, "the coarsest estimation level is below 8x8");
  std::string err;
  const vi_status st = vi::align_estimate(rgb, mask, W, H, T, prm, theta,
                                          static_cast<hipStream_t>(hip_stream), &err);
  return st == VI_OK ? VI_OK : fail(st, "vi_align_estimate: " + err);
}

vi_status vi_align_compose(const double* theta, int32_t T, double* M) {
  if (!M || T < 1 || (T > 1 && !theta)) return fail(VI_E_INVAL, "null argument or T < 1");
  if (vi::align_compose(theta, T, M) != VI_OK) return fail(VI_E_INVAL, "a singular frame map");
  return VI_OK;
}

namespace {
// device space for 6 T doubles, from the block pool of the current device
struct MapBuf {
  int dev = 0;
  double* p = nullptr;
  vi_status get(int32_t T) {
    if (hipGetDevice(&dev) != hipSuccess) return fail(VI_E_HIP, "no current device");
    p = static_cast<double*>(vi::pool_alloc(dev, sizeof(double) * 6 * (size_t)T));
    return p ? VI_OK : fail(VI_E_NOMEM, "device allocation failed");
  }
  ~MapBuf() {
    if (p) vi::pool_free(dev, p);
  }
};
}  // namespace

vi_status vi_align_warp(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H,
                        int32_t T, const double* M, uint8_t* out_rgb, uint8_t* out_mask,
                        void* hip_stream) {
  if (!rgb || !mask || !M || !out_rgb || !out_mask) return fail(VI_E_INVAL, "null argument");
  if (W < 1 || H < 1 || T < 1 || W >= 32768 || H >= 32768 ||
      (int64_t)W * H * T >= (int64_t(1) << 31))
    return fail(VI_E_INVAL, "W, H, T >= 1 and W*H*T < 2^31");
  MapBuf buf;
  VI_TRY(buf.get(T));
  const vi_status st = vi::align_warp(rgb, mask, W, H, T, M, buf.p, out_rgb, out_mask,
                                      static_cast<hipStream_t>(hip_stream));
  return st == VI_OK ? VI_OK : fail(st, "vi_align_warp failed (singular map or HIP error)");
}

vi_status vi_align_unwarp(const uint8_t* aligned, const uint8_t* rgb, const uint8_t* mask,
                          int32_t W, int32_t H, int32_t T, const double* M, uint8_t* out_rgb,
                          void* hip_stream) {
  if (!aligned || !rgb || !mask || !M || !out_rgb) return fail(VI_E_INVAL, "null argument");
  if (W < 1 || H < 1 || T < 1 || W >= 32768 || H >= 32768 ||
      (int64_t)W * H * T >= (int64_t(1) << 31))
    return fail(VI_E_INVAL, "W, H, T >= 1 and W*H*T < 2^31");
  MapBuf buf;
  VI_TRY(buf.get(T));
  const vi_status st = vi::align_unwarp(aligned, rgb, mask, W, H, T, M, buf.p, out_rgb,
                                        static_cast<hipStream_t>(hip_stream));
  return st == VI_OK ? VI_OK : fail(st, "vi_align_unwarp failed (HIP error)");
}

vi_status vi_closer_than_constant(const uint8_t* ref, int32_t n_ref, const uint8_t* vol,
                                  int32_t W, int32_t H, int32_t T, int32_t pw, int32_t ph,
                                  int32_t pt, int32_t mu, uint64_t* counts, void* hip_stream) {
  if (n_ref < 0 || n_ref >= (1 << 24)) return fail(VI_E_INVAL, "n_ref in [0, 2^24)");
  if (n_ref > 0 && (!ref || !vol || !counts)) return fail(VI_E_INVAL, "null argument");
  if (pw < 1 || ph < 1 || pt < 1 || (int64_t)pw * ph * pt > 128)
    return fail(VI_E_INVAL, "patch sizes >= 1 with pw * ph * pt <= 128");
  if (mu < 0 || mu > 255) return fail(VI_E_INVAL, "mu in [0, 255]");
  if (W < 1 || H < 1 || T < 1 || (int64_t)W * H * T >= (int64_t(1) << 30))
    return fail(VI_E_INVAL, "W, H, T >= 1 and W * H * T < 2^30");
  if (n_ref == 0) return VI_OK;
  // the packed references: a workspace from the library's pool, released
  // once the stream has passed the call
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(VI_E_HIP, "no current device");
  void* work = vi::pool_alloc(dev, vi::closer_work_bytes(n_ref));
  if (!work) return fail(VI_E_NOMEM, "device allocation of the reference workspace failed");
  hipStream_t hs = static_cast<hipStream_t>(hip_stream);
  vi_status st = vi::closer_than_constant(ref, n_ref, vol, W, H, T, pw, ph, pt, mu,
                                          reinterpret_cast<unsigned long long*>(counts), work,
                                          hs);
  if (hipStreamSynchronize(hs) != hipSuccess && st == VI_OK) st = VI_E_HIP;
  vi::pool_free(dev, work);
  return st == VI_OK ? VI_OK : fail(st, "vi_closer_than_constant: launch failed");
}

vi_status vi_pca_moments(vi_ctx* c, int32_t level, int32_t n_max, uint64_t* S1, uint64_t* S2,
                         int64_t* n) {
  VI_TRY(level_ok(c, level));
  if (!S1 || !S2 || !n) return fail(VI_E_INVAL, "null output");
  if (n_max < 1 || n_max > (1 << 20)) return fail(VI_E_INVAL, "n_max must be in [1, 2^20]");
  const int32_t dim = patch_dim(c->prm);
  PcaBuf work;
  VI_TRY(work.get(c->dev, vi::pca_work_bytes(dim, n_max)));
  unsigned long long *d1 = nullptr, *d2 = nullptr;
  *n = vi::pca_moments(c->st, c->lv[level].d, dim, n_max, work.p, &d1, &d2);
  VI_TRY(launched("moments"));
  VI_HIP(hipMemcpyAsync(S1, d1, sizeof(uint64_t) * dim, hipMemcpyDeviceToHost, c->st));
  VI_HIP(hipMemcpyAsync(S2, d2, sizeof(uint64_t) * (size_t)dim * dim, hipMemcpyDeviceToHost,
                        c->st));
  return sync(c);
}

vi_status vi_pca_basis(vi_ctx* c, int32_t level, int32_t d, int32_t n_max, int32_t iters,
                       int16_t* Q, double* variance) {
  VI_TRY(level_ok(c, level));
  if (!Q) return fail(VI_E_INVAL, "null output");
  if (d < 1 || d > vi::kMaxRed) return fail(VI_E_INVAL, "d must be in [1, 32]");
  if (n_max < 1 || n_max > (1 << 20)) return fail(VI_E_INVAL, "n_max must be in [1, 2^20]");
  if (iters < 0 || iters > 10000) return fail(VI_E_INVAL, "iters must be in [0, 10000]");
  if (c->batch) return fail(VI_E_STATE, "the clip is in a batch");
  // the level's basis buffer is reused: keep a basis in use intact
  Level& lv = c->lv[level];
  int32_t* keep = nullptr;
  if (lv.d.rd > 0) std::swap(keep, lv.redQp);
  const vi_status st = level_pca(c, level, d, n_max, iters, Q, variance);
  if (keep) {
    dfree(c, lv.redQp);
    lv.redQp = keep;
  }
  return st;
}

vi_status vi_set_reduction(vi_ctx* c, int32_t level, const int16_t* Q, int32_t d) {
  VI_TRY(level_ok(c, level));
  if (c->batch) return fail(VI_E_STATE, "the clip is in a batch");
  if (d < 0 || d > vi::kMaxRed) return fail(VI_E_INVAL, "d must be in [0, 32]");
  Level& lv = c->lv[level];
  if (d == 0) {
    VI_TRY(sync(c));
    dfree(c, lv.feat);
    dfree(c, lv.prev);
    lv.feat = nullptr;
    lv.prev = nullptr;
    lv.d.feat = nullptr;
    lv.d.prev = nullptr;
    lv.d.rd = 0;
    lv.red_n = 0;
    return VI_OK;
  }
  if (!Q) return fail(VI_E_INVAL, "null basis");
  const int32_t dim = patch_dim(c->prm);
  const int32_t dp = (d + 3) & ~3;
  // every feature's sum must stay inside int32: sum |Q| * 255 + 128 < 2^31;
  // the device layout pairs the coordinates of each patch row
  const int32_t rows = dim / 25;
  std::vector<uint32_t> qp((size_t)rows * vi::kPairs * dp, 0u);
  for (int k = 0; k < d; ++k) {
    int64_t a = 0;
    for (int i = 0; i < dim; ++i) {
      const int16_t v = Q[(size_t)k * dim + i];
      a += v < 0 ? -(int64_t)v : (int64_t)v;
      const int row = i / 25, cc = i % 25;
      qp[((size_t)row * vi::kPairs + cc / 2) * dp + k] |= (uint32_t)(uint16_t)v << (16 * (cc & 1));
    }
    if (a * 255 + 128 >= (int64_t(1) << 31))
      return fail(VI_E_INVAL, "a basis row whose feature sums could overflow 32 bits");
  }
  if (!lv.redQp) VI_TRY(dalloc(c, &lv.redQp, (size_t)rows * vi::kPairs * vi::kMaxRed));
  VI_TRY(sync(c));  // no queued search reads the old basis any more
  VI_HIP(hipMemcpyAsync(lv.redQp, qp.data(), sizeof(uint32_t) * qp.size(), hipMemcpyHostToDevice,
                        c->st));
  VI_TRY(install_reduction(c, level, d));
  return sync(c);
}

vi_status vi_features(const vi_ctx* c, int32_t level, int32_t d, int32_t* out) {
  VI_TRY(level_ok(c, level));
  if (!out) return fail(VI_E_INVAL, "null output");
  const Level& lv = c->lv[level];
  if (lv.d.rd == 0) return fail(VI_E_STATE, "the level has no reduced patch space");
  if (d != lv.red_n) return fail(VI_E_INVAL, "d is not the level's feature count");
  VI_HIP(hipMemcpy2DAsync(out, sizeof(int32_t) * lv.red_n, lv.feat, sizeof(int32_t) * lv.d.rd,
                          sizeof(int32_t) * lv.red_n, (size_t)lv.d.V, hipMemcpyDeviceToDevice,
                          c->st));
  return VI_OK;
}

vi_status vi_transition(vi_ctx* c, int32_t level) {
  VI_TRY(level_ok(c, level));
  if (level + 1 >= c->L) return fail(VI_E_INVAL, "no coarser level");
  return transition(c, level);
}

vi_status vi_inpaint(vi_ctx* c, uint8_t* out_rgb) {
  if (!c || !out_rgb) return fail(VI_E_INVAL, "null argument");
  VI_TRY(onion(c, nullptr));
  for (int32_t l = c->L - 1; l >= 0; --l) {
    if (l < c->L - 1) VI_TRY(transition(c, l));
    VI_TRY(inpaint_level(c, l, nullptr));
  }
  Level& l0 = c->lv[0];
  if (l0.nH > 0) VI_TRY(recon(c, 0, l0.hlist, l0.nH, nullptr, VI_RECON_BEST, nullptr, nullptr));
  c->phase = 2;
  c->cur_level = 0;
  vi::launch_out_rgb(c->st, l0.d, out_rgb);
  VI_TRY(launched("output"));
  return sync(c);
}

vi_status vi_output(vi_ctx* c, uint8_t* out_rgb) {
  if (!c || !out_rgb) return fail(VI_E_INVAL, "null argument");
  if (c->phase != 2) return fail(VI_E_STATE, "the clip has not finished");
  vi::launch_out_rgb(c->st, c->lv[0].d, out_rgb);
  VI_TRY(launched("output"));
  return sync(c);
}

int32_t vi_done(const vi_ctx* c) { return c && c->phase == 2 ? 1 : 0; }

vi_status vi_get_state(const vi_ctx* c, int32_t level, uint8_t* rgbt, int32_t* cand,
                       int32_t* dist, uint8_t* nvox) {
  VI_TRY(level_ok(c, level));
  vi::launch_get_state(c->st, c->lv[level].d, rgbt, cand, dist, nvox);
  return launched("get_state");
}

vi_status vi_set_state(vi_ctx* c, int32_t level, const uint8_t* rgbt, const int32_t* cand,
                       const int32_t* dist, const uint8_t* nvox) {
  VI_TRY(level_ok(c, level));
  // validate first: a rejected call writes nothing, so the level keeps its
  // previous (consistent) state and completeness
  vi::launch_fill_u64(c->st, c->d_u64 + 1, 2);
  vi::launch_set_state(c->st, c->lv[level].d, rgbt, cand, dist, nvox, c->d_u64 + 1, 0);
  VI_TRY(launched("set_state check"));
  unsigned long long bad[2] = {0, 0};
  VI_HIP(hipMemcpyAsync(bad, c->d_u64 + 1, sizeof(bad), hipMemcpyDeviceToHost, c->st));
  VI_TRY(sync(c));
  if (bad[0]) return fail(VI_E_INVAL, "cand outside [-1, V)");
  c->lv[level].recon_ok = false;
  vi::launch_set_state(c->st, c->lv[level].d, rgbt, cand, dist, nvox, c->d_u64 + 1, 1);
  VI_TRY(launched("set_state"));
  if (cand || nvox) c->lv[level].complete = cand ? bad[1] == 0 : c->lv[level].complete && bad[1] == 0;
  return VI_OK;
}

int64_t vi_nominal_evals(const vi_ctx* c, int32_t level) {
  if (level_ok(c, level) != VI_OK) return -1;
  const Level& lv = c->lv[level];
  return per_target_evals(c->prm, r_max(lv.d)) * (int64_t)lv.nS;
}

vi_status vi_get_counters(vi_ctx* c, vi_counters* out) {
  if (!c || !out) return fail(VI_E_INVAL, "null argument");
  unsigned long long v[4] = {0, 0, 0, 0};
  vi::launch_sum_spread(c->st, c->d_cnt + vi::kCntWords, 4, c->d_u64 + 3);
  VI_TRY(launched("counters"));
  VI_HIP(hipMemcpyAsync(v, c->d_u64 + 3, sizeof(v), hipMemcpyDeviceToHost, c->st));
  VI_TRY(sync(c));
  out->nominal_evals = c->n_nominal;
  out->effective_evals = (int64_t)(v[0] + v[1] + v[2] + v[3]);
  out->searches = c->n_searches;
  out->em_iters = c->n_em;
  out->recon_pixels = c->n_recon;
  out->pass_evals = (int64_t)(v[0] + v[3]);
  out->init_evals = (int64_t)v[1];
  out->onion_evals = (int64_t)v[2];
  out->pass_wide_evals = (int64_t)v[3];
  return VI_OK;
}

vi_status vi_reset_counters(vi_ctx* c) {
  if (!c) return fail(VI_E_INVAL, "null context");
  c->n_nominal = c->n_searches = c->n_em = c->n_recon = 0;
  vi::launch_fill_u64(c->st, c->d_cnt + vi::kCntWords, 4 * vi::kCntWords);
  return launched("fill");
}

vi_status vi_profile(vi_ctx* c, int32_t on) {
  if (!c) return fail(VI_E_INVAL, "null context");
  c->prof_mask = (uint32_t)on;
  return VI_OK;
}

int32_t vi_profile_read(vi_ctx* c, vi_kernel_time* out, int32_t cap) {
  if (!c || (cap > 0 && !out) || cap < 0) return fail(VI_E_INVAL, "bad argument");
  if (sync(c) != VI_OK) return VI_E_HIP;
  const int32_t n = (int32_t)c->recs.size() < cap ? (int32_t)c->recs.size() : cap;
  for (int32_t i = 0; i < n; ++i) {
    const vi_ctx::Rec& r = c->recs[(size_t)i];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->events[(size_t)r.ev], c->events[(size_t)r.ev + 1]) !=
        hipSuccess) {
      (void)hipGetLastError();
      ms = -1.f;
    }
    out[i].kind = r.kind;
    out[i].level = r.level;
    out[i].units = r.units;
    out[i].ms = ms;
    out[i].launches = r.launches;
  }
  c->recs.clear();
  return n;
}

}  // extern "C"

// ===========================================================================
// Batches: many clips advance together, one EM iteration per step.
// ===========================================================================
namespace {

// Alg. 4 driven step by step: after the EM loop of a level stops, transition
// to the next finer level or, at level 0, the final best-patch
// reconstruction.
vi_status drive_finish_level(vi_ctx* c) {
  c->lv[c->cur_level].complete = true;
  if (c->cur_level > 0) {
    VI_TRY(transition(c, c->cur_level - 1));
    c->cur_level -= 1;
    c->em_k = 0;
    return VI_OK;
  }
  Level& l0 = c->lv[0];
  if (l0.nH > 0) VI_TRY(recon(c, 0, l0.hlist, l0.nH, nullptr, VI_RECON_BEST, nullptr, nullptr));
  c->phase = 2;
  return VI_OK;
}

// levels without a hole run no EM iteration
vi_status drive_skip_empty(vi_ctx* c) {
  while (c->phase == 1 && c->lv[c->cur_level].nH == 0) VI_TRY(drive_finish_level(c));
  return VI_OK;
}

bool same_schedule(const vi_params& a, const vi_params& b) {
  if (a.pm_iters != b.pm_iters || a.n_jf != b.n_jf) return false;
  for (int i = 0; i < a.n_jf; ++i)
    if (a.jf_steps[i] != b.jf_steps[i]) return false;
  return true;
}

}  // namespace

struct vi_batch {
  hipStream_t st = nullptr;
  bool own_stream = false;
  std::vector<vi_ctx*> members;
  vi_params sched{};  // propagation schedule shared by all members
  bool have_sched = false;
  int32_t ncu = 0;
  // tile configuration
  int32_t blk = 0, grid_mult = 0;
  bool tuned = false;
  // device job table and chunk maps (capacities fixed at creation so that a
  // captured graph stays valid)
  int32_t cap_jobs = 0, cap_tchunks = 0, cap_pchunks = 0;
  vi::JobDesc* d_jobs = nullptr;
  int32_t* d_tchunk_job = nullptr;
  int32_t* d_pchunk_job = nullptr;
  int32_t* d_counts = nullptr;
  unsigned long long* d_abs = nullptr;
  unsigned long long* d_scratch = nullptr;     // spread counter of the tuner's launches
  unsigned long long* d_abs_spread = nullptr;  // cap_jobs spread |change| counters
  int32_t* d_queue = nullptr;
  std::vector<vi::JobDesc> h_jobs;
  std::vector<int32_t> h_tj, h_pj;
  std::vector<vi_ctx*> job_ctx;
  // pinned staging of the uploads, double-buffered: the host fills one
  // while the copy from the other may still be in flight
  struct Stage {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
  } stage[2];
  int stage_next = 0;
  unsigned long long* h_abs = nullptr;  // pinned, cap_jobs
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t steps_run = 0;
};

namespace {

// the clip leaves the batch once the batch's queued work is done, and gets
// its own stream back
void batch_detach(vi_batch* b, vi_ctx* c) {
  (void)hipStreamSynchronize(b->st);
  for (size_t i = 0; i < b->members.size(); ++i)
    if (b->members[i] == c) {
      b->members.erase(b->members.begin() + (long)i);
      break;
    }
  c->st = c->own_st;
  c->batch = nullptr;
}

void batch_free(vi_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  for (void* p : {(void*)b->d_jobs, (void*)b->d_tchunk_job, (void*)b->d_pchunk_job,
                  (void*)b->d_counts, (void*)b->d_abs, (void*)b->d_scratch, (void*)b->d_queue,
                  (void*)b->d_abs_spread})
    if (p) (void)hipFree(p);
  b->d_queue = nullptr;
  for (auto& st : b->stage) {
    if (st.done) (void)hipEventDestroy(st.done);
    if (st.host) (void)hipHostFree(st.host);
    st.done = nullptr;
    st.host = nullptr;
  }
  if (b->h_abs) (void)hipHostFree(b->h_abs);
  b->h_abs = nullptr;
  b->d_jobs = nullptr;
  b->d_tchunk_job = b->d_pchunk_job = b->d_counts = nullptr;
  b->d_abs = b->d_scratch = b->d_abs_spread = nullptr;
}


// uploads a job table and its chunk maps (chunks of `blk` targets and of
// kPixChunk hole pixels per job)
vi_status batch_upload(vi_batch* b, int blk) {
  b->h_tj.clear();
  b->h_pj.clear();
  for (size_t j = 0; j < b->h_jobs.size(); ++j) {
    vi::JobDesc& J = b->h_jobs[j];
    J.tchunk0 = (int32_t)b->h_tj.size();
    J.pchunk0 = (int32_t)b->h_pj.size();
    const int32_t nt = (J.nS + blk - 1) / blk;
    const int32_t np = (J.nH + vi::kPixChunk - 1) / vi::kPixChunk;
    for (int32_t i = 0; i < nt; ++i) b->h_tj.push_back((int32_t)j);
    for (int32_t i = 0; i < np; ++i) b->h_pj.push_back((int32_t)j);
  }
  if ((int32_t)b->h_jobs.size() > b->cap_jobs)
    return fail(VI_E_BUDGET, "more clips in the EM phase than the batch holds");
  if ((int32_t)b->h_tj.size() > b->cap_tchunks || (int32_t)b->h_pj.size() > b->cap_pchunks)
    return fail(VI_E_BUDGET, "the batch's work lists are full");
  const int32_t counts[4] = {(int32_t)b->h_tj.size(), (int32_t)b->h_pj.size(),
                             (int32_t)b->h_jobs.size(), 0};
  const size_t bj = sizeof(vi::JobDesc) * b->h_jobs.size();
  const size_t bt = sizeof(int32_t) * b->h_tj.size();
  const size_t bp = sizeof(int32_t) * b->h_pj.size();
  const size_t need = sizeof(counts) + bj + bt + bp;
  vi_batch::Stage& sg = b->stage[b->stage_next];
  b->stage_next ^= 1;
  if (sg.done) VI_HIP(hipEventSynchronize(sg.done));  // its previous copies are done
  if (sg.bytes < need) {
    if (sg.host) VI_HIP(hipHostFree(sg.host));
    sg.host = nullptr;
    sg.bytes = 0;
    VI_HIP(hipHostMalloc(&sg.host, need * 2, hipHostMallocDefault));
    sg.bytes = need * 2;
  }
  if (!sg.done) VI_HIP(hipEventCreateWithFlags(&sg.done, hipEventDisableTiming));
  char* h = static_cast<char*>(sg.host);
  std::memcpy(h, counts, sizeof(counts));
  std::memcpy(h + sizeof(counts), b->h_jobs.data(), bj);
  std::memcpy(h + sizeof(counts) + bj, b->h_tj.data(), bt);
  std::memcpy(h + sizeof(counts) + bj + bt, b->h_pj.data(), bp);
  VI_HIP(hipMemcpyAsync(b->d_counts, h, sizeof(counts), hipMemcpyHostToDevice, b->st));
  if (bj) VI_HIP(hipMemcpyAsync(b->d_jobs, h + sizeof(counts), bj, hipMemcpyHostToDevice, b->st));
  if (bt)
    VI_HIP(hipMemcpyAsync(b->d_tchunk_job, h + sizeof(counts) + bj, bt, hipMemcpyHostToDevice,
                          b->st));
  if (bp)
    VI_HIP(hipMemcpyAsync(b->d_pchunk_job, h + sizeof(counts) + bj + bt, bp,
                          hipMemcpyHostToDevice, b->st));
  VI_HIP(hipEventRecord(sg.done, b->st));
  return VI_OK;
}

vi::JobDesc job_for(vi_batch* b, vi_ctx* c, int32_t level, size_t slot, bool scratch_evals) {
  const Level& lv = c->lv[level];
  vi::JobDesc J{};
  J.L = lv.d;
  J.tlist = lv.tlist;
  J.hlist = lv.hlist;
  J.nS = lv.nS;
  J.nH = lv.nH;
  J.recon_mode = c->prm.recon_mode;
  J.recon_skip = lv.recon_ok && lv.recon_last == c->prm.recon_mode ? 1 : 0;
  J.step = (uint64_t)c->em_k;
  J.absdiff = b->d_abs_spread + slot * (size_t)vi::kCntWords;
  J.evals = scratch_evals ? b->d_scratch : c->d_cnt + vi::kCntWords;
  J.evals_init = scratch_evals ? b->d_scratch : c->d_cnt + 2 * (size_t)vi::kCntWords;
  const int32_t rmax = r_max(lv.d);
  for (int k = 0; k <= vi::kMaxPmIters; ++k) J.R[k] = k == 0 ? 0 : rs_radius(c->prm, rmax, k);
  return J;
}

// job table of the members in the EM phase, for a block size
vi_status batch_build(vi_batch* b, int blk, bool scratch_evals) {
  b->h_jobs.clear();
  b->job_ctx.clear();
  for (vi_ctx* c : b->members) {
    if (c->phase != 1) continue;
    b->h_jobs.push_back(job_for(b, c, c->cur_level, b->h_jobs.size(), scratch_evals));
    b->job_ctx.push_back(c);
  }
  return batch_upload(b, blk);
}

vi::BatchArgs batch_args(const vi_batch* b) {
  vi::BatchArgs B{};
  B.jobs = b->d_jobs;
  B.tchunk_job = b->d_tchunk_job;
  B.pchunk_job = b->d_pchunk_job;
  B.counts = b->d_counts;
  B.queue = b->d_queue;
  B.direct = b->grid_mult == 0 ? 1 : 0;
  return B;
}

// the launches of one batched EM iteration: step 0, every propagation pass
// with the random search fused into the last pass of each iteration, the copy
// back when the pass count is odd, and the reconstruction
// grid_mult == 0 selects direct launches, sized to this step's chunk counts
// (not captured in a graph); otherwise persistent launches of a fixed grid.
vi_status batch_enqueue_iteration(vi_batch* b, bool masked = false) {
  const vi::BatchArgs B = batch_args(b);
  const int32_t nt = (int32_t)b->h_tj.size(), np = (int32_t)b->h_pj.size();
  const int32_t grid = B.direct ? (nt > 0 ? nt : 1) : b->ncu * b->grid_mult;
  const int32_t rgrid = B.direct ? (np > 0 ? np : 1) : b->ncu * 8;
  int32_t slot = 0;
  vi::launch_batch_zero(b->st, B, b->cap_jobs);
  vi::launch_batch_s0(b->st, B, b->blk, grid, slot++, masked);
  int parity = 0;
  int32_t t = 0;
  const int32_t njf = b->sched.n_jf;
  for (int k = 1; k <= b->sched.pm_iters; ++k)
    for (int js = 0; js < njf; ++js) {
      ++t;
      vi::launch_batch_pass(b->st, B, b->blk, grid, b->sched.jf_steps[js],
                            js == njf - 1 ? k : 0, parity, slot++, t,
                            t > njf ? t - njf : 0, masked);
      parity ^= 1;
    }
  if (parity) vi::launch_batch_copy(b->st, B, b->blk, grid, slot++);
  vi::launch_batch_recon(b->st, B, rgrid, slot++, masked);
  vi::launch_batch_sum_abs(b->st, B, b->cap_jobs, b->d_abs);
  return launched("batched iteration");
}

// Onion peels (Sec. 3.5, Alg. 3) of clips that start together: layer k of
// every clip is peeled at once.  Each clip's masks and target lists are built
// on the batch's stream, the layer sizes of all clips come back with one
// synchronisation, and the layer's masked searches and reconstructions run as
// one set of batched launches.  Per clip the sequence of operations and the
// random numbers (step 2^32 + layer) are those of vi_onion_init.
vi_status batch_onion(vi_batch* b, std::vector<vi_ctx*> active) {
  // before tuning, the onion runs direct launches of 256-target workgroups
  const int blk = b->blk > 0 ? b->blk : 256;
  const int saved_blk = b->blk, saved_mult = b->grid_mult;
  b->blk = blk;
  if (!b->tuned) b->grid_mult = 0;
  for (vi_ctx* c : active) VI_TRY(onion_prepare(c));
  std::vector<uint8_t*> Hp(active.size()), E(active.size());
  for (size_t i = 0; i < active.size(); ++i) {
    Hp[i] = active[i]->o_Hp;
    E[i] = active[i]->o_E;
  }
  std::vector<int32_t> cnt(2 * active.size());
  for (int32_t layer = 0; !active.empty(); ++layer) {
    for (size_t i = 0; i < active.size(); ++i) {
      vi_ctx* c = active[i];
      const vi::DevLevel& d = c->lv[c->L - 1].d;
      vi::launch_erode3(b->st, Hp[i], E[i], c->o_bd, d.W, d.H, d.T);
      vi::launch_dilate5(b->st, c->o_bd, c->o_S, c->o_t1, c->o_t2, d.W, d.H, d.T, Hp[i]);
      VI_HIP(vi::compact(b->st, c->o_bd, d.V, c->o_pl, c->d_count, c->ctemp, c->ctemp_bytes));
      VI_HIP(vi::compact(b->st, c->o_S, d.V, c->o_tl, c->d_count + 1, c->ctemp, c->ctemp_bytes));
      VI_HIP(hipMemcpyAsync(&cnt[2 * i], c->d_count, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                            b->st));
    }
    VI_TRY(launched("onion layer"));
    VI_HIP(hipStreamSynchronize(b->st));
    std::vector<vi_ctx*> next;
    std::vector<uint8_t*> nH, nE;
    b->h_jobs.clear();
    for (size_t i = 0; i < active.size(); ++i) {
      vi_ctx* c = active[i];
      if (cnt[2 * i] == 0) {  // H' is empty: this clip's peel is finished
        c->lv[c->L - 1].complete = false;
        c->phase = 1;
        c->cur_level = c->L - 1;
        c->em_k = 0;
        continue;
      }
      const int32_t level = c->L - 1;
      vi::JobDesc J = job_for(b, c, level, b->h_jobs.size(), false);
      J.tlist = c->o_tl;
      J.nS = cnt[2 * i + 1];
      J.hlist = c->o_pl;
      J.nH = cnt[2 * i];
      J.smask = c->o_S;
      J.excl = Hp[i];
      J.step = (uint64_t(1) << 32) + (uint64_t)layer;
      J.recon_skip = 0;
      J.evals = c->d_cnt + 3 * (size_t)vi::kCntWords;
      J.evals_init = c->d_cnt + 3 * (size_t)vi::kCntWords;
      c->n_nominal += per_target_evals(c->prm, r_max(c->lv[level].d)) * (int64_t)J.nS;
      c->n_searches += 1;
      c->n_recon += J.nH;
      b->h_jobs.push_back(J);
      next.push_back(c);
      nH.push_back(E[i]);  // H' <- erosion for the next layer
      nE.push_back(Hp[i]);
    }
    if (!b->h_jobs.empty()) {
      VI_TRY(batch_upload(b, blk));
      VI_TRY(batch_enqueue_iteration(b, true));
      for (vi_ctx* c : next) {
        Level& lv = c->lv[c->L - 1];
        next_epoch(lv);
        lv.recon_ok = false;
      }
    }
    active.swap(next);
    Hp.swap(nH);
    E.swap(nE);
  }
  b->blk = saved_blk;
  b->grid_mult = saved_mult;
  return VI_OK;
}

// Times one propagation pass (reading buffer 0, writing buffer 1, which the
// next real pass overwrites before reading) for each candidate tile shape
// and keeps the fastest.  Step 0 is re-run first; it is idempotent for the
// current state and EM index.
vi_status batch_autotune(vi_batch* b) {
  static const int kBlk[3] = {64, 128, 256};
  static const int kMult[4] = {0, 2, 4, 8};  // 0: direct launches
  hipEvent_t e0, e1;
  VI_HIP(hipEventCreate(&e0));
  VI_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bb = 256, bm = 4;
  vi_status st = VI_OK;
  for (int ib = 0; ib < 3 && st == VI_OK; ++ib) {
    if ((st = batch_build(b, kBlk[ib], true)) != VI_OK) break;
    const vi::BatchArgs B = batch_args(b);
    vi::launch_batch_zero(b->st, B, b->cap_jobs);
    // step 0 over every target chunk (direct: one workgroup per chunk)
    vi::BatchArgs B0 = B;
    B0.direct = 1;
    vi::launch_batch_s0(b->st, B0, kBlk[ib], std::max<int32_t>(1, (int32_t)b->h_tj.size()), 0);
    for (int im = 0; im < 4; ++im) {
      vi::BatchArgs Bm = B;
      Bm.direct = kMult[im] == 0 ? 1 : 0;
      const int32_t grid = Bm.direct ? (int32_t)b->h_tj.size() : b->ncu * kMult[im];
      const int32_t s = b->sched.n_jf > 0 ? b->sched.jf_steps[0] : 1;
      if (grid <= 0) continue;
      vi::launch_batch_pass(b->st, Bm, kBlk[ib], grid, s, 1, 0, 1 + 4 * im, 1, 0);
      (void)hipEventRecord(e0, b->st);
      for (int r = 0; r < 3; ++r)
        vi::launch_batch_pass(b->st, Bm, kBlk[ib], grid, s, 1, 0, 2 + 4 * im + r, 1, 0);
      (void)hipEventRecord(e1, b->st);
      if ((st = launched("autotune")) != VI_OK) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = fail(VI_E_HIP, "autotune event");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        bb = kBlk[ib];
        bm = kMult[im];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != VI_OK) return st;
  b->blk = bb;
  b->grid_mult = bm;
  b->tuned = true;
  return VI_OK;
}

}  // namespace

extern "C" {

vi_status vi_batch_create(vi_batch** out, const vi_tune* tune, void* hip_stream) {
  if (!out) return fail(VI_E_INVAL, "null output handle");
  *out = nullptr;
  if (tune && tune->tuned) {
    if (tune->block != 64 && tune->block != 128 && tune->block != 256)
      return fail(VI_E_INVAL, "tune.block must be 64, 128 or 256");
    if (tune->grid_mult < 0 || tune->grid_mult > 64)
      return fail(VI_E_INVAL, "tune.grid_mult must be in [0, 64]");
  }
  vi_batch* b = new (std::nothrow) vi_batch();
  if (!b) return fail(VI_E_NOMEM, "host allocation failed");
  if (hip_stream) {
    b->st = static_cast<hipStream_t>(hip_stream);
  } else {
    // graph capture needs a stream of its own (default priority)
    if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return fail(VI_E_HIP, "stream creation failed");
    }
    b->own_stream = true;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    vi_batch_destroy(b);
    return fail(VI_E_HIP, "device query failed");
  }
  b->ncu = prop.multiProcessorCount;
  if (tune && tune->tuned) {
    b->blk = tune->block;
    b->grid_mult = tune->grid_mult;
    b->tuned = true;
  }
  b->cap_jobs = 1024;
  b->cap_tchunks = 1 << 21;
  b->cap_pchunks = 1 << 21;
  void* p = nullptr;
  auto alloc = [&](size_t bytes) -> void* {
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return q;
  };
  b->d_jobs = static_cast<vi::JobDesc*>(alloc(sizeof(vi::JobDesc) * (size_t)b->cap_jobs));
  b->d_tchunk_job = static_cast<int32_t*>(alloc(sizeof(int32_t) * (size_t)b->cap_tchunks));
  b->d_pchunk_job = static_cast<int32_t*>(alloc(sizeof(int32_t) * (size_t)b->cap_pchunks));
  b->d_counts = static_cast<int32_t*>(alloc(sizeof(int32_t) * 4));
  if (hipHostMalloc((void**)&b->h_abs, sizeof(unsigned long long) * b->cap_jobs,
                    hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    b->h_abs = nullptr;
  }
  b->d_abs = static_cast<unsigned long long*>(alloc(sizeof(unsigned long long) * b->cap_jobs));
  b->d_scratch = static_cast<unsigned long long*>(alloc(sizeof(unsigned long long) * vi::kCntWords));
  b->d_abs_spread = static_cast<unsigned long long*>(
      alloc(sizeof(unsigned long long) * vi::kCntWords * (size_t)b->cap_jobs));
  b->d_queue = static_cast<int32_t*>(alloc(sizeof(int32_t) * vi::kQueueSlots));
  (void)p;
  if (!b->d_jobs || !b->d_tchunk_job || !b->d_pchunk_job || !b->d_counts || !b->d_abs ||
      !b->d_scratch || !b->d_queue || !b->h_abs || !b->d_abs_spread) {
    vi_batch_destroy(b);
    return fail(VI_E_NOMEM, "batch allocation failed");
  }
  const int32_t zero[4] = {0, 0, 0, 0};
  if (hipMemcpy(b->d_counts, zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) {
    vi_batch_destroy(b);
    return fail(VI_E_HIP, "batch initialisation failed");
  }
  *out = b;
  return VI_OK;
}

void vi_batch_destroy(vi_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->st);
  // members outlive the batch: they go back to their own streams
  for (vi_ctx* c : b->members) {
    c->st = c->own_st;
    c->batch = nullptr;
  }
  b->members.clear();
  batch_free(b);
  if (b->own_stream) (void)hipStreamDestroy(b->st);
  delete b;
}

vi_status vi_batch_add(vi_batch* b, vi_ctx* c) {
  if (!b || !c) return fail(VI_E_INVAL, "null argument");
  if (c->batch == b) return fail(VI_E_INVAL, "the clip is already in the batch");
  if (c->batch) return fail(VI_E_INVAL, "the clip is in another batch");
  if (c->prm.n_jf < 1) return fail(VI_E_INVAL, "batched clips need at least one propagation step");
  if (b->have_sched && !same_schedule(b->sched, c->prm))
    return fail(VI_E_INVAL, "all clips of a batch share pm_iters and jf_steps");
  if ((int32_t)b->members.size() >= b->cap_jobs) return fail(VI_E_BUDGET, "the batch is full");
  if (c->phase == 2) return fail(VI_E_STATE, "the clip has already finished");
  for (int l = 0; l < c->L; ++l)
    if (c->lv[l].d.rd > 0)
      return fail(VI_E_INVAL, "clips searched with the reduced distance run alone");
  if (!b->have_sched) {
    b->sched = c->prm;
    b->have_sched = true;
  }
  // the clip's work is ordered on the batch's stream from now on
  (void)hipStreamSynchronize(c->st);
  c->own_st = c->st;
  c->st = b->st;
  c->batch = b;
  b->members.push_back(c);
  return VI_OK;
}

vi_status vi_batch_remove(vi_batch* b, vi_ctx* c) {
  if (!b || !c) return fail(VI_E_INVAL, "null argument");
  if (c->batch != b) return fail(VI_E_INVAL, "the clip is not in the batch");
  batch_detach(b, c);
  return VI_OK;
}

int32_t vi_batch_size(const vi_batch* b) { return b ? (int32_t)b->members.size() : 0; }

vi_status vi_batch_get_tune(const vi_batch* b, vi_tune* out) {
  if (!b || !out) return fail(VI_E_INVAL, "null argument");
  out->block = b->blk;
  out->grid_mult = b->grid_mult;
  out->tuned = b->tuned ? 1 : 0;
  return VI_OK;
}

vi_status vi_batch_step(vi_batch* b, int32_t* n_done) {
  if (!b) return fail(VI_E_INVAL, "null batch");
  if (n_done) *n_done = 0;
  int32_t done = 0;
  // clips that have not started: onion peels of their coarsest levels,
  // layer by layer for all of them together
  std::vector<vi_ctx*> fresh;
  for (vi_ctx* c : b->members)
    if (c->phase == 0) fresh.push_back(c);
  if (fresh.size() == 1) {
    // one clip alone runs the single-clip launches: the same per-target
    // code and random numbers, without job tables
    vi_ctx* c = fresh[0];
    VI_TRY(onion(c, nullptr));
    c->phase = 1;
    c->cur_level = c->L - 1;
    c->em_k = 0;
  } else if (!fresh.empty()) {
    VI_TRY(batch_onion(b, fresh));
  }
  for (vi_ctx* c : b->members) VI_TRY(drive_skip_empty(c));
  bool any = false;
  vi_ctx* lone = nullptr;
  int32_t n_em = 0;
  for (vi_ctx* c : b->members)
    if (c->phase == 1) {
      any = true;
      lone = c;
      ++n_em;
    }
  if (n_em == 1) {
    // one EM iteration of the only clip in its EM phase, as vi_inpaint_level
    vi_ctx* c = lone;
    const int32_t level = c->cur_level;
    Level& lv = c->lv[level];
    VI_TRY(search(c, level, lv.tlist, lv.nS, lv.d.htil, nullptr, (uint64_t)c->em_k));
    VI_TRY(recon(c, level, lv.hlist, lv.nH, nullptr, c->prm.recon_mode, nullptr, c->d_u64));
    ++b->steps_run;
    c->n_em += 1;
    c->em_k += 1;
    double e = INFINITY;
    if (c->prm.em_tol >= 0) {
      unsigned long long s = 0;
      VI_HIP(hipMemcpyAsync(&s, c->d_u64, sizeof(s), hipMemcpyDeviceToHost, b->st));
      VI_HIP(hipStreamSynchronize(b->st));
      e = (double)s / (3.0 * (double)lv.nH);
    }
    if (!(e > c->prm.em_tol && c->em_k < c->prm.em_max_iters)) {
      VI_TRY(drive_finish_level(c));
      VI_TRY(drive_skip_empty(c));
    }
    any = false;
  }
  if (any) {
    if (!b->tuned) VI_TRY(batch_autotune(b));
    VI_TRY(batch_build(b, b->blk, false));
    if (b->grid_mult == 0) {
      VI_TRY(batch_enqueue_iteration(b));
    } else if (!b->exec) {
      VI_HIP(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
      const vi_status cs = batch_enqueue_iteration(b);
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(b->st, &g);
      if (cs != VI_OK) return cs;
      if (ce != hipSuccess) return fail(VI_E_HIP, std::string("graph capture failed: ") +
                                                      hipGetErrorString(ce));
      b->graph = g;
      VI_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    if (b->grid_mult != 0) VI_HIP(hipGraphLaunch(b->exec, b->st));
    const size_t nj = b->h_jobs.size();
    // the stopping test needs this step's |change| sums; clips with a fixed
    // number of iterations (em_tol < 0) need no read-back
    bool need_abs = false;
    for (size_t j = 0; j < nj; ++j) need_abs = need_abs || b->job_ctx[j]->prm.em_tol >= 0;
    if (need_abs) {
      VI_HIP(hipMemcpyAsync(b->h_abs, b->d_abs, sizeof(unsigned long long) * nj,
                            hipMemcpyDeviceToHost, b->st));
      VI_HIP(hipStreamSynchronize(b->st));
    }
    ++b->steps_run;
    for (size_t j = 0; j < nj; ++j) {
      vi_ctx* c = b->job_ctx[j];
      Level& lv = c->lv[c->cur_level];
      next_epoch(lv);  // this step's full reconstruction of the level
      lv.recon_ok = true;
      lv.recon_last = c->prm.recon_mode;
      c->n_nominal += per_target_evals(c->prm, r_max(lv.d)) * (int64_t)lv.nS;
      c->n_searches += 1;
      c->n_em += 1;
      c->n_recon += lv.nH;
      c->em_k += 1;
      const double e = c->prm.em_tol >= 0 ? (double)b->h_abs[j] / (3.0 * (double)lv.nH) : INFINITY;
      if (!(e > c->prm.em_tol && c->em_k < c->prm.em_max_iters)) {
        VI_TRY(drive_finish_level(c));
        VI_TRY(drive_skip_empty(c));
      }
    }
  }
  for (vi_ctx* c : b->members) done += c->phase == 2 ? 1 : 0;
  VI_TRY(launched("batch step"));
  if (n_done) *n_done = done;
  return VI_OK;
}

}  // extern "C"
