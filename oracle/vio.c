/* vio.c -- CPU oracle (test infrastructure only; see vio.h).
 *
 * Plain loops, no blocking or fusion.  OpenMP is used only over independent
 * targets or pixels: every propagation pass reads the state from before the
 * pass (Jacobi), so results do not depend on the thread count.
 *
 * Paper anchors (Newson et al., "Video Inpainting of Complex Scenes"):
 *   Sec. 2, Eq. (2.1)-(2.2)  energy and patch distance
 *   Sec. 3.1, Alg. 1, Eq. (3.1)  ANN search: init, propagation, random search
 *   Sec. 3.2, Eqs. (3.2)-(3.4)   weighted-mean and best-patch reconstruction
 *   Sec. 3.3, Eqs. (3.5)-(3.8)   texture features, texture pyramid and their
 *                                 reconstruction
 *   Sec. 3.5, Eqs. (3.9)-(3.11), Alg. 3  onion-peel initialisation with the
 *                                 partial distance
 *   Sec. 3.6   no temporal subsampling, NN upsampling of the shift map
 *   Sec. 3.7, Alg. 4  stopping criterion, parameters, complete algorithm
 */
#include "vio.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int32_t W, H, T;
  int64_t V;
  uint8_t* rgbt;   /* [V][5] R,G,B,Tx,Ty */
  uint8_t* hole;   /* H^l */
  uint8_t* dsrc;   /* D~^l */
  uint8_t* htil;   /* H~^l */
  int64_t* dlist;  /* D~^l in ascending linear order */
  int64_t nD;
  int64_t nH, nHt;
  int32_t* cand;
  int32_t* dist;
  uint8_t* nvox;
  int searched;    /* a shift map exists on H~^l */
  /* dimensionality-reduced distance (Sec. 5): basis and voxel features */
  int32_t red_d;   /* 0: the exact distance */
  int16_t* redQ;   /* [red_d][5 x patch voxels] */
  int32_t* feat;   /* [V][red_d] */
} level_t;

struct vio_ctx {
  vio_params prm;
  int32_t L;
  level_t lv[16];
};

int vio_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int vio_params_default(vio_params* o) {
  if (!o) return VIO_E_INVAL;
  memset(o, 0, sizeof(*o));
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
  o->recon_mode = VIO_RECON_WEIGHTED;
  o->seed = 0;
  o->temporal_subsample = 0;
  return VIO_OK;
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 64x64->128 multiplications,   */
/* a fixed word permutation and a Weyl-sequence key schedule.               */
/* ------------------------------------------------------------------------ */
void vio_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* uniform integer in [0, n) from the high 32 bits of a 64-bit word */
static int64_t draw_below(uint64_t w, int64_t n) {
  return (int64_t)(((w >> 32) * (uint64_t)n) >> 32);
}

int64_t vio_draw_below(uint64_t w, int64_t n) { return n > 0 ? draw_below(w, n) : -1; }

/* ------------------------------------------------------------------------ */
/* helpers                                                                  */
/* ------------------------------------------------------------------------ */
static void unlin(const level_t* L, int64_t i, int32_t* x, int32_t* y, int32_t* t) {
  *x = (int32_t)(i % L->W);
  *y = (int32_t)((i / L->W) % L->H);
  *t = (int32_t)(i / ((int64_t)L->W * L->H));
}
static int64_t lin(const level_t* L, int64_t x, int64_t y, int64_t t) {
  return (t * L->H + y) * L->W + x;
}
static int inside(const level_t* L, int64_t x, int64_t y, int64_t t) {
  return x >= 0 && y >= 0 && t >= 0 && x < L->W && y < L->H && t < L->T;
}

static void free_level(level_t* L) {
  free(L->rgbt); free(L->hole); free(L->dsrc); free(L->htil); free(L->dlist);
  free(L->cand); free(L->dist); free(L->nvox);
  free(L->redQ); free(L->feat);
  memset(L, 0, sizeof(*L));
}

void vio_destroy(vio_ctx* ctx) {
  if (!ctx) return;
  for (int l = 0; l < 16; ++l) free_level(&ctx->lv[l]);
  free(ctx);
}

/* ------------------------------------------------------------------------ */
/* Sets (Sec. 2): D~ = {p in D : N_p in D} restricted to centres whose whole */
/* patch lies in the volume; H~ = union of N_p over the hole, in the volume. */
/* ------------------------------------------------------------------------ */
static int build_sets(vio_ctx* ctx, level_t* L) {
  const int hx = ctx->prm.patch[0] / 2, hy = ctx->prm.patch[1] / 2, ht = ctx->prm.patch[2] / 2;
  int64_t nD = 0, nH = 0, nHt = 0;
#pragma omp parallel for schedule(static) reduction(+ : nD, nH, nHt)
  for (int32_t t = 0; t < L->T; ++t)
    for (int32_t y = 0; y < L->H; ++y)
      for (int32_t x = 0; x < L->W; ++x) {
        int64_t i = lin(L, x, y, t);
        int ok = x >= hx && y >= hy && t >= ht && x < L->W - hx && y < L->H - hy && t < L->T - ht;
        int near_hole = 0;
        for (int dt = -ht; dt <= ht; ++dt)
          for (int dy = -hy; dy <= hy; ++dy)
            for (int dx = -hx; dx <= hx; ++dx) {
              if (!inside(L, x + dx, y + dy, t + dt)) continue;
              if (L->hole[lin(L, x + dx, y + dy, t + dt)]) near_hole = 1;
            }
        L->dsrc[i] = (uint8_t)(ok && !near_hole);
        L->htil[i] = (uint8_t)near_hole; /* the box is symmetric: q in N_p <=> p in N_q */
        nD += L->dsrc[i];
        nH += L->hole[i];
        nHt += L->htil[i];
      }
  L->nD = nD;
  L->nH = nH;
  L->nHt = nHt;
  L->dlist = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nD > 0 ? nD : 1));
  if (!L->dlist) return VIO_E_NOMEM;
  int64_t k = 0;
  for (int64_t i = 0; i < L->V; ++i)
    if (L->dsrc[i]) L->dlist[k++] = i;
  return VIO_OK;
}

static int alloc_level(level_t* L, int32_t W, int32_t H, int32_t T) {
  L->W = W; L->H = H; L->T = T;
  L->V = (int64_t)W * H * T;
  size_t V = (size_t)L->V;
  L->rgbt = (uint8_t*)calloc(V * 5, 1);
  L->hole = (uint8_t*)calloc(V, 1);
  L->dsrc = (uint8_t*)calloc(V, 1);
  L->htil = (uint8_t*)calloc(V, 1);
  L->cand = (int32_t*)malloc(V * sizeof(int32_t));
  L->dist = (int32_t*)malloc(V * sizeof(int32_t));
  L->nvox = (uint8_t*)calloc(V, 1);
  if (!L->rgbt || !L->hole || !L->dsrc || !L->htil || !L->cand || !L->dist || !L->nvox)
    return VIO_E_NOMEM;
  for (size_t i = 0; i < V; ++i) { L->cand[i] = -1; L->dist[i] = -1; }
  return VIO_OK;
}

/* ------------------------------------------------------------------------ */
/* Pyramids (Alg. 4 first lines; Sec. 3.3 Eqs. (3.5), (3.7); Sec. 3.6).     */
/* Image pyramid: 2x2 spatial box mean rounded half up, no temporal         */
/* subsampling (2x2x2 blocks and T^l(x,y,t) = T(2^l x, 2^l y, 2^l t) when   */
/* temporal_subsample is set).  Occlusion pyramid: OR over the 2x2 block.  Texture T at    */
/* the finest level: mean over the square nu (side 2^(L-1), anchored at the */
/* pixel) of |grey(x+1)-grey(x-1)| resp. along y, with grey = (R+G+B)/3,     */
/* known pixels only; coarser levels subsample it: T^l(x,y,t)=T(2^l x,2^l y,t). */
/* ------------------------------------------------------------------------ */
static void texture_finest(vio_ctx* ctx, const uint8_t* rgb, const uint8_t* mask,
                           uint8_t* Tx, uint8_t* Ty) {
  level_t* L = &ctx->lv[0];
  const int32_t W = L->W, H = L->H, T = L->T;
  const int32_t s = 1 << (ctx->L - 1);
  int32_t* gx = (int32_t*)malloc(sizeof(int32_t) * (size_t)L->V); /* -1 = undefined */
  int32_t* gy = (int32_t*)malloc(sizeof(int32_t) * (size_t)L->V);
#pragma omp parallel for schedule(static)
  for (int32_t t = 0; t < T; ++t)
    for (int32_t y = 0; y < H; ++y)
      for (int32_t x = 0; x < W; ++x) {
        int64_t i = lin(L, x, y, t);
        gx[i] = -1;
        gy[i] = -1;
        if (x - 1 >= 0 && x + 1 < W) {
          int64_t a = lin(L, x - 1, y, t), b = lin(L, x + 1, y, t);
          if (!mask[a] && !mask[b]) {
            int ga = rgb[3 * a] + rgb[3 * a + 1] + rgb[3 * a + 2];
            int gb = rgb[3 * b] + rgb[3 * b + 1] + rgb[3 * b + 2];
            gx[i] = abs(gb - ga);
          }
        }
        if (y - 1 >= 0 && y + 1 < H) {
          int64_t a = lin(L, x, y - 1, t), b = lin(L, x, y + 1, t);
          if (!mask[a] && !mask[b]) {
            int ga = rgb[3 * a] + rgb[3 * a + 1] + rgb[3 * a + 2];
            int gb = rgb[3 * b] + rgb[3 * b + 1] + rgb[3 * b + 2];
            gy[i] = abs(gb - ga);
          }
        }
      }
#pragma omp parallel for schedule(static)
  for (int32_t t = 0; t < T; ++t)
    for (int32_t y = 0; y < H; ++y)
      for (int32_t x = 0; x < W; ++x) {
        int64_t sx = 0, cx = 0, sy = 0, cy = 0;
        for (int32_t yy = y; yy < y + s && yy < H; ++yy)
          for (int32_t xx = x; xx < x + s && xx < W; ++xx) {
            int64_t j = lin(L, xx, yy, t);
            if (gx[j] >= 0) { sx += gx[j]; cx++; }
            if (gy[j] >= 0) { sy += gy[j]; cy++; }
          }
        /* round half up of the mean of |grey difference| = S/(3c) */
        int64_t i = lin(L, x, y, t);
        Tx[i] = (uint8_t)(cx ? (2 * sx + 3 * cx) / (6 * cx) : 0);
        Ty[i] = (uint8_t)(cy ? (2 * sy + 3 * cy) / (6 * cy) : 0);
      }
  free(gx);
  free(gy);
}

int vio_create(vio_ctx** out, const vio_params* prm, int32_t W, int32_t H, int32_t T,
               const uint8_t* rgb, const uint8_t* mask) {
  if (!out || !prm || !rgb || !mask) return VIO_E_INVAL;
  *out = NULL;
  if (prm->levels < 1 || prm->levels > 16) return VIO_E_INVAL;
  for (int a = 0; a < 3; ++a)
    if (prm->patch[a] < 1 || prm->patch[a] % 2 == 0) return VIO_E_INVAL;
  if (prm->patch[0] * prm->patch[1] * prm->patch[2] > 1024) return VIO_E_INVAL;
  if (prm->n_jf < 0 || prm->n_jf > 8 || prm->pm_iters < 0 || prm->lambda < 0) return VIO_E_INVAL;
  if (prm->recon_mode != VIO_RECON_WEIGHTED && prm->recon_mode != VIO_RECON_MEAN)
    return VIO_E_INVAL;
  if (prm->temporal_subsample != 0 && prm->temporal_subsample != 1) return VIO_E_INVAL;
  vio_ctx* ctx = (vio_ctx*)calloc(1, sizeof(vio_ctx));
  if (!ctx) return VIO_E_NOMEM;
  ctx->prm = *prm;
  ctx->L = prm->levels;
  const int ts = prm->temporal_subsample;
  int32_t w = W, h = H, tl = T;
  for (int l = 0; l < ctx->L; ++l) {
    if (w < prm->patch[0] || h < prm->patch[1] || tl < prm->patch[2]) {
      vio_destroy(ctx);
      return VIO_E_INVAL;
    }
    if (alloc_level(&ctx->lv[l], w, h, tl) != VIO_OK) {
      vio_destroy(ctx);
      return VIO_E_NOMEM;
    }
    w = (w + 1) / 2;
    h = (h + 1) / 2;
    if (ts) tl = (tl + 1) / 2;
  }
  /* level 0: the input, zero under the hole (those values are never read) */
  level_t* L0 = &ctx->lv[0];
  for (int64_t i = 0; i < L0->V; ++i) {
    L0->hole[i] = mask[i] ? 1 : 0;
    for (int c = 0; c < 3; ++c) L0->rgbt[5 * i + c] = L0->hole[i] ? 0 : rgb[3 * i + c];
  }
  /* image and occlusion pyramids */
  for (int l = 1; l < ctx->L; ++l) {
    level_t* F = &ctx->lv[l - 1];
    level_t* C = &ctx->lv[l];
#pragma omp parallel for schedule(static)
    for (int32_t t = 0; t < C->T; ++t)
      for (int32_t y = 0; y < C->H; ++y)
        for (int32_t x = 0; x < C->W; ++x) {
          int64_t i = lin(C, x, y, t);
          int any = 0, cnt = 0;
          int sum[3] = {0, 0, 0};
          /* the in-volume 2x2 block (2x2x2 with temporal subsampling) */
          for (int bt = 0; bt < (ts ? 2 : 1); ++bt)
            for (int by = 0; by < 2; ++by)
              for (int bx = 0; bx < 2; ++bx) {
                int32_t fx = 2 * x + bx, fy = 2 * y + by, ft = ts ? 2 * t + bt : t;
                if (fx >= F->W || fy >= F->H || ft >= F->T) continue;
                int64_t j = lin(F, fx, fy, ft);
                any |= F->hole[j];
                cnt++;
                for (int c = 0; c < 3; ++c) sum[c] += F->rgbt[5 * j + c];
              }
          C->hole[i] = (uint8_t)any;
          for (int c = 0; c < 3; ++c)
            C->rgbt[5 * i + c] = (uint8_t)(any ? 0 : (sum[c] + cnt / 2) / cnt);
        }
  }
  /* texture features and their pyramid */
  uint8_t* Tx = (uint8_t*)malloc((size_t)L0->V);
  uint8_t* Ty = (uint8_t*)malloc((size_t)L0->V);
  if (!Tx || !Ty) {
    free(Tx); free(Ty);
    vio_destroy(ctx);
    return VIO_E_NOMEM;
  }
  texture_finest(ctx, rgb, L0->hole, Tx, Ty);
  for (int l = 0; l < ctx->L; ++l) {
    level_t* C = &ctx->lv[l];
    for (int32_t t = 0; t < C->T; ++t)
      for (int32_t y = 0; y < C->H; ++y)
        for (int32_t x = 0; x < C->W; ++x) {
          int64_t i = lin(C, x, y, t);
          int64_t j = lin(L0, (int64_t)x << l, (int64_t)y << l, ts ? (int64_t)t << l : t);
          C->rgbt[5 * i + 3] = C->hole[i] ? 0 : Tx[j];
          C->rgbt[5 * i + 4] = C->hole[i] ? 0 : Ty[j];
        }
  }
  free(Tx);
  free(Ty);
  for (int l = 0; l < ctx->L; ++l) {
    int st = build_sets(ctx, &ctx->lv[l]);
    if (st != VIO_OK) {
      vio_destroy(ctx);
      return st;
    }
    if (ctx->lv[l].nD == 0) {
      vio_destroy(ctx);
      return VIO_E_EMPTY_SOURCE;
    }
  }
  *out = ctx;
  return VIO_OK;
}

int vio_level_info(const vio_ctx* ctx, int32_t level, int32_t dims[3], int64_t counts[3]) {
  if (!ctx || level < 0 || level >= ctx->L) return VIO_E_INVAL;
  const level_t* L = &ctx->lv[level];
  if (dims) { dims[0] = L->W; dims[1] = L->H; dims[2] = L->T; }
  if (counts) { counts[0] = L->nH; counts[1] = L->nHt; counts[2] = L->nD; }
  return VIO_OK;
}

int vio_level_sets(const vio_ctx* ctx, int32_t level, uint8_t* hole, uint8_t* dsrc,
                   uint8_t* htil) {
  if (!ctx || level < 0 || level >= ctx->L) return VIO_E_INVAL;
  const level_t* L = &ctx->lv[level];
  if (hole) memcpy(hole, L->hole, (size_t)L->V);
  if (dsrc) memcpy(dsrc, L->dsrc, (size_t)L->V);
  if (htil) memcpy(htil, L->htil, (size_t)L->V);
  return VIO_OK;
}

int vio_get_state(const vio_ctx* ctx, int32_t level, uint8_t* rgbt, int32_t* cand,
                  int32_t* dist, uint8_t* nvox) {
  if (!ctx || level < 0 || level >= ctx->L) return VIO_E_INVAL;
  const level_t* L = &ctx->lv[level];
  if (rgbt) memcpy(rgbt, L->rgbt, (size_t)L->V * 5);
  if (cand) memcpy(cand, L->cand, (size_t)L->V * sizeof(int32_t));
  if (dist) memcpy(dist, L->dist, (size_t)L->V * sizeof(int32_t));
  if (nvox) memcpy(nvox, L->nvox, (size_t)L->V);
  return VIO_OK;
}

int vio_set_state(vio_ctx* ctx, int32_t level, const uint8_t* rgbt, const int32_t* cand,
                  const int32_t* dist, const uint8_t* nvox) {
  if (!ctx || level < 0 || level >= ctx->L) return VIO_E_INVAL;
  level_t* L = &ctx->lv[level];
  if (rgbt) {
    /* only hole voxels are state; known voxels stay the input */
    for (int64_t i = 0; i < L->V; ++i)
      if (L->hole[i]) memcpy(&L->rgbt[5 * i], &rgbt[5 * i], 5);
  }
  if (cand) {
    for (int64_t i = 0; i < L->V; ++i)
      if (cand[i] < -1 || cand[i] >= L->V) return VIO_E_INVAL;
    /* the map is complete when every target holds a source of D~ */
    int complete = 1;
    for (int64_t i = 0; i < L->V; ++i) {
      L->cand[i] = L->htil[i] ? cand[i] : -1;
      if (L->htil[i] && (cand[i] < 0 || !L->dsrc[cand[i]])) complete = 0;
    }
    L->searched = complete;
  }
  if (dist)
    for (int64_t i = 0; i < L->V; ++i) L->dist[i] = L->htil[i] ? dist[i] : -1;
  if (nvox)
    for (int64_t i = 0; i < L->V; ++i) L->nvox[i] = L->htil[i] ? nvox[i] : 0;
  return VIO_OK;
}

/* ------------------------------------------------------------------------ */
/* Patch distance (Sec. 2, Eq. (2.2); Sec. 3.3 texture-augmented form;      */
/* Sec. 3.5 partial form).  Integer SSD over the compared voxels, without   */
/* the 1/N normalisation, which is carried separately as n (the number of   */
/* compared voxels).  Voxels p+o outside the volume are not compared.       */
/* ------------------------------------------------------------------------ */
static int64_t ssd(const vio_ctx* ctx, const level_t* L, int64_t p, int64_t c,
                   const uint8_t* count_mask, int32_t* n_out) {
  const int hx = ctx->prm.patch[0] / 2, hy = ctx->prm.patch[1] / 2, ht = ctx->prm.patch[2] / 2;
  const int64_t lambda = ctx->prm.lambda;
  int32_t px, py, pt, cx, cy, ct;
  unlin(L, p, &px, &py, &pt);
  unlin(L, c, &cx, &cy, &ct);
  int64_t sum = 0;
  int32_t n = 0;
  for (int dt = -ht; dt <= ht; ++dt)
    for (int dy = -hy; dy <= hy; ++dy)
      for (int dx = -hx; dx <= hx; ++dx) {
        if (!inside(L, px + dx, py + dy, pt + dt)) continue;
        int64_t a = lin(L, px + dx, py + dy, pt + dt);
        if (count_mask && !count_mask[a]) continue;
        int64_t b = lin(L, cx + dx, cy + dy, ct + dt);
        const uint8_t* ua = &L->rgbt[5 * a];
        const uint8_t* ub = &L->rgbt[5 * b];
        int64_t col = 0, tex = 0;
        for (int ch = 0; ch < 3; ++ch) col += (int64_t)(ua[ch] - ub[ch]) * (ua[ch] - ub[ch]);
        for (int ch = 3; ch < 5; ++ch) tex += (int64_t)(ua[ch] - ub[ch]) * (ua[ch] - ub[ch]);
        sum += col + lambda * tex;
        n++;
      }
  if (n_out) *n_out = n;
  return sum;
}

int64_t vio_patch_ssd(const vio_ctx* ctx, int32_t level, int64_t p, int64_t c,
                      const uint8_t* count_mask, int32_t* n_out) {
  if (!ctx || level < 0 || level >= ctx->L) return -1;
  const level_t* L = &ctx->lv[level];
  if (p < 0 || p >= L->V || c < 0 || c >= L->V || !L->dsrc[c]) return -1;
  return ssd(ctx, L, p, c, count_mask, n_out);
}

/* ------------------------------------------------------------------------ */
/* Dimensionality-reduced patch space (Sec. 5 suggests it as an             */
/* acceleration; the construction is this implementation's reading).        */
/*                                                                          */
/* The patch vector x(p) lists, for the offsets o in the order dt, dy, dx,  */
/* the channels R, G, B, Tx, Ty of the voxel p + o, its coordinates clamped */
/* to the volume.  With w = 1 on colour and sqrt(lambda) on texture, the    */
/* squared distance of the weighted vectors w x is the patch distance.  A   */
/* basis Q [d][dim] of integers (a linear map scaled by 256) gives the      */
/* features f_k(p) = floor((sum_i Q[k][i] x_i(p) + 128) / 256), and the     */
/* reduced distance of p and c is sum_k (f_k(p) - f_k(c))^2, saturated at   */
/* 2^31 - 1.                                                                */
/* ------------------------------------------------------------------------ */
static int64_t clampi(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

static void features_of(const vio_ctx* ctx, const level_t* L, int64_t p, int32_t* f) {
  const int hx = ctx->prm.patch[0] / 2, hy = ctx->prm.patch[1] / 2, ht = ctx->prm.patch[2] / 2;
  const int dim = 5 * ctx->prm.patch[0] * ctx->prm.patch[1] * ctx->prm.patch[2];
  int32_t px, py, pt;
  unlin(L, p, &px, &py, &pt);
  for (int k = 0; k < L->red_d; ++k) {
    const int16_t* q = L->redQ + (int64_t)k * dim;
    int64_t acc = 0;
    int i = 0;
    for (int dt = -ht; dt <= ht; ++dt)
      for (int dy = -hy; dy <= hy; ++dy)
        for (int dx = -hx; dx <= hx; ++dx) {
          const int64_t a = lin(L, clampi(px + dx, 0, L->W - 1), clampi(py + dy, 0, L->H - 1),
                                clampi(pt + dt, 0, L->T - 1));
          for (int ch = 0; ch < 5; ++ch, ++i) acc += (int64_t)q[i] * L->rgbt[5 * a + ch];
        }
    /* floor division by 256 of acc + 128 */
    const int64_t v = acc + 128;
    f[k] = (int32_t)(v >= 0 ? v / 256 : -((-v + 255) / 256));
  }
}

static int64_t red_dist(const level_t* L, int64_t p, int64_t c) {
  const int32_t* a = L->feat + p * L->red_d;
  const int32_t* b = L->feat + c * L->red_d;
  int64_t s = 0;
  for (int k = 0; k < L->red_d; ++k) {
    const int64_t e = (int64_t)a[k] - b[k];
    s += e * e;
    if (s > 2147483647) return 2147483647;
  }
  return s;
}

/* the distance a search compares: reduced when the level has a basis and
   the search is the unmasked one of the EM loop, else the exact one */
static int64_t search_dist(const vio_ctx* ctx, const level_t* L, int red, int64_t p, int64_t c,
                           const uint8_t* cmask, int32_t* n_out) {
  if (red) return red_dist(L, p, c);
  return ssd(ctx, L, p, c, cmask, n_out);
}

/* ------------------------------------------------------------------------ */
/* ANN search (Sec. 3.1, Alg. 1), made synchronous.                         */
/*                                                                          */
/* Random numbers: Philox4x64-10 with key (seed, 0) and counter             */
/* (lin(p), step, k, (level << 8) | purpose); purpose 1 = initialisation,    */
/* 0 = random search; k = PatchMatch iteration (0 for initialisation).       */
/*                                                                          */
/* Step 0: targets with no valid match get a uniformly random source from   */
/*   D~; every target's distance is re-evaluated (u changed since).         */
/* Each iteration k = 1..K:                                                 */
/*   propagation, for each step s: candidates are the incumbent (index 0)   */
/*   and, for the six axial neighbours q = p -/+ s e_x, e_y, e_t (indices   */
/*   1..6) that are targets, the neighbour's shift applied at p; only       */
/*   candidates in D~ are taken; the new match minimises (SSD, index);      */
/*   all reads are from the state before the pass;                          */
/*   random search: one candidate drawn uniformly in the window of radius   */
/*   floor(r_max rho^k) around the current match (clipped to the centres   */
/*   whose patch fits the volume), r_max = largest dimension of the level;  */
/*   adopted if it is in D~ and strictly better.                            */
/* ------------------------------------------------------------------------ */
/* Random-search radius of PatchMatch iteration k (Eq. (3.1)):
 * floor(r_max rho^k), rho^k formed by k successive multiplications. */
static int64_t rs_radius(const vio_params* P, int32_t r_max, int k) {
  double r = (double)r_max;
  for (int i = 0; i < k; ++i) r *= P->rho;
  return (int64_t)floor(r);
}

/* The random-search candidate of target p around its match c0 (Eq. (3.1)):
 * per axis the window [c0 - R, c0 + R] clipped to the centres whose whole
 * patch lies in the volume, and one uniform integer drawn in it from the
 * high half of Philox word x, y, t respectively. */
static int64_t rs_candidate(const vio_ctx* ctx, int32_t level, int64_t p, int64_t c0lin,
                            int64_t R, uint64_t step, int k) {
  const level_t* L = &ctx->lv[level];
  const vio_params* P = &ctx->prm;
  int32_t c0x, c0y, c0t;
  unlin(L, c0lin, &c0x, &c0y, &c0t);
  const int64_t c0[3] = {c0x, c0y, c0t};
  const int64_t dim[3] = {L->W, L->H, L->T};
  const int64_t hh[3] = {P->patch[0] / 2, P->patch[1] / 2, P->patch[2] / 2};
  const uint64_t key[2] = {P->seed, 0};
  uint64_t ctr[4] = {(uint64_t)p, step, (uint64_t)k, ((uint64_t)level << 8) | 0u};
  uint64_t w[4];
  vio_philox4x64_10(ctr, key, w);
  int64_t c[3];
  for (int a = 0; a < 3; ++a) {
    const int64_t lo = c0[a] - R > hh[a] ? c0[a] - R : hh[a];
    const int64_t hi = c0[a] + R < dim[a] - 1 - hh[a] ? c0[a] + R : dim[a] - 1 - hh[a];
    c[a] = lo + draw_below(w[a], hi - lo + 1);
  }
  return lin(L, c[0], c[1], c[2]);
}

int64_t vio_rs_candidate(const vio_ctx* ctx, int32_t level, int64_t p, int64_t c0, int32_t k,
                         uint64_t step) {
  if (!ctx || level < 0 || level >= ctx->L || k < 1) return -1;
  const level_t* L = &ctx->lv[level];
  if (p < 0 || p >= L->V || c0 < 0 || c0 >= L->V || !L->dsrc[c0]) return -1;
  const int32_t r_max = L->W > L->H ? (L->W > L->T ? L->W : L->T) : (L->H > L->T ? L->H : L->T);
  const int64_t R = rs_radius(&ctx->prm, r_max, k);
  if (R < 1) return -1;
  return rs_candidate(ctx, level, p, c0, R, step, k);
}

static void search(vio_ctx* ctx, int32_t level, const uint8_t* tmask, const uint8_t* cmask,
                   uint64_t step) {
  level_t* L = &ctx->lv[level];
  const vio_params* P = &ctx->prm;
  const int64_t V = L->V;
  /* target list in ascending order */
  int64_t nS = 0;
  for (int64_t i = 0; i < V; ++i) nS += tmask[i] ? 1 : 0;
  int64_t* S = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nS > 0 ? nS : 1));
  int32_t* ncand = (int32_t*)malloc(sizeof(int32_t) * (size_t)V);
  int32_t* ndist = (int32_t*)malloc(sizeof(int32_t) * (size_t)V);
  {
    int64_t k = 0;
    for (int64_t i = 0; i < V; ++i)
      if (tmask[i]) S[k++] = i;
  }
  const uint64_t key[2] = {P->seed, 0};
  /* the reduced distance: the targets' features on the current video (the
     sources' patches never change within a level) */
  const int red = L->red_d > 0 && cmask == NULL;
  if (red) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < nS; ++j) features_of(ctx, L, S[j], L->feat + S[j] * L->red_d);
  }

  /* step 0: initialisation of missing / invalid matches, re-evaluation */
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t j = 0; j < nS; ++j) {
    int64_t p = S[j];
    if (L->cand[p] < 0 || L->cand[p] >= V || !L->dsrc[L->cand[p]]) {
      uint64_t ctr[4] = {(uint64_t)p, step, 0, ((uint64_t)level << 8) | 1u};
      uint64_t w[4];
      vio_philox4x64_10(ctr, key, w);
      L->cand[p] = (int32_t)L->dlist[draw_below(w[0], L->nD)];
    }
    int32_t n = 0;
    L->dist[p] = (int32_t)search_dist(ctx, L, red, p, L->cand[p], cmask, &n);
    if (!red) L->nvox[p] = (uint8_t)n;
  }

  const int32_t r_max = L->W > L->H ? (L->W > L->T ? L->W : L->T) : (L->H > L->T ? L->H : L->T);
  for (int k = 1; k <= P->pm_iters; ++k) {
    /* propagation */
    for (int js = 0; js < P->n_jf; ++js) {
      const int32_t s = P->jf_steps[js];
      memcpy(ncand, L->cand, sizeof(int32_t) * (size_t)V);
      memcpy(ndist, L->dist, sizeof(int32_t) * (size_t)V);
#pragma omp parallel for schedule(dynamic, 256)
      for (int64_t j = 0; j < nS; ++j) {
        int64_t p = S[j];
        int32_t px, py, pt;
        unlin(L, p, &px, &py, &pt);
        int64_t best_c = L->cand[p];
        int64_t best_d = L->dist[p];
        for (int idx = 1; idx <= 6; ++idx) {
          int axis = (idx - 1) / 2;
          int sign = ((idx - 1) % 2 == 0) ? -1 : 1;
          int32_t qx = px + (axis == 0 ? sign * s : 0);
          int32_t qy = py + (axis == 1 ? sign * s : 0);
          int32_t qt = pt + (axis == 2 ? sign * s : 0);
          if (!inside(L, qx, qy, qt)) continue;
          int64_t q = lin(L, qx, qy, qt);
          if (!tmask[q]) continue;
          int32_t cqx, cqy, cqt;
          unlin(L, L->cand[q], &cqx, &cqy, &cqt);
          /* c = p + phi(q) with phi(q) = cand(q) - q */
          int32_t cx = px + (cqx - qx), cy = py + (cqy - qy), ct = pt + (cqt - qt);
          if (!inside(L, cx, cy, ct)) continue;
          int64_t c = lin(L, cx, cy, ct);
          if (!L->dsrc[c]) continue;
          int64_t d = search_dist(ctx, L, red, p, c, cmask, NULL);
          if (d < best_d) { best_d = d; best_c = c; }
        }
        ncand[p] = (int32_t)best_c;
        ndist[p] = (int32_t)best_d;
      }
      memcpy(L->cand, ncand, sizeof(int32_t) * (size_t)V);
      memcpy(L->dist, ndist, sizeof(int32_t) * (size_t)V);
    }
    /* random search, Eq. (3.1) */
    const int64_t R = rs_radius(P, r_max, k);
    if (R < 1) continue;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < nS; ++j) {
      int64_t p = S[j];
      int64_t c = rs_candidate(ctx, level, p, L->cand[p], R, step, k);
      if (!L->dsrc[c]) continue;
      int64_t d = search_dist(ctx, L, red, p, c, cmask, NULL);
      if (d < L->dist[p]) {
        L->cand[p] = (int32_t)c;
        L->dist[p] = (int32_t)d;
      }
    }
  }
  /* the reduced distance only chooses the matches: every target's match
     is evaluated with the exact distance, which the reconstruction uses */
  if (red) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t j = 0; j < nS; ++j) {
      const int64_t p = S[j];
      int32_t n = 0;
      L->dist[p] = (int32_t)ssd(ctx, L, p, L->cand[p], NULL, &n);
      L->nvox[p] = (uint8_t)n;
    }
  }
  free(S);
  free(ncand);
  free(ndist);
  L->searched = 1;
}

int vio_nnf_search(vio_ctx* ctx, int32_t level, int32_t em_iter) {
  if (!ctx || level < 0 || level >= ctx->L || em_iter < 0) return VIO_E_INVAL;
  search(ctx, level, ctx->lv[level].htil, NULL, (uint64_t)em_iter);
  return VIO_OK;
}

int vio_nnf_search_set(vio_ctx* ctx, int32_t level, const uint8_t* target_mask,
                       const uint8_t* count_mask, uint64_t step) {
  if (!ctx || level < 0 || level >= ctx->L || !target_mask) return VIO_E_INVAL;
  search(ctx, level, target_mask, count_mask, step);
  return VIO_OK;
}

/* ------------------------------------------------------------------------ */
/* Reconstruction (Sec. 3.2).                                               */
/* For a hole pixel p, the contributors are q = p - o over the patch        */
/* offsets o (in offset order) that lie in the volume and pass the filter;  */
/* contributor q votes u(q + phi(q) + (p - q)) = u(cand(q) + o).            */
/* delta_q = dist(q) / nvox(q) (the normalised squared patch distance);     */
/* WEIGHTED (Eqs. (3.2)-(3.3)): sigma^2 = the ceil(0.75 m)-th smallest       */
/* delta (nearest-rank 75th percentile), s_q = exp(-delta_q / (2 sigma^2)), */
/* or [delta_q = 0] when sigma^2 = 0;  MEAN: s_q = 1;                        */
/* BEST (Eq. (3.4)): the vote of the contributor with the smallest delta    */
/* (first in offset order on ties).                                         */
/* Weights and sums are float32, accumulated in offset order; the result is */
/* rounded half up to uint8 and written back (colour and texture).          */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t dist;
  int32_t n;
  int64_t src; /* cand(q) + o */
} contrib_t;

/* a/b < c/d for positive b, d */
static int rat_less(int64_t a, int64_t b, int64_t c, int64_t d) { return a * d < c * b; }

static int64_t recon_pixel(const vio_ctx* ctx, level_t* L, int64_t p, const uint8_t* filt,
                           int mode, float* out5) {
  const int hx = ctx->prm.patch[0] / 2, hy = ctx->prm.patch[1] / 2, ht = ctx->prm.patch[2] / 2;
  contrib_t Q[1024];
  int m = 0;
  int32_t px, py, pt;
  unlin(L, p, &px, &py, &pt);
  for (int dt = -ht; dt <= ht; ++dt)
    for (int dy = -hy; dy <= hy; ++dy)
      for (int dx = -hx; dx <= hx; ++dx) {
        int32_t qx = px - dx, qy = py - dy, qt = pt - dt;
        if (!inside(L, qx, qy, qt)) continue;
        int64_t q = lin(L, qx, qy, qt);
        if (filt && !filt[q]) continue;
        int32_t cx, cy, ct;
        unlin(L, L->cand[q], &cx, &cy, &ct);
        Q[m].dist = L->dist[q];
        Q[m].n = L->nvox[q];
        Q[m].src = lin(L, cx + dx, cy + dy, ct + dt);
        m++;
      }
  float s[1024];
  uint8_t* up = &L->rgbt[5 * p];
  uint8_t old[3] = {up[0], up[1], up[2]};
  if (mode == VIO_RECON_BEST) {
    int b = 0;
    for (int i = 1; i < m; ++i)
      if (rat_less(Q[i].dist, Q[i].n, Q[b].dist, Q[b].n)) b = i;
    const uint8_t* v = &L->rgbt[5 * Q[b].src];
    for (int c = 0; c < 5; ++c) {
      if (out5) out5[c] = (float)v[c] / 255.0f;
      up[c] = v[c];
    }
  } else {
    if (mode == VIO_RECON_MEAN) {
      for (int i = 0; i < m; ++i) s[i] = 1.0f;
    } else {
      /* nearest-rank percentile: sort a copy of the deltas (insertion sort) */
      int order[1024];
      for (int i = 0; i < m; ++i) order[i] = i;
      for (int i = 1; i < m; ++i) {
        int v = order[i], j = i - 1;
        while (j >= 0 && rat_less(Q[v].dist, Q[v].n, Q[order[j]].dist, Q[order[j]].n)) {
          order[j + 1] = order[j];
          --j;
        }
        order[j + 1] = v;
      }
      const int r = (3 * m + 3) / 4; /* ceil(0.75 m), 1-based */
      const int64_t sd = Q[order[r - 1]].dist, sn = Q[order[r - 1]].n;
      for (int i = 0; i < m; ++i) {
        if (sd > 0) {
          /* delta_q / (2 sigma^2) = (dist_q n_r) / (2 dist_r n_q) */
          double num = (double)((int64_t)Q[i].dist * sn);
          double den = (double)(2 * sd * (int64_t)Q[i].n);
          float tq = (float)(num / den);
          s[i] = expf(-tq);
        } else {
          s[i] = Q[i].dist == 0 ? 1.0f : 0.0f;
        }
      }
    }
    float wsum = 0.0f, acc[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < m; ++i) {
      const uint8_t* v = &L->rgbt[5 * Q[i].src];
      wsum += s[i];
      for (int c = 0; c < 5; ++c) acc[c] = fmaf(s[i], (float)v[c], acc[c]);
    }
    for (int c = 0; c < 5; ++c) {
      float o = acc[c] / wsum;
      if (out5) out5[c] = o / 255.0f;
      int q = (int)floorf(o + 0.5f);
      up[c] = (uint8_t)(q > 255 ? 255 : q);
    }
  }
  return (int64_t)abs(up[0] - old[0]) + abs(up[1] - old[1]) + abs(up[2] - old[2]);
}

/* reconstruct the pixels of pmask (ascending order), contributors filtered by filt */
static int64_t reconstruct(vio_ctx* ctx, level_t* L, const uint8_t* pmask, const uint8_t* filt,
                           int mode, float* out_f) {
  int64_t nP = 0;
  for (int64_t i = 0; i < L->V; ++i) nP += pmask[i] ? 1 : 0;
  int64_t* P = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nP > 0 ? nP : 1));
  int64_t k = 0;
  for (int64_t i = 0; i < L->V; ++i)
    if (pmask[i]) P[k++] = i;
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total)
  for (int64_t j = 0; j < nP; ++j)
    total += recon_pixel(ctx, L, P[j], filt, mode, out_f ? &out_f[5 * j] : NULL);
  free(P);
  return total;
}

int vio_reconstruct(vio_ctx* ctx, int32_t level, int32_t mode, float* out_f, int64_t* absdiff) {
  if (!ctx || level < 0 || level >= ctx->L) return VIO_E_INVAL;
  if (mode != VIO_RECON_WEIGHTED && mode != VIO_RECON_MEAN && mode != VIO_RECON_BEST)
    return VIO_E_INVAL;
  level_t* L = &ctx->lv[level];
  if (!L->searched) return VIO_E_STATE;
  int64_t s = reconstruct(ctx, L, L->hole, NULL, mode, out_f);
  if (absdiff) *absdiff = s;
  return VIO_OK;
}

int vio_set_reduction(vio_ctx* ctx, int32_t level, const int16_t* Q, int32_t d) {
  if (!ctx || level < 0 || level >= ctx->L || d < 0 || (d > 0 && !Q)) return VIO_E_INVAL;
  level_t* L = &ctx->lv[level];
  const int dim = 5 * ctx->prm.patch[0] * ctx->prm.patch[1] * ctx->prm.patch[2];
  if (d > dim) return VIO_E_INVAL;
  free(L->redQ);
  free(L->feat);
  L->redQ = NULL;
  L->feat = NULL;
  L->red_d = 0;
  if (d == 0) return VIO_OK;
  L->redQ = (int16_t*)malloc(sizeof(int16_t) * (size_t)d * dim);
  L->feat = (int32_t*)malloc(sizeof(int32_t) * (size_t)d * (size_t)L->V);
  if (!L->redQ || !L->feat) return VIO_E_NOMEM;
  memcpy(L->redQ, Q, sizeof(int16_t) * (size_t)d * dim);
  L->red_d = d;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t p = 0; p < L->V; ++p) features_of(ctx, L, p, L->feat + p * d);
  return VIO_OK;
}

int vio_features(const vio_ctx* ctx, int32_t level, int32_t* out) {
  if (!ctx || level < 0 || level >= ctx->L || !out) return VIO_E_INVAL;
  const level_t* L = &ctx->lv[level];
  if (L->red_d == 0) return VIO_E_STATE;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t p = 0; p < L->V; ++p) features_of(ctx, L, p, out + p * L->red_d);
  return VIO_OK;
}

/* Moments of the patch vectors of a sample of the sources: every k-th
   entry of D~ in ascending order, k = ceil(|D~| / n_max), so at most n_max
   samples.  S1[i] = sum of x_i, S2[i][j] = sum of x_i x_j (all dim x dim
   entries), exact integers. */
int vio_pca_moments(const vio_ctx* ctx, int32_t level, int32_t n_max, uint64_t* S1,
                    uint64_t* S2, int64_t* n_out) {
  if (!ctx || level < 0 || level >= ctx->L || n_max < 1 || !S1 || !S2 || !n_out)
    return VIO_E_INVAL;
  const level_t* L = &ctx->lv[level];
  const int hx = ctx->prm.patch[0] / 2, hy = ctx->prm.patch[1] / 2, ht = ctx->prm.patch[2] / 2;
  const int dim = 5 * ctx->prm.patch[0] * ctx->prm.patch[1] * ctx->prm.patch[2];
  const int64_t k = (L->nD + n_max - 1) / n_max;
  memset(S1, 0, sizeof(uint64_t) * dim);
  memset(S2, 0, sizeof(uint64_t) * (size_t)dim * dim);
  int64_t n = 0;
  uint8_t* x = (uint8_t*)malloc((size_t)dim);
  if (!x) return VIO_E_NOMEM;
  for (int64_t j = 0; k > 0 && j < L->nD; j += k, ++n) {
    int32_t cx, cy, ct;
    unlin(L, L->dlist[j], &cx, &cy, &ct);
    int i = 0;
    for (int dt = -ht; dt <= ht; ++dt)
      for (int dy = -hy; dy <= hy; ++dy)
        for (int dx = -hx; dx <= hx; ++dx) {
          const int64_t a = lin(L, cx + dx, cy + dy, ct + dt);
          for (int ch = 0; ch < 5; ++ch) x[i++] = L->rgbt[5 * a + ch];
        }
    for (int a = 0; a < dim; ++a) {
      S1[a] += x[a];
      for (int b = 0; b < dim; ++b) S2[(size_t)a * dim + b] += (uint64_t)x[a] * x[b];
    }
  }
  free(x);
  *n_out = n;
  return VIO_OK;
}

/* ------------------------------------------------------------------------ */
/* EM loop of one level (Alg. 4): search, reconstruct, stop when the mean   */
/* absolute colour change per channel per hole pixel is at most em_tol, or  */
/* after em_max_iters iterations.                                           */
/* ------------------------------------------------------------------------ */
int vio_inpaint_level(vio_ctx* ctx, int32_t level, int32_t* iters_run) {
  if (!ctx || level < 0 || level >= ctx->L) return VIO_E_INVAL;
  level_t* L = &ctx->lv[level];
  int32_t k = 0;
  if (L->nH > 0) {
    double e;
    do {
      search(ctx, level, L->htil, NULL, (uint64_t)k);
      int64_t s = reconstruct(ctx, L, L->hole, NULL, ctx->prm.recon_mode, NULL);
      ++k;
      e = (double)s / (3.0 * (double)L->nH);
    } while (e > ctx->prm.em_tol && k < ctx->prm.em_max_iters);
  }
  /* with no hole the target set is empty and the (empty) map is complete */
  L->searched = 1;
  if (iters_run) *iters_run = k;
  return VIO_OK;
}

/* ------------------------------------------------------------------------ */
/* Onion-peel initialisation (Sec. 3.5, Alg. 3).  H' starts as the coarsest */
/* hole; each layer is H' minus its erosion by the 3x3x3 cube (voxels       */
/* outside the volume count as occluded).  The layer's targets are the      */
/* voxels outside H' whose patch touches the layer; they are matched with   */
/* the partial distance over voxels outside H' (Eq. (3.10)), and the layer  */
/* is reconstructed from those targets only (Eq. (3.11)).                   */
/* ------------------------------------------------------------------------ */
int vio_onion_layer(vio_ctx* ctx, uint8_t* Hp, int32_t layer, uint8_t* bd_out, uint8_t* S_out,
                    float* out_f, int64_t* n_layer) {
  if (!ctx || !Hp || layer < 0) return VIO_E_INVAL;
  const int32_t level = ctx->L - 1;
  level_t* L = &ctx->lv[level];
  const int hx = ctx->prm.patch[0] / 2, hy = ctx->prm.patch[1] / 2, ht = ctx->prm.patch[2] / 2;
  const size_t V = (size_t)L->V;
  if (layer == 0) /* the peel starts from an empty shift map */
    for (size_t i = 0; i < V; ++i) { L->cand[i] = -1; L->dist[i] = -1; L->nvox[i] = 0; }
  uint8_t* E = (uint8_t*)malloc(V);
  uint8_t* bd = (uint8_t*)malloc(V);
  uint8_t* S = (uint8_t*)malloc(V);
  uint8_t* M = (uint8_t*)malloc(V);
  if (!E || !bd || !S || !M) {
    free(E); free(bd); free(S); free(M);
    return VIO_E_NOMEM;
  }
  /* E = erosion of H' by the 3x3x3 cube, outside the volume counting as
   * occluded; the layer is H' minus E */
  int64_t nb = 0;
  for (int32_t t = 0; t < L->T; ++t)
    for (int32_t y = 0; y < L->H; ++y)
      for (int32_t x = 0; x < L->W; ++x) {
        int all = 1;
        for (int dt = -1; dt <= 1; ++dt)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
              if (inside(L, x + dx, y + dy, t + dt) && !Hp[lin(L, x + dx, y + dy, t + dt)])
                all = 0;
        int64_t i = lin(L, x, y, t);
        E[i] = (uint8_t)(Hp[i] && all);
        bd[i] = (uint8_t)(Hp[i] && !E[i]);
        nb += bd[i];
      }
  /* targets: voxels outside H' whose patch touches the layer */
  for (int32_t t = 0; t < L->T; ++t)
    for (int32_t y = 0; y < L->H; ++y)
      for (int32_t x = 0; x < L->W; ++x) {
        int64_t i = lin(L, x, y, t);
        int near = 0;
        for (int dt = -ht; dt <= ht; ++dt)
          for (int dy = -hy; dy <= hy; ++dy)
            for (int dx = -hx; dx <= hx; ++dx)
              if (inside(L, x + dx, y + dy, t + dt) && bd[lin(L, x + dx, y + dy, t + dt)])
                near = 1;
        S[i] = (uint8_t)(near && !Hp[i]);
        M[i] = (uint8_t)!Hp[i];
      }
  if (nb > 0) {
    search(ctx, level, S, M, (1ULL << 32) + (uint64_t)layer);
    reconstruct(ctx, L, bd, M, ctx->prm.recon_mode, out_f);
  }
  L->searched = 0; /* the inner layers' targets may still be unmatched */
  if (bd_out) memcpy(bd_out, bd, V);
  if (S_out) memcpy(S_out, S, V);
  memcpy(Hp, E, V);
  free(E); free(bd); free(S); free(M);
  if (n_layer) *n_layer = nb;
  return VIO_OK;
}

int vio_onion_init(vio_ctx* ctx, int32_t* layers_run) {
  if (!ctx) return VIO_E_INVAL;
  level_t* L = &ctx->lv[ctx->L - 1];
  uint8_t* Hp = (uint8_t*)malloc((size_t)L->V);
  if (!Hp) return VIO_E_NOMEM;
  memcpy(Hp, L->hole, (size_t)L->V);
  int32_t layer = 0;
  for (;;) {
    int64_t nb = 0;
    int st = vio_onion_layer(ctx, Hp, layer, NULL, NULL, NULL, &nb);
    if (st) {
      free(Hp);
      return st;
    }
    if (nb == 0) break; /* H' is empty */
    ++layer;
  }
  free(Hp);
  if (layers_run) *layers_run = layer;
  return VIO_OK;
}

/* ------------------------------------------------------------------------ */
/* Level transition (Sec. 3.6): nearest-neighbour upsampling of the shift   */
/* map (spatial components doubled; the temporal one kept, or doubled too   */
/* with temporal subsampling); the fine target inherits its parent's        */
/* distance and count; then the finer hole is reconstructed.                */
/* ------------------------------------------------------------------------ */
int vio_transition(vio_ctx* ctx, int32_t level) {
  if (!ctx || level < 0 || level + 1 >= ctx->L) return VIO_E_INVAL;
  level_t* F = &ctx->lv[level];
  level_t* C = &ctx->lv[level + 1];
  if (!C->searched) return VIO_E_STATE;
  for (int32_t t = 0; t < F->T; ++t)
    for (int32_t y = 0; y < F->H; ++y)
      for (int32_t x = 0; x < F->W; ++x) {
        int64_t i = lin(F, x, y, t);
        if (!F->htil[i]) {
          F->cand[i] = -1; F->dist[i] = -1; F->nvox[i] = 0;
          continue;
        }
        const int ts = ctx->prm.temporal_subsample;
        const int32_t Pt = ts ? t / 2 : t;
        int64_t P = lin(C, x / 2, y / 2, Pt);
        int32_t cx, cy, ct;
        unlin(C, C->cand[P], &cx, &cy, &ct);
        /* the parent's shift, doubled along every subsampled axis */
        int32_t fx = x + 2 * (cx - x / 2), fy = y + 2 * (cy - y / 2);
        int32_t ft = ts ? t + 2 * (ct - Pt) : t + (ct - t);
        F->cand[i] = (int32_t)lin(F, fx, fy, ft);
        F->dist[i] = C->dist[P];
        F->nvox[i] = C->nvox[P];
      }
  F->searched = 1;
  reconstruct(ctx, F, F->hole, NULL, ctx->prm.recon_mode, NULL);
  return VIO_OK;
}

/* Alg. 4 without the realignment pre- and post-processing. */
int vio_inpaint(vio_ctx* ctx, uint8_t* out_rgb) {
  if (!ctx || !out_rgb) return VIO_E_INVAL;
  int st = vio_onion_init(ctx, NULL);
  if (st) return st;
  for (int32_t l = ctx->L - 1; l >= 0; --l) {
    if (l < ctx->L - 1) {
      st = vio_transition(ctx, l);
      if (st) return st;
    }
    st = vio_inpaint_level(ctx, l, NULL);
    if (st) return st;
  }
  level_t* L0 = &ctx->lv[0];
  if (L0->nH > 0) reconstruct(ctx, L0, L0->hole, NULL, VIO_RECON_BEST, NULL);
  for (int64_t i = 0; i < L0->V; ++i)
    for (int c = 0; c < 3; ++c) out_rgb[3 * i + c] = L0->rgbt[5 * i + c];
  return VIO_OK;
}

int64_t vio_energy(const vio_ctx* ctx, int32_t level) {
  if (!ctx || level < 0 || level >= ctx->L) return -1;
  const level_t* L = &ctx->lv[level];
  int64_t E = 0;
  for (int64_t i = 0; i < L->V; ++i)
    if (L->htil[i] && L->cand[i] >= 0) E += ssd(ctx, L, i, L->cand[i], NULL, NULL);
  return E;
}
