/* vio.h -- CPU oracle for the global patch-based video inpainting of
 * Newson, Almansa, Fradet, Gousseau, Perez, "Video Inpainting of Complex
 * Scenes" (SIAM J. Imaging Sciences 2014, arXiv 1503.05528).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls it.  It shares no code with the HIP library.
 *
 * All pointers are HOST pointers.  Every function returns vio_status
 * (0 = OK, < 0 = error) unless stated otherwise.
 *
 * Conventions (the paper is silent on them; readings listed in the design
 * notes):
 *   position p = (x, y, t), 0-based, lin(p) = (t*H + y)*W + x;
 *   level 0 is the finest, level L-1 the coarsest;
 *   patch offsets o are enumerated dt-major, then dy, then dx, each
 *   ascending from -h to +h;
 *   colour and texture channels are 0..255 integers (uint8);
 *   a voxel carries 5 channels R, G, B, Tx, Ty.
 */
#ifndef VIO_H
#define VIO_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  VIO_OK = 0,
  VIO_E_INVAL = -1,
  VIO_E_NOMEM = -2,
  VIO_E_STATE = -4,
  VIO_E_EMPTY_SOURCE = -5
};
enum { VIO_RECON_WEIGHTED = 0, VIO_RECON_MEAN = 1, VIO_RECON_BEST = 2 };

typedef struct {
  int32_t abi_version;  /* 1 */
  int32_t patch[3];     /* patch size (x, y, t), odd; 5x5x5 (Sec. 3.7) */
  int32_t levels;       /* pyramid levels L >= 1 */
  int32_t lambda;       /* texture weight, 50 (Sec. 3.7) */
  int32_t pm_iters;     /* PatchMatch iterations, 10 (Sec. 3.1, 3.7) */
  int32_t n_jf;         /* propagation steps per iteration */
  int32_t jf_steps[8];  /* {4, 2, 1} */
  double rho;           /* random-search window reduction, 0.5 (Eq. 3.1 of Sec. 3.1) */
  int32_t em_max_iters; /* 20 (Sec. 3.7) */
  double em_tol;        /* 0.1, mean absolute colour change; < 0: run em_max_iters */
  int32_t recon_mode;   /* VIO_RECON_WEIGHTED or VIO_RECON_MEAN */
  uint64_t seed;        /* Philox key word 0 */
  int32_t temporal_subsample; /* 0: coarser levels keep every frame (Sec. 3.6);
                                 1: each coarser level also halves the frame
                                 count (2x2x2 blocks) */
} vio_params;

typedef struct vio_ctx vio_ctx;

int vio_params_default(vio_params* out);

/* Builds the image, occlusion and texture-feature pyramids and the source /
 * target sets of every level.  rgb [T][H][W][3], mask [T][H][W] (1 = hole);
 * rgb values under the mask are never read. */
int vio_create(vio_ctx** out, const vio_params* prm, int32_t W, int32_t H, int32_t T,
               const uint8_t* rgb, const uint8_t* mask);
void vio_destroy(vio_ctx* ctx);

/* dims[3] = (W_l, H_l, T); counts[3] = (|H^l|, |H~^l|, |D~^l|) */
int vio_level_info(const vio_ctx* ctx, int32_t level, int32_t dims[3], int64_t counts[3]);
/* byte masks over the level volume: hole H^l, sources D~^l, targets H~^l */
int vio_level_sets(const vio_ctx* ctx, int32_t level, uint8_t* hole, uint8_t* dsrc,
                   uint8_t* htil);

/* State of a level.  rgbt [V][5]; cand [V] absolute linear index (-1 unset or
 * outside H~); dist [V] integer SSD (-1 outside H~); nvox [V] number of
 * voxels the SSD counted (0 outside H~).  NULL pointers are skipped. */
int vio_get_state(const vio_ctx* ctx, int32_t level, uint8_t* rgbt, int32_t* cand,
                  int32_t* dist, uint8_t* nvox);
int vio_set_state(vio_ctx* ctx, int32_t level, const uint8_t* rgbt, const int32_t* cand,
                  const int32_t* dist, const uint8_t* nvox);

/* Integer SSD between the patches centred at p and at c (linear indices) at
 * a level; count_mask (or NULL for all) selects the compared voxels p+o. */
int64_t vio_patch_ssd(const vio_ctx* ctx, int32_t level, int64_t p, int64_t c,
                      const uint8_t* count_mask, int32_t* n_out);

/* Philox4x64-10 block: out = Philox(counter, key). */
void vio_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* The uniform integer in [0, n) that a 64-bit random word maps to: the high
 * 32 bits times n, divided by 2^32 (-1 for n <= 0). */
int64_t vio_draw_below(uint64_t w, int64_t n);
/* The random-search candidate (linear index) the search draws for target p
 * around its match c0 (a source) in PatchMatch iteration k >= 1 with random
 * step `step` (Eq. (3.1)); -1 for bad arguments or a radius below 1. */
int64_t vio_rs_candidate(const vio_ctx* ctx, int32_t level, int64_t p, int64_t c0, int32_t k,
                         uint64_t step);

/* ANN search (Alg. "ANN search with 3D PatchMatch", redesigned as
 * synchronous propagation) over the target set H~^level with the full
 * distance; em_iter keys the random numbers. */
int vio_nnf_search(vio_ctx* ctx, int32_t level, int32_t em_iter);
/* The same search over an arbitrary target set and comparison mask
 * (count_mask NULL = all voxels); step keys the random numbers. */
int vio_nnf_search_set(vio_ctx* ctx, int32_t level, const uint8_t* target_mask,
                       const uint8_t* count_mask, uint64_t step);

/* Reconstruction of the hole H^level (Eqs. of Sec. 3.2).  out_f, if not NULL,
 * receives [|H^l|][5] values in [0,1] in ascending linear order of the hole;
 * absdiff, if not NULL, receives sum over the hole of |new - old| over RGB. */
int vio_reconstruct(vio_ctx* ctx, int32_t level, int32_t mode, float* out_f, int64_t* absdiff);

/* One pyramid level of the EM loop (Alg. "Proposed video inpainting
 * algorithm", inner while loop); iters_run receives the number of
 * iterations. */
int vio_inpaint_level(vio_ctx* ctx, int32_t level, int32_t* iters_run);
/* Onion-peel initialisation at the coarsest level (Sec. 3.5, Alg. 3). */
int vio_onion_init(vio_ctx* ctx, int32_t* layers_run);
/* One layer of the onion peel at the coarsest level.  Hp [V] holds the
 * current occlusion H' on entry and its erosion by the 3x3x3 cube (outside
 * the volume counted as occluded) on return.  The layer is H' minus that
 * erosion; its targets are the voxels outside H' whose patch touches it;
 * they are searched with the partial distance over voxels outside H'
 * (Eq. (3.10)) and the layer is reconstructed from those contributors only
 * (Eq. (3.11)).  layer keys the random numbers (step 2^32 + layer); layer 0
 * first empties the level's shift map.  bd_out / S_out [V] (or NULL) receive
 * the layer and its targets, out_f [|layer|][5] (or NULL) the reconstructed
 * values in [0,1] in ascending linear order, n_layer the layer's size (0:
 * H' was empty and nothing was done). */
int vio_onion_layer(vio_ctx* ctx, uint8_t* Hp, int32_t layer, uint8_t* bd_out, uint8_t* S_out,
                    float* out_f, int64_t* n_layer);
/* Level transition level+1 -> level: nearest-neighbour upsampling of the
 * shift map, then reconstruction of the finer hole (Sec. 3.6). */
int vio_transition(vio_ctx* ctx, int32_t level);
/* The whole method minus realignment: out_rgb [T][H][W][3]. */
int vio_inpaint(vio_ctx* ctx, uint8_t* out_rgb);

/* ---- Realignment of a video with a moving camera (Sec. 3.4, Alg. 2) ----
 * Affine maps are 6 doubles m: x' = m0 x + m1 y + m2, y' = m3 x + m4 y + m5,
 * in pixel coordinates of a frame (x right, y down). */
typedef struct {
  int32_t levels; /* grey pyramid levels of the motion estimation, 3 */
  int32_t iters;  /* robust Gauss-Newton steps per level, 8 */
  double tukey_c; /* Tukey biweight constant, grey levels (0..255), 20 */
} vio_align_params;
int vio_align_params_default(vio_align_params* out);
/* The dominant affine motion of every pair of successive frames (Alg. 2,
 * first loop): theta [T-1][6], theta_n maps frame n's pixels to their
 * positions in frame n+1.  rgb [T][H][W][3]; mask [T][H][W] nonzero =
 * occluded (excluded from the estimation). */
int vio_align_estimate(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H,
                       int32_t T, const vio_align_params* prm, double* theta);
/* Composition to the reference frame T/2 (0-based; Alg. 2, second loop):
 * M [T][6], M_n maps frame n's pixels to the reference frame. */
int vio_align_compose(const double* theta, int32_t T, double* M);
/* inverse of an affine map (VIO_E_INVAL if singular) */
int vio_affine_inverse(const double m[6], double inv[6]);
/* The aligned video (Alg. 2, AffineWarp): pixel y of aligned frame n is
 * frame n sampled at M_n^-1(y) by bilinear interpolation, rounded half up;
 * out_mask = 1 (and out_rgb 0) where a neighbour of nonzero weight lies
 * outside the frame or is occluded. */
int vio_align_warp(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H, int32_t T,
                   const double* M, uint8_t* out_rgb, uint8_t* out_mask);
/* The inverse (Alg. 4, last step): out_rgb = rgb, except every occluded
 * pixel x of mask, which takes the aligned video sampled at M_n(x) (clamped
 * to the frame) by bilinear interpolation. */
int vio_align_unwarp(const uint8_t* aligned, const uint8_t* rgb, const uint8_t* mask, int32_t W,
                     int32_t H, int32_t T, const double* M, uint8_t* out_rgb);

/* ---- Dimensionality-reduced patch distance (Sec. 5) ----
 * A basis Q [d][dim] (dim = 5 x patch voxels; int16, a linear map scaled
 * by 256) for one level: the features of voxel p are
 * f_k(p) = floor((sum_i Q[k][i] x_i(p) + 128) / 256), x(p) the patch
 * vector (offsets dt, dy, dx; channels R, G, B, Tx, Ty; coordinates clamped
 * to the volume), and the level's unmasked searches compare
 * sum_k (f_k(p) - f_k(c))^2 (saturated at 2^31 - 1) instead of the patch
 * distance; after each search every target's match is evaluated with the
 * exact distance.  d = 0 restores the exact search. */
int vio_set_reduction(vio_ctx* ctx, int32_t level, const int16_t* Q, int32_t d);
/* the features of every voxel of the level: out [V][d] */
int vio_features(const vio_ctx* ctx, int32_t level, int32_t* out);
/* Exact moments of the patch vectors of every k-th source (D~ ascending,
 * k = ceil(|D~| / n_max)): S1 [dim], S2 [dim][dim], *n = samples. */
int vio_pca_moments(const vio_ctx* ctx, int32_t level, int32_t n_max, uint64_t* S1,
                    uint64_t* S2, int64_t* n);

/* ---- The textured-patch experiment of App. B ----
 * For every reference patch W_r (ref [n_ref][pt][ph][pw], grey values) and
 * every patch V of the grey volume vol [T][H][W] that lies wholly inside
 * it, counts[r] = the number of V with SSD(W_r, V) < SSD(W_r, Z), Z the
 * constant patch of value mu (0..255).  A volume smaller than the patch
 * has no candidates (all counts 0). */
int vio_closer_than_constant(const uint8_t* ref, int32_t n_ref, const uint8_t* vol, int32_t W,
                             int32_t H, int32_t T, int32_t pw, int32_t ph, int32_t pt,
                             int32_t mu, uint64_t* counts);

/* E = sum over H~^level of SSD(q, cand(q)) (unnormalised). */
int64_t vio_energy(const vio_ctx* ctx, int32_t level);

/* number of OpenMP threads the oracle uses (1 without OpenMP) */
int vio_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
