/* vi.h -- C ABI of libvi, the MI355X (gfx950) implementation of the hot path
 * of Newson, Almansa, Fradet, Gousseau, Perez, "Video Inpainting of Complex
 * Scenes" (SIAM J. Imaging Sciences 7(4), 2014; arXiv 1503.05528).
 *
 * The problem (Sec. 2): a colour video u over a space-time volume Omega and
 * an occlusion H (a set of positions) are given; the method fills u on H by
 * alternating an approximate-nearest-neighbour search of a shift map phi over
 * 5x5x5 patches (Sec. 3.1) and a reconstruction of every occluded pixel from
 * the patches that cover it (Sec. 3.2), inside a multi-resolution pyramid
 * with texture features (Sec. 3.3, 3.6) and an onion-peel initialisation
 * (Sec. 3.5); the complete loop is Alg. 4.  Affine realignment (Sec. 3.4) is
 * not part of this library.
 *
 * Conventions
 *   - Every function returns vi_status (VI_OK = 0, negative = error) unless
 *     stated otherwise; no C++ exception crosses the ABI; vi_last_error()
 *     returns a thread-local message for the last failing call.
 *   - (dev) marks device pointers (memory of the GPU the context was created
 *     on, e.g. a torch tensor's data_ptr()); (host) marks host pointers.
 *   - All device work is enqueued on the context's HIP stream; a call returns
 *     after enqueueing unless marked "syncs".  The caller owns every buffer
 *     it passes; the context owns everything it allocates.
 *   - Positions p = (x, y, t) are 0-based; linear index lin(p) =
 *     (t*H_l + y)*W_l + x at level l; level 0 is the finest.
 *   - Colour and texture channels are integers 0..255; a voxel carries five
 *     channels R, G, B, Tx, Ty.
 *   - Limits: W < 32768, H < 32768, T < 32768, W*H*T < 2^31, levels <= 8,
 *     patch = 5x5x5 (or 5x5x1 with T = 1), 1 <= jump-flood step <= 4,
 *     lambda <= 130 (keeps the integer distance below 2^31).
 */
#ifndef VI_H
#define VI_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VI_OK = 0,
  VI_E_INVAL = -1,        /* bad argument (null pointer, size, parameter)      */
  VI_E_NOMEM = -2,        /* a device or host allocation failed                */
  VI_E_HIP = -3,          /* a HIP runtime call failed                          */
  VI_E_STATE = -4,        /* call out of order (e.g. reconstruct before search) */
  VI_E_EMPTY_SOURCE = -5, /* some level has no hole-free patch (D~ empty)       */
  VI_E_BUDGET = -6        /* a batch has no room for another context            */
} vi_status;

typedef enum { VI_RECON_WEIGHTED = 0, VI_RECON_MEAN = 1, VI_RECON_BEST = 2 } vi_recon_mode;

/* Method parameters; vi_params_default() fills the paper's values (Sec. 3.7). */
typedef struct {
  int32_t abi_version;  /* 1 */
  int32_t patch[3];     /* (x, y, t) patch size: {5, 5, 5} for videos (Sec. 3.7),
                           or {5, 5, 1} for a single image (T = 1): 2-D image
                           inpainting with the same method (Sec. 3.1, 3.5) */
  int32_t levels;       /* pyramid levels L >= 1 (Sec. 3.6) */
  int32_t lambda;       /* texture weight in the distance, 50 (Sec. 3.3, 3.7) */
  int32_t pm_iters;     /* PatchMatch iterations K, 10 (Sec. 3.1, 3.7) */
  int32_t n_jf;         /* synchronous propagation steps per iteration, 3 */
  int32_t jf_steps[8];  /* their strides, {4, 2, 1}; each in [1, 4] */
  double rho;           /* random-search window reduction, 0.5 (Eq. (3.1)) */
  int32_t em_max_iters; /* at most 20 iterations per level (Alg. 4) */
  double em_tol;        /* stop when the mean |change| per colour channel per
                           hole pixel is <= 0.1 (Sec. 3.7); < 0 runs exactly
                           em_max_iters iterations */
  int32_t recon_mode;   /* VI_RECON_WEIGHTED (Eqs. (3.2)-(3.3)) or
                           VI_RECON_MEAN (s = 1); used by every reconstruction
                           except the final one, which is VI_RECON_BEST */
  uint64_t seed;        /* key of the Philox4x64-10 random numbers */
  int32_t temporal_subsample; /* 0 (default): coarser levels keep every frame
                                 (Sec. 3.6); 1: each coarser level also halves
                                 the frame count (2x2x2 box means and
                                 OR-pooled occlusion, texture features taken
                                 at (2^l x, 2^l y, 2^l t), shift maps
                                 upsampled in time as in space), for objects
                                 that stay long behind the occlusion; the
                                 coarsest level must keep >= 5 frames */
  int32_t reduce_dims;  /* 0 (default): searches compare whole patches.
                           1..32: the dimensionality-reduced patch space that
                           Sec. 5 proposes as an acceleration: at creation
                           every level gets the reduce_dims leading principal
                           directions of its source patches (65536 sampled
                           sources, 32 steps of orthogonal iteration; see
                           vi_pca_basis), and the searches of the EM loop
                           compare those features (vi_set_reduction) */
  int32_t wide_pass_max; /* execution only, results do not depend on it:
                            -1 (default) lets the library choose; otherwise
                            the exact passes (the onion peel's included) over
                            at most this many targets compute each
                            candidate's distance with a group of eight lanes
                            (two round trips at most) instead of one lane
                            with early exit (0: never) */
} vi_params;

typedef struct vi_ctx vi_ctx; /* one clip: all its device state */

vi_status vi_params_default(vi_params* out /*(host)*/);

/* Creates a context for one clip and builds, on the GPU, the image and
 * occlusion pyramids (Alg. 4), the texture features and their pyramid
 * (Sec. 3.3, Eqs. (3.5), (3.7)) and the source set D~ and target set H~ of
 * every level (Sec. 2).
 *   video_rgb (dev) [T][H][W][3] uint8; values where mask = 1 are never read.
 *   mask      (dev) [T][H][W] uint8; nonzero = occluded (in H).
 *   hip_stream: hipStream_t used for all work of this context, or NULL for
 *   the default stream.
 * The inputs are copied; they may be released once the stream has passed
 * this call.  Syncs (set sizes are read back).
 * Errors: VI_E_INVAL (null pointer, unsupported parameter, volume too small
 * for the levels), VI_E_EMPTY_SOURCE, VI_E_NOMEM, VI_E_HIP. */
vi_status vi_create(vi_ctx** out, const vi_params* prm, int32_t W, int32_t H, int32_t T,
                    const uint8_t* video_rgb, const uint8_t* mask, void* hip_stream);

/* dims (host) = (W_l, H_l, T); counts (host) = (|H^l|, |H~^l|, |D~^l|). */
vi_status vi_level_info(const vi_ctx* ctx, int32_t level, int32_t dims[3], int64_t counts[3]);

/* Byte masks over the level volume (dev, [T][H_l][W_l] each, NULL skips):
 * hole H^l, sources D~^l, targets H~^l. */
vi_status vi_level_sets(const vi_ctx* ctx, int32_t level, uint8_t* hole, uint8_t* dsrc,
                        uint8_t* htil);

/* ANN search of the shift map on H~^level (Sec. 3.1, Alg. 1, Eq. (3.1)),
 * redesigned as synchronous propagation: targets without a valid match get a
 * uniform random source of D~; then K iterations of n_jf Jacobi propagation
 * passes (six axial neighbours at stride s) and one random-search draw per
 * target.  em_iter keys the random numbers (Philox counter word 1). */
vi_status vi_nnf_search(vi_ctx* ctx, int32_t level, int32_t em_iter);

/* Reconstruction of H^level (Sec. 3.2): mode VI_RECON_WEIGHTED (Eqs.
 * (3.2)-(3.3), sigma = nearest-rank 75th percentile), VI_RECON_MEAN or
 * VI_RECON_BEST (Eq. (3.4)).  Colour and texture are both rebuilt (Eq. (3.8)).
 *   out_f   (dev) [|H^l|][5] float in [0,1], hole voxels in ascending linear
 *           order, or NULL.
 *   absdiff (dev) one uint64 receiving sum over H^l of |new - old| over the
 *           three colour channels (the stopping test of Alg. 4), or NULL.
 * Without out_f, a weighted or plain reconstruction that follows one of the
 * same mode on the level recomputes only the pixels with a contributing
 * patch whose match, distance or count changed since; the others already
 * hold the value it would compute.
 * Errors: VI_E_STATE if the level has no complete shift map. */
vi_status vi_reconstruct(vi_ctx* ctx, int32_t level, int32_t mode, float* out_f,
                         uint64_t* absdiff);

/* The EM loop of one level (Alg. 4 inner loop).  em_iters_run (host) or
 * NULL.  Syncs once per iteration to read the stopping test, unless em_tol
 * < 0. */
vi_status vi_inpaint_level(vi_ctx* ctx, int32_t level, int32_t* em_iters_run);

/* Onion-peel initialisation of the coarsest level (Sec. 3.5, Alg. 3, Eqs.
 * (3.9)-(3.11)).  layers_run (host) or NULL.  Syncs once per layer. */
vi_status vi_onion_init(vi_ctx* ctx, int32_t* layers_run);

/* One layer of the onion peel (Sec. 3.5, Alg. 3), as vi_onion_init runs it,
 * for driving and testing the peel a layer at a time.
 *   Hp      (dev) [T][H_c][W_c] bytes of the coarsest level: the current
 *           occlusion H' on entry (nonzero = occluded), its erosion by the
 *           3x3x3 cube (outside the volume counted as occluded) on return.
 *   layer   keys the random numbers (step 2^32 + layer); layer 0 first
 *           empties the level's shift map.
 *   out_f   (dev) [|layer|][5] float in [0,1] receiving the reconstructed
 *           layer H' minus its erosion, in ascending linear order, or NULL.
 *   n_layer (host) receives the layer's size (0: H' was empty, nothing was
 *           searched), or NULL.
 * The layer's targets (voxels outside H' whose patch touches the layer) are
 * searched with the distance over the voxels outside H' (Eq. (3.10)), and
 * the layer is rebuilt from those contributors only (Eq. (3.11)).  Leaves the
 * level incomplete (vi_reconstruct refuses it until a full search).  Syncs.
 * Errors: VI_E_INVAL (null Hp, layer < 0), VI_E_STATE (clip in a batch). */
vi_status vi_onion_layer(vi_ctx* ctx, uint8_t* Hp, int32_t layer, float* out_f,
                         int64_t* n_layer);

/* vi_onion_layer for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same layer, the same kernels and results, but its work buffers live in a
 * fixed 16 MiB device array of the library (one per GPU, held until the
 * process ends) instead of memory allocated on the first call.  It calls no
 * allocator.  The coarsest level may hold at most 1 198 336 voxels;
 * larger levels return VI_E_BUDGET.  Every call on a GPU shares that GPU's
 * array: calls that overlap on one GPU (several host threads, or several
 * streams) race and must be serialised by the caller.  Timing records
 * (vi_profile) are not taken.  Arguments and other errors as
 * vi_onion_layer. */
vi_status vi_onion_layer_noalloc(vi_ctx* ctx, uint8_t* Hp, int32_t layer, float* out_f,
                                 int64_t* n_layer);

/* Level transition level+1 -> level (Sec. 3.6): nearest-neighbour upsampling
 * of the shift map and reconstruction of H^level with recon_mode. */
vi_status vi_transition(vi_ctx* ctx, int32_t level);

/* The complete algorithm (Alg. 4 without realignment): onion peel, EM loop
 * per level with transitions, final best-patch reconstruction.
 *   out_rgb (dev) [T][H][W][3]; voxels outside H equal the input.  Syncs. */
vi_status vi_inpaint(vi_ctx* ctx, uint8_t* out_rgb);

/* State of a level, for checkpointing and teacher-forced testing (dev
 * pointers, NULL skips):
 *   rgbt [T][H_l][W_l][5] uint8;  cand [..] int32 absolute linear index of
 *   the match, -1 outside H~ or unset;  dist [..] int32 integer SSD, -1
 *   outside H~;  nvox [..] uint8 number of compared voxels, 0 outside H~.
 * vi_set_state writes only hole voxels of rgbt and only H~ entries of the
 * map.  It syncs to validate cand first: if some cand is outside [-1, V) it
 * returns VI_E_INVAL and writes nothing, so the level keeps its previous
 * state.  After a write, the level counts as complete (vi_reconstruct
 * accepted) only if every H~ entry of cand is in D~ and, when nvox is given,
 * every H~ entry of nvox is nonzero. */
vi_status vi_get_state(const vi_ctx* ctx, int32_t level, uint8_t* rgbt, int32_t* cand,
                       int32_t* dist, uint8_t* nvox);
vi_status vi_set_state(vi_ctx* ctx, int32_t level, const uint8_t* rgbt, const int32_t* cand,
                       const int32_t* dist, const uint8_t* nvox);

/* Upper bound of the device bytes vi_create would hold for such a clip
 * (admission control).  Returns 0 for invalid arguments. */
size_t vi_footprint_bytes(const vi_params* prm, int32_t W, int32_t H, int32_t T,
                          double hole_fraction);

/* Device bytes this context holds. */
size_t vi_ctx_bytes(const vi_ctx* ctx);

/* Device memory released by destroyed contexts is kept by the library, per
 * device and size class, for the next vi_create (at most VI_POOL_BYTES bytes
 * per device, environment variable, default 8 GiB); a failed allocation
 * first gives the cache back and retries.  vi_pool_trim frees the cached
 * memory of the current device and returns the bytes freed. */
size_t vi_pool_trim(void);

/* Failure injection, for tests of the library's error handling (callers
 * that must see an exhausted device handled cleanly): after this call the
 * next n device allocations of contexts (the memory pool above) succeed and
 * every later one fails as an exhausted device would, so that the call
 * needing it returns VI_E_NOMEM; n < 0 turns the injection off.  Returns
 * the bytes of pool blocks held by live contexts at the time of the call,
 * so that a test can check that a failed call released what it took.
 * Process-wide; not for production use. */
int64_t vi_debug_fail_allocs(int64_t n);

/* Rebinds the context to another stream (hipStream_t or NULL). */
vi_status vi_set_stream(vi_ctx* ctx, void* hip_stream);

/* Frees everything the context owns; NULL-safe.  Syncs its stream. */
void vi_destroy(vi_ctx* ctx);

/* Thread-local message of the last error (never NULL). */
const char* vi_last_error(void);

/* Nominal patch-distance evaluations of one vi_nnf_search at a level:
 * |H~^l| * (1 + sum over iterations k of (6 n_jf + [floor(r_max rho^k) >= 1]))
 * (the initial evaluation, six neighbour candidates per propagation pass,
 * one random candidate per iteration).  Returns -1 on error. */
int64_t vi_nominal_evals(const vi_ctx* ctx, int32_t level);

/* Output of a finished clip (vi_inpaint done, or finished inside a batch):
 * out_rgb (dev) [T][H][W][3].  VI_E_STATE before the clip has finished.
 * Syncs. */
vi_status vi_output(vi_ctx* ctx, uint8_t* out_rgb);
/* 1 when the clip has completed the whole algorithm, else 0. */
int32_t vi_done(const vi_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Batches.  Many clips of uneven sizes and masks advance together: every
 * vi_batch_step runs one EM iteration (search + reconstruction, Alg. 4 inner
 * loop) of every member in the EM phase as one set of launches over all
 * members' targets and hole pixels — a captured HIP graph of persistent
 * kernels, or direct launches sized to the step (vi_tune); the onion peels
 * of members that start together run layer by layer as batched launches;
 * level transitions and final reconstructions of individual members run
 * between steps.  Each member's result is bit-identical to
 * vi_inpaint on that clip alone.  Members must share pm_iters and jf_steps
 * (n_jf >= 1).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t block;     /* targets per workgroup: 64, 128 or 256 */
  int32_t grid_mult; /* 1..64: persistent kernels, grid = compute units x grid_mult,
                        one captured graph per step; 0: one workgroup per chunk,
                        launched directly with grids sized to the step */
  int32_t tuned;     /* nonzero: use these values; zero: autotune at the first step */
} vi_tune;
typedef struct vi_batch vi_batch;

/* tune (host) or NULL: autotune on the first step (times one propagation
 * pass per candidate shape on the live batch, into scratch buffers).
 * hip_stream: stream for all batch work, or NULL for a stream of its own
 * (graph capture cannot use the legacy default stream). */
vi_status vi_batch_create(vi_batch** out, const vi_tune* tune, void* hip_stream);
/* Adds a clip that has not finished; its work moves to the batch's stream
 * while it is a member (vi_set_stream then returns VI_E_STATE).
 * VI_E_BUDGET when the batch holds 1024 clips; VI_E_INVAL when the clip is
 * already in this or another batch. */
vi_status vi_batch_add(vi_batch* b, vi_ctx* ctx);
/* Waits for the batch's queued work, removes the clip and gives it back the
 * stream it had before vi_batch_add.  vi_destroy of a member does the same
 * before freeing it. */
vi_status vi_batch_remove(vi_batch* b, vi_ctx* ctx);
/* One step of every member; n_done (host) receives the number of members
 * whose work has all been enqueued (their results are final once the stream
 * reaches this point; vi_output syncs).  Syncs once per step when some member
 * uses the stopping test (em_tol >= 0); otherwise only enqueues. */
vi_status vi_batch_step(vi_batch* b, int32_t* n_done);
vi_status vi_batch_get_tune(const vi_batch* b, vi_tune* out);
int32_t vi_batch_size(const vi_batch* b);
/* Frees the batch (not its members, which get their own streams back and
 * stay usable); NULL-safe.  Syncs the batch's stream. */
void vi_batch_destroy(vi_batch* b);

/* ---- Realignment of a video filmed by a moving camera (Sec. 3.4, Alg. 2;
 * the inverse warp of Alg. 4) ----
 * An affine map is 6 doubles m in pixel coordinates (x right, y down):
 * x' = m0 x + m1 y + m2, y' = m3 x + m4 y + m5.  The pipeline: estimate the
 * dominant motion of every frame pair, compose the maps to the reference
 * (middle) frame, warp the video and its occlusion to the reference frame,
 * inpaint the aligned video, unwarp its result into the original occlusion. */
typedef struct {
  int32_t levels; /* grey pyramid levels of the motion estimation, 3 */
  int32_t iters;  /* robust Gauss-Newton steps per level, 8 */
  double tukey_c; /* Tukey biweight constant in grey levels (0..255), 20 */
} vi_align_params;
vi_status vi_align_params_default(vi_align_params* out);
/* The dominant affine motion of every pair of successive frames (Alg. 2,
 * first loop; the robust estimator the paper borrows is written out as a
 * coarse-to-fine, Tukey-weighted Gauss-Newton fit of brightness constancy on
 * the grey level (R+G+B)/3 over the unoccluded pixels).
 *   rgb (dev) [T][H][W][3], mask (dev) [T][H][W] (nonzero = occluded,
 *   excluded), theta (host) [T-1][6]: theta_n maps frame n's pixels to their
 *   positions in frame n+1.  T >= 2; W, H >= 8 << (levels - 1) roughly (the
 *   coarsest estimation level must keep 8 x 8 pixels).  Syncs; allocates its
 *   working memory.  Errors: VI_E_INVAL, VI_E_NOMEM, VI_E_HIP. */
vi_status vi_align_estimate(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H,
                            int32_t T, const vi_align_params* prm, double* theta,
                            void* hip_stream);
/* Composition to the reference frame T/2 (0-based; Alg. 2, second loop):
 * M (host) [T][6], M_n maps frame n's pixels to the reference frame (the
 * identity for the reference; the inverse pair maps after it).  Host only.
 * Errors: VI_E_INVAL (null pointer, T < 1, a singular map). */
vi_status vi_align_compose(const double* theta, int32_t T, double* M);
/* The aligned video (Alg. 2, AffineWarp): pixel y of aligned frame n is
 * frame n sampled at M_n^-1(y) by bilinear interpolation in double
 * precision, rounded half up; out_mask (dev) [T][H][W] = 1 (and out_rgb 0)
 * where a neighbour of nonzero weight is outside the frame or occluded, so
 * the occlusion is warped with the video.  rgb, mask, out_rgb, out_mask
 * (dev); M (host) [T][6].  Syncs.  Errors: VI_E_INVAL (null pointer, sizes,
 * singular map), VI_E_HIP. */
vi_status vi_align_warp(const uint8_t* rgb, const uint8_t* mask, int32_t W, int32_t H,
                        int32_t T, const double* M, uint8_t* out_rgb, uint8_t* out_mask,
                        void* hip_stream);
/* The inverse (Alg. 4, last step): out_rgb (dev) = rgb, except every pixel
 * x of mask, which takes aligned (dev, the inpainted aligned video) sampled
 * at M_n(x), clamped to the frame, by bilinear interpolation.  Syncs.
 * Errors: VI_E_INVAL, VI_E_HIP. */
vi_status vi_align_unwarp(const uint8_t* aligned, const uint8_t* rgb, const uint8_t* mask,
                          int32_t W, int32_t H, int32_t T, const double* M, uint8_t* out_rgb,
                          void* hip_stream);

/* ---- Dimensionality-reduced patch space (Sec. 5) ----
 * Sec. 5 proposes dimensionality-reducing transformations of the patch space
 * to accelerate the method without fixing one.  Here: the patch vector x(p)
 * of a voxel lists, offset by offset (dt, dy, dx) of the patch, the channels
 * R, G, B, Tx, Ty of voxel p + o, its coordinates clamped to the volume
 * (dim = 5 x patch voxels: 625, or 125 for 5x5x1 patches).  A basis Q
 * [d][dim] of 16-bit integers (a linear map scaled by 256) defines the
 * features f_k(p) = floor((sum_i Q[k][i] x_i(p) + 128) / 256), and the
 * reduced distance sum_k (f_k(p) - f_k(c))^2 (saturated at 2^31 - 1).
 * With Q = rint(256 w_i b_ik), w = 1 on colour and sqrt(lambda) on texture
 * and b the principal directions of the weighted patch vectors, the reduced
 * distance approximates the patch distance (Secs. 2 and 3.3) with d instead
 * of dim coordinates.
 *
 * vi_set_reduction: the level's searches of the EM loop (vi_nnf_search,
 * vi_inpaint_level, vi_inpaint) compare reduced distances: each search first
 * computes the features of its targets on the current video (the sources'
 * patches never change at a level), and afterwards evaluates every target's
 * match with the exact distance, which the reconstruction uses.  The onion
 * peel keeps the exact partial distance.  Q (host) [d][dim]; d in [1, 32],
 * or 0 to return to the exact distance (Q unused).  Computes the features
 * of every voxel; syncs.  Contexts with a reduced level cannot join a batch.
 * Errors: VI_E_INVAL (d out of range, null Q, a row with
 * sum |Q[k][i]| x 255 + 128 >= 2^31), VI_E_STATE (the clip is in a batch),
 * VI_E_NOMEM. */
vi_status vi_set_reduction(vi_ctx* ctx, int32_t level, const int16_t* Q, int32_t d);

/* The features of every voxel of the level as last computed (after
 * vi_set_reduction: all voxels on the video of that moment; a search
 * refreshes its targets'): out (dev) [T][H][W][d] int32, d the level's
 * feature count (checked).  Enqueued.
 * Errors: VI_E_INVAL (null out, d not the level's count), VI_E_STATE (no
 * reduction at the level). */
vi_status vi_features(const vi_ctx* ctx, int32_t level, int32_t d, int32_t* out);

/* Exact moments of the patch vectors of every k-th source of the level (D~
 * in ascending linear order, k = ceil(|D~| / n_max), so n <= n_max samples):
 * S1 (host) [dim] sums, S2 (host) [dim][dim] sums of products.  Syncs.
 * n_max in [1, 2^20].  Errors: VI_E_INVAL, VI_E_NOMEM, VI_E_HIP. */
vi_status vi_pca_moments(vi_ctx* ctx, int32_t level, int32_t n_max, uint64_t* S1, uint64_t* S2,
                         int64_t* n);

/* The PCA basis of the level's source patches: from the moments above, the
 * covariance C_ij = (w_i w_j)(S2_ij / n - (S1_i / n)(S1_j / n)) of the
 * weighted vectors in double precision, then `iters` steps of orthogonal
 * iteration (d columns rounded up to a multiple of 4, fixed pseudo-random
 * start, orthonormalised by classical Gram-Schmidt applied twice after
 * every fourth product and after the last), and Q[k][i] =
 * rint(256 w_i b_ik) for the first d columns.  Q (host) [d][dim];
 * variance (host) [d] or NULL: b_k' C b_k, the variance each direction
 * captures.  Does not change the level's reduction.  Syncs.
 * d in [1, 32], n_max in [1, 2^20], iters in [0, 10000].
 * Errors: VI_E_INVAL, VI_E_STATE (the clip is in a batch), VI_E_NOMEM,
 * VI_E_HIP. */
vi_status vi_pca_basis(vi_ctx* ctx, int32_t level, int32_t d, int32_t n_max, int32_t iters,
                       int16_t* Q, double* variance);

/* ---- The textured-patch experiment (App. B) ----
 * App. B asks how likely a random patch V is to be closer to a random
 * reference patch W than the constant patch Z of the same mean, for white
 * noise of grey-level variance 25, and tabulates it for seven patch sizes.
 * This call counts the event: for every reference patch W_r and every
 * patch V lying wholly inside the grey volume,
 *   counts[r] = #{ V : SSD(W_r, V) < SSD(W_r, Z) },
 * Z the constant patch of value mu, SSD the sum of squared differences
 * over the patch's voxels (the patch distance of Sec. 2, one channel).
 *   ref    (dev) [n_ref][pt][ph][pw] uint8, voxels ordered dt, dy, dx
 *   vol    (dev) [T][H][W] uint8
 *   counts (dev) [n_ref] uint64, overwritten
 * pw * ph * pt in [1, 128]; mu in [0, 255]; W, H, T >= 1 with
 * W * H * T < 2^30; 0 <= n_ref < 2^24.  A volume smaller than the patch
 * has no candidates (every count 0); n_ref = 0 does nothing.  Runs on
 * hip_stream (NULL = the null stream) and syncs it; the references are
 * packed into n_ref x 132 bytes of device memory from the library's pool
 * for the duration of the call.  The reference-candidate inner products
 * run on the matrix cores (8-bit integer products, exact).
 * Errors: VI_E_INVAL (a null pointer with n_ref > 0, sizes out of range),
 * VI_E_NOMEM, VI_E_HIP. */
vi_status vi_closer_than_constant(const uint8_t* ref, int32_t n_ref, const uint8_t* vol,
                                  int32_t W, int32_t H, int32_t T, int32_t pw, int32_t ph,
                                  int32_t pt, int32_t mu, uint64_t* counts, void* hip_stream);

/* Work counters of a context since creation or the last reset (host out).
 * effective_evals is read back from the device: syncs. */
typedef struct {
  int64_t nominal_evals;   /* sum of the nominal counts of every search run */
  int64_t effective_evals; /* distances actually computed */
  int64_t searches;        /* searches run (EM iterations and onion layers) */
  int64_t em_iters;        /* EM iterations run (all levels) */
  int64_t recon_pixels;    /* hole pixels reconstructed (all reconstructions) */
  int64_t pass_evals;      /* of effective_evals: propagation and random-search passes */
  int64_t init_evals;      /* of effective_evals: step 0 of the EM-loop searches */
  int64_t onion_evals;     /* of effective_evals: onion-peel searches */
  int64_t pass_wide_evals; /* of pass_evals: passes of the wide form (see
                              vi_params.wide_pass_max) */
} vi_counters;
vi_status vi_get_counters(vi_ctx* ctx, vi_counters* out);
vi_status vi_reset_counters(vi_ctx* ctx);

/* Kernel timing with HIP events recorded on the context's stream while
 * profiling is on: one event pair around each launch, except the
 * propagation passes of one search, which run back to back and share one
 * pair (launches > 1; their average duration is ms / launches). */
typedef enum {
  VI_K_INIT = 0,   /* search step 0; units = targets */
  VI_K_PASS = 1,   /* propagation / random-search pass; units = targets x passes */
  VI_K_RECON = 2,  /* reconstruction; units = hole pixels */
  VI_K_OTHER = 3,  /* upsampling, copies; units = voxels */
  VI_K_ONION = 4,  /* any launch of the onion-peel initialisation */
  VI_K_PASS_WIDE = 5 /* VI_K_PASS in the wide form (small target lists, see
                        vi_params.wide_pass_max) */
} vi_kernel_kind;
typedef struct {
  int32_t kind;  /* vi_kernel_kind */
  int32_t level;
  int64_t units;
  float ms;
  int32_t launches; /* launches the record covers */
} vi_kernel_time;
/* kinds: bit mask of the vi_kernel_kind values timed (1 << kind), 0 = off */
#define VI_PROFILE_ALL 0x3F
vi_status vi_profile(vi_ctx* ctx, int32_t kinds);
/* Copies up to cap records (host) of the launches timed since the last read
 * and clears them; returns the number of records or a negative status.
 * Syncs. */
int32_t vi_profile_read(vi_ctx* ctx, vi_kernel_time* out, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif
