/*
 * spdhg.h - C ABI of the MI355X (gfx950) SPDHG library for Poisson PET reconstruction
 * with non-smooth priors (Ehrhardt, Markiewicz, Schoenlieb, "Faster PET reconstruction
 * with non-smooth priors by randomization and preconditioning", arXiv:1808.07150).
 *
 * The library solves Problem 1 of the paper,
 *     min_u  sum_i D_i(P_i u) + alpha R(u) + i_+(u),
 * in the generic form of Problem 2 (sum_i f_i(A_i x) + g(x)) with the stochastic
 * primal-dual hybrid gradient method (Algorithm 2) and the scalar or preconditioned step
 * sizes of Theorem 2.  P = diag(mult) G, where G is a ray-driven Joseph projector for
 * parallel-beam rays with oblique planes (geometry below) and mult holds normalisation
 * times attenuation factors (Section 1.2: P "includes geometric factors, attenuation and
 * normalization").
 *
 * Conventions shared by every entry point
 *   - Every pointer argument documented as "device" is device memory on the device that
 *     is current when the call is made.  The library allocates no device memory: every
 *     scratch array lives in a caller-provided workspace (sized by the *_workspace_bytes
 *     queries, 256-byte aligned), and it never frees caller memory.
 *   - Images are float32 [nz][ny][nx] (x fastest); sinograms are float32
 *     [angle][plane][radial] (radial fastest).  Planes are ordered by segment
 *     0, +1, -1, +2, -2, ... and, inside a segment, by axial position.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every entry point
 *     only enqueues work on it and returns without synchronising, except where stated.
 *   - Status: 0 (SPDHG_OK) or a negative SPDHG_E_* code.  spdhg_last_error() returns a
 *     thread-local message for the last failing call.  Asynchronous kernel faults are
 *     reported by a later call.
 *   - Subsets are "equidistantly divided angles" (Section 4): with m subsets, subset i
 *     holds angles i, i+m, i+2m, ...  A subset's sinogram rows are packed as
 *     [angle of the subset][plane][radial] wherever a packed subset buffer is used.
 */
#ifndef SPDHG_H
#define SPDHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPDHG_MAX_SEG 128

#define SPDHG_OK 0
#define SPDHG_E_ARG (-1)       /* invalid argument (null pointer, out-of-range value)   */
#define SPDHG_E_SHAPE (-2)     /* inconsistent geometry / sizes                          */
#define SPDHG_E_DOMAIN (-3)    /* data outside the model's domain (b<0, r<0, mult<0 ...)  */
#define SPDHG_E_HIP (-4)       /* HIP runtime error                                      */
#define SPDHG_E_WORKSPACE (-5) /* workspace missing or too small                        */
#define SPDHG_E_STATE (-6)     /* call made on a context in the wrong state              */
#define SPDHG_E_NOTIMPL (-7)   /* option not implemented                                 */

/* Scanner / image geometry (a reading: the paper leaves the geometry to its projector
 * package).  Voxel centres (i - (n-1)/2) v per axis; angle a has phi = a pi / n_ang;
 * radial bin k sits at s = (k - (n_rad-1)/2) d_rad; segment g holds seg_planes[g] planes
 * with axial centres (p - (N_g-1)/2) pitch_g vz and axial slope seg_tan[g] (mm of z per
 * mm of in-plane path), where pitch_g = seg_pitch[g] is 1 (0 means 1: consecutive image
 * planes, e.g. span-11 data) or 2 (every other image plane: the ring pairs of span-1 data,
 * whose ring pitch is two image planes); nz - 1 - pitch_g (N_g - 1) must be even and
 * >= 0.  A ray is sampled at every image row when 4a <= n_ang or 4a >= 3 n_ang, else at
 * every column, and the image is interpolated bilinearly (zero outside) in the other
 * in-plane axis and z.
 *
 * Scanner model (Section 1.2: the system matrix "includes geometric factors"; all fields
 * zero = off).  det_radius: detector ring radius R (mm).  nonarc: radial bin k sits at
 * s = R sin((k - (n_rad-1)/2) d_rad / R) (bins not arc-corrected).  oblique_s: the slope
 * of segment g at radial position s is seg_tan[g] R / sqrt(R^2 - s^2) (a line of response
 * spans the chord between its two detectors), and so is its step length's.  span (odd,
 * >= 3): the segments must be the ring-pair segments of rings = (nz + 1) / 2 rings, ring
 * difference d = 0, +1, -1, +2, -2, ... with rings - |d| planes at pitch 2, and every
 * sinogram the library reads or writes (b, r, mult, subset and caller layouts) holds the
 * span-compressed data planes instead: data segment 0 takes |d| <= (span-1)/2, data
 * segment +-G the d in +-[G span - (span-1)/2, G span + (span-1)/2]; its plane of ring
 * sum S (from the segment's smallest ring sum G span - (span-1)/2, 0 for segment 0, up
 * to 2 (rings - 1) minus that) is the sum of the rays of the ring pairs (r1, r2) with
 * r1 + r2 = S, so G = C G1 with G1 the ring-pair projector and C the 0/1 sum.  The data
 * planes are ordered like segments (0, +1, -1, ...) and inside a segment by ring sum.
 * Detector gaps are zeros of mult (and of b, r). */
typedef struct spdhg_geom {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    int32_t n_rad;
    double d_rad;
    int32_t n_ang;
    int32_t n_seg;
    int32_t seg_planes[SPDHG_MAX_SEG];
    double seg_tan[SPDHG_MAX_SEG];
    int32_t seg_pitch[SPDHG_MAX_SEG];
    double det_radius; /* scanner model (see above): ring radius R, mm                 */
    int32_t nonarc;    /* 1: radial bins at R sin(...)                                  */
    int32_t oblique_s; /* 1: slopes seg_tan R / sqrt(R^2 - s^2)                         */
    int32_t span;      /* 0: data planes = the segments' planes; odd >= 3: compression  */
} spdhg_geom;

#define SPDHG_PRIOR_NONE 0 /* ML: n = m blocks                                        */
#define SPDHG_PRIOR_TV 1   /* f_n = alpha ||.||_{2,1}, A_n = grad (eq. setting TV)      */
#define SPDHG_PRIOR_ATV 2  /* f_n = alpha ||.||_{1,1}, A_n = grad (Section 4.3, aTV)    */
#define SPDHG_PRIOR_DTV 3  /* f_n = alpha ||.||_{2,1}, A_n = D grad (Section 4.3)       */
#define SPDHG_PRIOR_TGV 4  /* x = (u, w): f_{n-1} = alpha ||.||_{2,1}, A_{n-1} = (grad, -I);
                            * f_n = alpha1 ||.||_{2,1}, A_n = (0, E) (eq. setting TGV)  */

#define SPDHG_SAMPLING_UNIFORM 0  /* p_i = 1/n (Section 4.2)                          */
#define SPDHG_SAMPLING_BALANCED 1 /* data 1/(2m) each, prior 1/2 (Section 4.2)        */
#define SPDHG_SAMPLING_CUSTOM 2   /* a constant tuned distribution (Discussion): prior
                                   * blocks together p_prior, data (1 - p_prior)/m each;
                                   * TGV: block n gets p_tgv_n of p_prior (0: half)    */

#define SPDHG_FLAG_EM 1 /* also set up the EM-type updates of eq. OSEM (spdhg_em_iterate):
                          * m sensitivity images in the workspace */
#define SPDHG_FLAG_TGV_SPLIT_T 2 /* TGV: each prior block's scalar step caps only the
                                  * variables its operator acts on (block n = (0, E): w
                                  * only), instead of the minimum over all blocks for u and w
                                  * alike; Theorem 1 bounds ||S_i^1/2 A_i T^1/2|| per block,
                                  * and T_u does not enter block n's bound */
#define SPDHG_FLAG_COMPENSATED 4 /* hold the primal state x and z of Algorithm 2 as FP32
                                  * pairs (value + low part) and take the primal step in
                                  * FP64 on them, so that per-iteration changes below half
                                  * an FP32 ulp accumulate instead of being rounded away
                                  * (with many subsets, e.g. one angle each, they do); the
                                  * projector reads the FP32 value.  Costs 8 bytes per voxel
                                  * of workspace and 16 bytes per voxel of traffic per
                                  * iteration.  TV, aTV, dTV and no prior (SPDHG_E_NOTIMPL
                                  * with TGV); PDHG iterations use it too.  EM sub-iterations
                                  * (SPDHG_FLAG_EM) restart the iterate's low part at 0. */

typedef struct spdhg_params {
    int32_t n_subsets; /* m >= 1                                                      */
    int32_t prior;     /* SPDHG_PRIOR_*                                               */
    int32_t sampling;  /* SPDHG_SAMPLING_*                                            */
    int32_t precond;   /* 1: diagonal steps (eq. STEPSIZE:PRECOND), 0: scalar steps    */
    double alpha;      /* prior weight                                                */
    double eta;        /* dTV: xi = grad s / sqrt(|grad s|^2 + eta^2)                  */
    double gamma_d;    /* dTV: D = I - gamma_d xi xi^T                                 */
    double gamma;      /* step parameter gamma > 0 (the paper uses 1)                 */
    double rho;        /* step parameter 0 < rho < 1                                  */
    uint64_t seed;     /* SplitMix64 seed of the block sequence                        */
    int32_t power_iters; /* scalar steps: power iterations for ||A_i|| (e.g. 100)      */
    int32_t flags;       /* SPDHG_FLAG_* (0 for plain SPDHG)                            */
    double alpha1;     /* TGV: weight of ||E w|| (alpha is the weight of ||grad u - w||) */
    double p_prior;    /* SPDHG_SAMPLING_CUSTOM: total probability of the prior blocks   */
    double p_tgv_n;    /* SPDHG_SAMPLING_CUSTOM, TGV: probability of block n (0: half)   */
} spdhg_params;

typedef struct spdhg_ctx spdhg_ctx;

/* Thread-local message describing the last failure (never NULL). */
const char* spdhg_last_error(void);

/* Number of bins of a geometry / of subset `subset` of `n_subsets` (-1: all angles). */
int64_t spdhg_subset_bins(const spdhg_geom* geom, int32_t n_subsets, int32_t subset);

/* Bytes of device workspace the stand-alone operator calls below (spdhg_project,
 * spdhg_backproject, spdhg_nnz, spdhg_normalised_backprojection) need for `geom`, for any
 * subset: the geometry tables, two z-fastest images, the staging of 16 angles' sinogram
 * rows and FP64 partials over every bin.  The workspace is the caller's (e.g. a torch
 * uint8 tensor), 256-byte aligned; a call overwrites it, so calls that share one
 * workspace must be ordered (the same stream). */
int spdhg_op_workspace_bytes(const spdhg_geom* geom, size_t* bytes);

/* y_out = A_i x for subset `subset` of `n_subsets` (Algorithm 2, dual step: the
 * projection of the current image), A_i = diag(mult) G restricted to the subset's rows.
 *   x       device, image, read only.
 *   mult    device, FULL sinogram of factors, or NULL for G alone.
 *   y_out   device, packed subset rows ([n_angles_of_subset][planes][radial]); subset -1
 *           means all angles (the full sinogram).  Overwritten.
 *   ws      device workspace of at least spdhg_op_workspace_bytes() bytes.
 * FP32 arithmetic and accumulation.  Errors: SPDHG_E_ARG, SPDHG_E_SHAPE,
 * SPDHG_E_WORKSPACE, SPDHG_E_HIP. */
int spdhg_project(const spdhg_geom* geom, int32_t n_subsets, int32_t subset,
                  const float* mult, const float* x, float* y_out, void* ws, size_t ws_bytes,
                  void* stream);

/* spdhg_project for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same projection,
 * bitwise, with its scratch (geometry tables and the z-fastest copy of x) taken from a
 * fixed array inside the library instead of a caller workspace.  The array holds 64 MiB on
 * every GPU the library runs on, until the process ends: enough for the 344 x 344 x 127
 * mMR image; a geometry whose tables and image need more is rejected with
 * SPDHG_E_WORKSPACE before any GPU work.  The call allocates nothing.  Every call on one
 * GPU shares that GPU's array, so calls that overlap on one GPU (other streams or host
 * threads) race; calls ordered on one stream do not.  Arguments and errors as
 * spdhg_project. */
int spdhg_project_noalloc(const spdhg_geom* geom, int32_t n_subsets, int32_t subset,
                          const float* mult, const float* x, float* y_out, void* stream);

/* x_out = A_i^T y (Algorithm 2, backprojected dual change), the exact transpose of
 * spdhg_project computed by a voxel-driven gather with the same weights (deterministic,
 * no atomics).
 *   y       device, packed subset rows as produced by spdhg_project, read only.
 *   mult    device, FULL sinogram of factors, or NULL.
 *   x_out   device, image, overwritten.
 *   ws      device workspace of at least spdhg_op_workspace_bytes() bytes. */
int spdhg_backproject(const spdhg_geom* geom, int32_t n_subsets, int32_t subset,
                      const float* mult, const float* y, float* x_out, void* ws,
                      size_t ws_bytes, void* stream);

/* The normalised backprojection (A^T b) / (A^T 1) over all angles, 0 where A^T 1 = 0
 * (A^T 1 is the sensitivity of the EM-type update, eq. MLEM; A^T b / A^T 1 is the first
 * MLEM iterate from a constant image up to a factor):
 *   b, mult     device, full sinograms (counts, factors), read only.
 *   out         device image, overwritten.
 *   stats_dev   device, 3 doubles: [sum, count, count / sum] of the positive voxels of
 *               out (the last is the scale that brings their mean to 1; 1 if none).
 *   ws          device workspace of at least spdhg_op_workspace_bytes() bytes. */
int spdhg_normalised_backprojection(const spdhg_geom* geom, const float* b, const float* mult,
                                    float* out, double* stats_dev, void* ws, size_t ws_bytes,
                                    void* stream);

/* Number of nonzero entries of A_i (taps of the rays of subset `subset` that fall inside
 * the image with a nonzero interpolation weight), written to *out (host).  Measurement
 * helper: uses the operator workspace `ws` and synchronises `stream`. */
int spdhg_nnz(const spdhg_geom* geom, int32_t n_subsets, int32_t subset, double* out,
              void* ws, size_t ws_bytes, void* stream);

/* Bytes of device workspace a reconstruction needs (duals, z, step sizes, scratch). */
int spdhg_workspace_bytes(const spdhg_geom* geom, const spdhg_params* params, size_t* bytes);

/* Set up a reconstruction (Algorithm 2, inputs and initialisation):
 *   b, r, mult  device, full sinograms: counts b >= 0, background r >= 0, factors
 *               mult >= 0 (0: a bin of zero efficiency, e.g. a detector gap, whose row of
 *               A is zero).  Borrowed: they must stay valid until spdhg_destroy.
 *   side        device image (dTV side information) or NULL.  Borrowed.
 *   x           device image: initial image on entry (negative values are clipped, the
 *               first primal step with z = 0); the iterate is returned here after every
 *               spdhg_epoch / spdhg_iterate call.  Borrowed.
 *   ws          device workspace of at least spdhg_workspace_bytes(); owned by the
 *               caller, used by the library until spdhg_destroy.
 * Computes the step sizes of Theorem 2 (sensitivities A_i 1, A_i^T 1 or power
 * iterations), sets y = 0, z = 0.  Synchronises `stream` once (domain checks and norm
 * estimates come back to the host).  Errors: SPDHG_E_ARG, SPDHG_E_SHAPE,
 * SPDHG_E_DOMAIN (b < 0, r < 0, mult < 0, or a bin with b > 0 and r = 0 that no voxel
 * reaches (or with mult = 0), whose objective term is infinite), SPDHG_E_WORKSPACE, SPDHG_E_HIP. */
int spdhg_init(spdhg_ctx** out, const spdhg_geom* geom, const spdhg_params* params,
               const float* b, const float* r, const float* mult, const float* side,
               float* x, void* ws, size_t ws_bytes, void* stream);

/* Run n_iters iterations of Algorithm 2: draw block i (SplitMix64, probabilities of
 * `sampling`), dual prox of block i, backprojection of the dual change, extrapolation
 * z_bar = z + dz / p_i and the primal prox max(x - T z_bar, 0).  x holds the iterate
 * after the last primal step when the enqueued work completes. */
int spdhg_iterate(spdhg_ctx* ctx, int64_t n_iters, void* stream);

/* n_epochs epochs; an epoch is m / sum_{i<=m} p_i iterations (Section 4: the number of
 * iterations that in expectation use all data once). */
int spdhg_epoch(spdhg_ctx* ctx, int32_t n_epochs, void* stream);

/* The same iterations as spdhg_epoch (bitwise the same result), launched as a persistent
 * HIP graph: the context's own spdhg_graph (below), built on the first call and kept until
 * spdhg_destroy or a change of the tuning or walk.  Asynchronous on `stream` like
 * spdhg_epoch (the graph's two executable copies alternate; the host waits for a copy's
 * previous run before rewriting its arguments).  Not with per-kernel profiling on
 * (SPDHG_E_STATE). */
int spdhg_epoch_graph(spdhg_ctx* ctx, int32_t n_epochs, void* stream);

/* Persistent epoch graph of one or more problems (Algorithm 2's epochs of independent
 * reconstructions, of any sizes and subset counts, in one HIP graph): per problem a chain
 * of kernel nodes, one group per iteration slot of an epoch, each group holding every
 * kernel an iteration of any block could launch in that slot (then the end of the epoch).
 * The graph is instantiated once.  spdhg_graph_epoch draws each problem's blocks on the
 * host exactly as spdhg_epoch does, writes the arguments of the resulting launches into the
 * matching nodes, disables the others and launches the graph on `stream`: every problem
 * advances one epoch per graph launch, bitwise as in a solo spdhg_epoch.  The contexts must
 * outlive the graph; an eager call on a context between graph epochs is ordered by the
 * stream like any other.  Not with per-kernel profiling on (SPDHG_E_STATE). */
typedef struct spdhg_graph spdhg_graph;
int spdhg_graph_create(spdhg_ctx* const* ctxs, int32_t n, spdhg_graph** out);
int spdhg_graph_epoch(spdhg_graph* graph, int32_t n_epochs, void* stream);
int spdhg_graph_destroy(spdhg_graph* graph);

/* Batched reconstructions: n independent problems (contexts from spdhg_init, each with
 * its own geometry, subsets, prior and workspace) each advance n_epochs of their own
 * epochs.  Problem i runs on worker stream i mod n_streams (at most 8, default priority)
 * forked from and joined back to `stream`, so the problems overlap on the GPU; every
 * problem's launches are exactly those of a solo spdhg_epoch (bitwise the same result).
 * use_graph != 0 runs the n_epochs batch epochs as one persistent spdhg_graph over the
 * problems (built, launched n_epochs times, released; returns after it has run);
 * otherwise the call is asynchronous on `stream`.  A context may appear once. */
int spdhg_batch_epoch(spdhg_ctx* const* ctxs, int32_t n, int32_t n_epochs, int32_t n_streams,
                      int32_t use_graph, void* stream);

/* Ray-bundle tiling of the subset projection: wavefronts per (angle, radial bin) bundle,
 * splitting its primary steps (1, 2, 4 or 8) or its planes (20: two wavefronts, 40: four;
 * at most 1024 planes per wavefront); 0 = chosen from the launch size.  spdhg_autotune times each choice on
 * the subset-0 projection of the current image (no state changes) and keeps the fastest;
 * *fwd_split and *ms receive the choice and its time per launch. */
int spdhg_set_tuning(spdhg_ctx* ctx, int32_t fwd_split);
int spdhg_autotune(spdhg_ctx* ctx, int32_t* fwd_split, double* ms, void* stream);

/* Ray-to-lane mapping of the forward walk (the projection of Section 4.1, every mode):
 * 0 (default) = runs of 15 consecutive planes of one segment per lane where the geometry
 * allows it (more than 256 planes, all segments on consecutive image planes, at most 64
 * such runs, e.g. the 837 planes of span 11), else interleaved; 1 = always interleaved (plane q on lane q mod 64).
 * Both give bitwise identical projections; runs read the LDS column once per run instead
 * of once per ray.  SPDHG_E_ARG for other values. */
int spdhg_set_walk(spdhg_ctx* ctx, int32_t interleave);

/* Tiling of the gather backprojection: 1 = strips of 10 voxel columns along the secondary
 * axis (for 32 <= nz <= 127, one plane pitch and tap tables within one workgroup's LDS),
 * one strip per workgroup; 3 = the same strips, those of four consecutive primary indices
 * in one workgroup (they read nearly the same rays through one L1); 2 = groups of whole
 * voxel columns (any geometry); 0 = the automatic choice (strips where they apply).
 * Tilings 1 and 3 give bitwise identical results.  spdhg_autotune also times each on the
 * subset-0 backprojection and keeps the fastest; spdhg_get_tuning reports the split and
 * the gather in use (1, 2 or 3). */
int spdhg_set_gather(spdhg_ctx* ctx, int32_t gather);
int spdhg_get_tuning(const spdhg_ctx* ctx, int32_t* fwd_split, int32_t* gather);

/* n_iters iterations of deterministic PDHG (Algorithm 1): every block's dual step from the
 * same x, the backprojected dual changes summed, z += dz, extrapolation z_bar = z + dz and
 * the primal step max(x - T z_bar, 0).  Needs a context with one data block (n_subsets =
 * 1, else SPDHG_E_STATE); its step sizes are those of Theorem 2 with the context's block
 * probabilities in the role of the weights that sum to 1 (1/2 data, 1/2 prior; 1 for ML),
 * which the convergence condition of PDHG with several blocks needs.  TV, aTV, dTV and
 * no prior (TGV: SPDHG_E_NOTIMPL).  The reference minimiser of the relative objective
 * (Section 4: 5,000 PDHG iterations) is computed with it.  Asynchronous on `stream`. */
int spdhg_pdhg_iterate(spdhg_ctx* ctx, int64_t n_iters, void* stream);

/* EM-type sub-iterations (eq. MLEM; eq. OSEM with the context's m subsets, visited in
 * the order 0, 1, ..., m - 1, continuing where the previous call stopped): on subset i,
 *     x = x / (A_i^T 1) * A_i^T (b_i / (A_i x + r_i)),
 * with b / (.) taken as 0 on bins with b = 0 and x = 0 where A_i^T 1 = 0.  With m = 1 this
 * is MLEM.  Acts on the context's image only (the SPDHG duals are left as they are); the
 * image is returned in the caller's x as after spdhg_iterate.  EM keeps zero voxels at
 * zero, so start it from a positive image.  Needs a context set up with SPDHG_FLAG_EM
 * (else SPDHG_E_STATE).  Asynchronous on `stream`. */
int spdhg_em_iterate(spdhg_ctx* ctx, int64_t n_subiters, void* stream);

/* Iterations per epoch and iterations done so far. */
int spdhg_info(const spdhg_ctx* ctx, int64_t* iters_per_epoch, int64_t* iters_done);

/* FP64 objective of an image (Problem 1): out_dev[0] = Psi, [1] = data term
 * sum_j phi_j((A x)_j) over all bins, [2] = prior term alpha R(x) (infinite if x has a
 * negative entry), [3] = the failure flag: the number of non-finite voxels of x (for the
 * current TGV iterate, of u and w), 0 for a healthy iterate.  x = NULL means the current
 * iterate.  out_dev is device memory for 4 doubles.  Deterministic (fixed reduction
 * order). */
int spdhg_objective(spdhg_ctx* ctx, const float* x, double* out_dev, void* stream);

/* Duality gap of the current state (x, y) for the problem with g = indicator of [0, U]
 * (U above the largest value of a minimiser, so both problems share it; with g = the
 * non-negativity indicator alone, g* of -A^T y is infinite at almost every iterate):
 *   gap = Psi(x) + sum_i f_i*(y_i) + U sum_v max(0, -(A^T y)_v)
 * (Problem "Generic Saddle Point Problem", Theorem "Convergence"; f_i* of the data blocks
 * is eq. PET:CVX, of the prior blocks the indicator of the dual ball).  Rows with
 * (A 1)_j = 0 are left out of Psi (they are constants).  A^T y is the iterate's z, which
 * Algorithm 2 maintains.  out_dev (device, 4 doubles) = [gap, Psi over the rows reached,
 * sum f_i*(y_i) (+inf for an infeasible prior dual), U-term].  Not defined for TGV
 * (SPDHG_E_NOTIMPL).  Asynchronous on `stream`. */
int spdhg_gap(spdhg_ctx* ctx, double U, double* out_dev, void* stream);

/* Device pointers of internal arrays (for inspection and checkpoints):
 *   0 y (full sinogram)   1 z (image)   2 T (image)   3 sigma (full sinogram, or NULL
 *   with scalar steps)   4 prior dual (3 images, current buffer; TGV: q1)
 *   5 TGV w (3 images)   6 TGV q2 (6 images)   7 TGV z_w (3 images)
 *   8 low part of z   9 low part of the iterate
 *   (SPDHG_FLAG_COMPENSATED: the state is the sum of the two parts)
 * Images are z-fastest ([y][x][z]) and sinograms [angle][radial][plane] inside the
 * library; *n_floats receives the element count (0 for an array the problem lacks). */
int spdhg_buffer(spdhg_ctx* ctx, int32_t which, float** ptr, int64_t* n_floats);

/* Step-size scalars: data sigma (scalar steps) of subset i, or the sigma of prior
 * block i - n_subsets, the probability p_i of block i and the operator norm used. */
int spdhg_block_info(const spdhg_ctx* ctx, int32_t i, double* sigma, double* p, double* norm);

/* Checkpoint: state = x, y, z, prior duals (TGV: also w, z_w; SPDHG_FLAG_COMPENSATED: also
 * the low parts of z and x) and the iteration counter (which fixes the
 * rest of the random block sequence).  spdhg_state_bytes gives the size; save writes it
 * to `dst` (device), load reads it back; both enqueue copies on `stream`. */
int spdhg_state_bytes(const spdhg_ctx* ctx, size_t* bytes);
int spdhg_save_state(spdhg_ctx* ctx, void* dst, size_t bytes, void* stream);
int spdhg_load_state(spdhg_ctx* ctx, const void* src, size_t bytes, void* stream);

/* Per-kernel timing of the iteration (HIP events recorded on the caller's stream around
 * each launch; adds no synchronisation inside spdhg_iterate).  spdhg_set_profiling turns
 * it on or off and clears the totals; spdhg_profile waits for the recorded events and
 * returns, per kernel kind (SPDHG_PROF_*), the summed milliseconds and launch counts.
 * spdhg_set_profiling_kinds limits the timing to the kinds whose bit (1 << SPDHG_PROF_*)
 * is set in `mask` (default: every kind), for launches enqueued after the call: each
 * event pair costs the stream a few microseconds, so timing one kind disturbs the
 * others less.  SPDHG_E_ARG for a mask without a kind or with other bits. */
#define SPDHG_PROF_FWD 0   /* forward projection fused with the KL-dual prox          */
#define SPDHG_PROF_BWD 1   /* gather backprojection fused with the primal epilogue    */
#define SPDHG_PROF_PRIOR 2 /* prior dual update fused with its adjoint and epilogue    */
#define SPDHG_PROF_KINDS 3
int spdhg_set_profiling(spdhg_ctx* ctx, int32_t on);
int spdhg_set_profiling_kinds(spdhg_ctx* ctx, int32_t mask);
int spdhg_profile(spdhg_ctx* ctx, double* ms, int64_t* launches);

/* Release the context (host memory only; caller memory is untouched). */
int spdhg_destroy(spdhg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SPDHG_H */
