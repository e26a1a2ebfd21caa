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
 *     is current when the call is made; the library never frees caller memory.
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

#define SPDHG_MAX_SEG 64

#define SPDHG_OK 0
#define SPDHG_E_ARG (-1)       /* invalid argument (null pointer, out-of-range value)   */
#define SPDHG_E_SHAPE (-2)     /* inconsistent geometry / sizes                          */
#define SPDHG_E_DOMAIN (-3)    /* data outside the model's domain (b<0, r<0, mult<=0 ...) */
#define SPDHG_E_HIP (-4)       /* HIP runtime error                                      */
#define SPDHG_E_WORKSPACE (-5) /* workspace missing or too small                        */
#define SPDHG_E_STATE (-6)     /* call made on a context in the wrong state              */
#define SPDHG_E_NOTIMPL (-7)   /* option not implemented                                 */

/* Scanner / image geometry (a reading: the paper leaves the geometry to its projector
 * package).  Voxel centres (i - (n-1)/2) v per axis; angle a has phi = a pi / n_ang;
 * radial bin k sits at s = (k - (n_rad-1)/2) d_rad; segment g holds seg_planes[g] planes
 * with axial centres (p - (N_g-1)/2) vz and axial slope seg_tan[g] (mm of z per mm of
 * in-plane path); nz - seg_planes[g] must be even.  A ray is sampled at every image row
 * when 4a <= n_ang or 4a >= 3 n_ang, else at every column, and the image is interpolated
 * bilinearly (zero outside) in the other in-plane axis and z. */
typedef struct spdhg_geom {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    int32_t n_rad;
    double d_rad;
    int32_t n_ang;
    int32_t n_seg;
    int32_t seg_planes[SPDHG_MAX_SEG];
    double seg_tan[SPDHG_MAX_SEG];
} spdhg_geom;

#define SPDHG_PRIOR_NONE 0 /* ML: n = m blocks                                        */
#define SPDHG_PRIOR_TV 1   /* f_n = alpha ||.||_{2,1}, A_n = grad (eq. setting TV)      */
#define SPDHG_PRIOR_ATV 2  /* f_n = alpha ||.||_{1,1}, A_n = grad (Section 4.3, aTV)    */
#define SPDHG_PRIOR_DTV 3  /* f_n = alpha ||.||_{2,1}, A_n = D grad (Section 4.3)       */
#define SPDHG_PRIOR_TGV 4  /* x = (u, w): f_{n-1} = alpha ||.||_{2,1}, A_{n-1} = (grad, -I);
                            * f_n = alpha1 ||.||_{2,1}, A_n = (0, E) (eq. setting TGV)  */

#define SPDHG_SAMPLING_UNIFORM 0  /* p_i = 1/n (Section 4.2)                          */
#define SPDHG_SAMPLING_BALANCED 1 /* data 1/(2m) each, prior 1/2 (Section 4.2)        */

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
    int32_t reserved;
    double alpha1;     /* TGV: weight of ||E w|| (alpha is the weight of ||grad u - w||) */
} spdhg_params;

typedef struct spdhg_ctx spdhg_ctx;

/* Thread-local message describing the last failure (never NULL). */
const char* spdhg_last_error(void);

/* Number of bins of a geometry / of subset `subset` of `n_subsets` (-1: all angles). */
int64_t spdhg_subset_bins(const spdhg_geom* geom, int32_t n_subsets, int32_t subset);

/* y_out = A_i x for subset `subset` of `n_subsets` (Algorithm 2, dual step: the
 * projection of the current image), A_i = diag(mult) G restricted to the subset's rows.
 *   x       device, image, read only.
 *   mult    device, FULL sinogram of factors, or NULL for G alone.
 *   y_out   device, packed subset rows ([n_angles_of_subset][planes][radial]); subset -1
 *           means all angles (the full sinogram).  Overwritten.
 * FP32 arithmetic and accumulation.  Errors: SPDHG_E_ARG, SPDHG_E_SHAPE, SPDHG_E_HIP. */
int spdhg_project(const spdhg_geom* geom, int32_t n_subsets, int32_t subset,
                  const float* mult, const float* x, float* y_out, void* stream);

/* x_out = A_i^T y (Algorithm 2, backprojected dual change), the exact transpose of spdhg_project computed
 * by a voxel-driven gather with the same weights (deterministic, no atomics).
 *   y       device, packed subset rows as produced by spdhg_project, read only.
 *   mult    device, FULL sinogram of factors, or NULL.
 *   x_out   device, image, overwritten. */
int spdhg_backproject(const spdhg_geom* geom, int32_t n_subsets, int32_t subset,
                      const float* mult, const float* y, float* x_out, void* stream);

/* Number of nonzero entries of A_i (taps of the rays of subset `subset` that fall inside
 * the image with a nonzero interpolation weight), written to *out (host).  Measurement
 * helper: allocates a small scratch array, synchronises `stream`. */
int spdhg_nnz(const spdhg_geom* geom, int32_t n_subsets, int32_t subset, double* out,
              void* stream);

/* Bytes of device workspace a reconstruction needs (duals, z, step sizes, scratch). */
int spdhg_workspace_bytes(const spdhg_geom* geom, const spdhg_params* params, size_t* bytes);

/* Set up a reconstruction (Algorithm 2, inputs and initialisation):
 *   b, r, mult  device, full sinograms: counts b >= 0, background r >= 0, factors
 *               mult > 0.  Borrowed: they must stay valid until spdhg_destroy.
 *   side        device image (dTV side information) or NULL.  Borrowed.
 *   x           device image: initial image on entry (negative values are clipped, the
 *               first primal step with z = 0); the iterate is returned here after every
 *               spdhg_epoch / spdhg_iterate call.  Borrowed.
 *   ws          device workspace of at least spdhg_workspace_bytes(); owned by the
 *               caller, used by the library until spdhg_destroy.
 * Computes the step sizes of Theorem 2 (sensitivities A_i 1, A_i^T 1 or power
 * iterations), sets y = 0, z = 0.  Synchronises `stream` once (domain checks and norm
 * estimates come back to the host).  Errors: SPDHG_E_ARG, SPDHG_E_SHAPE,
 * SPDHG_E_DOMAIN (b < 0, r < 0, mult <= 0, or a bin with b > 0 and r = 0 that no voxel
 * reaches, whose objective term is infinite), SPDHG_E_WORKSPACE, SPDHG_E_HIP. */
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

/* The same iterations as spdhg_epoch (bitwise the same result), with each epoch's
 * launches recorded by stream capture into one HIP graph and launched as a graph (the
 * epoch is a fixed sequence of kernels once its random blocks are drawn).  Returns after
 * the stream has run the graphs (the graphs are then released).  Not with per-kernel
 * profiling on (SPDHG_E_STATE). */
int spdhg_epoch_graph(spdhg_ctx* ctx, int32_t n_epochs, void* stream);

/* Batched reconstructions: n independent problems (contexts from spdhg_init, each with
 * its own geometry, subsets, prior and workspace) each advance n_epochs of their own
 * epochs.  Problem i runs on worker stream i mod n_streams (at most 8, default priority)
 * forked from and joined back to `stream`, so the problems overlap on the GPU; every
 * problem's launches are exactly those of a solo spdhg_epoch (bitwise the same result).
 * use_graph != 0 records the whole forked batch epoch with stream capture into one HIP
 * graph and launches it (needs a non-default `stream`; returns after it has run);
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

/* Iterations per epoch and iterations done so far. */
int spdhg_info(const spdhg_ctx* ctx, int64_t* iters_per_epoch, int64_t* iters_done);

/* FP64 objective of an image (Problem 1): out_dev[0] = Psi, [1] = data term
 * sum_j phi_j((A x)_j) over all bins, [2] = prior term alpha R(x) (infinite if x has a
 * negative entry), [3] = reserved (0).  x = NULL means the current iterate.  out_dev
 * is device memory for 4 doubles.  Deterministic (fixed reduction order). */
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
 * Images are z-fastest ([y][x][z]) and sinograms [angle][radial][plane] inside the
 * library; *n_floats receives the element count (0 for an array the problem lacks). */
int spdhg_buffer(spdhg_ctx* ctx, int32_t which, float** ptr, int64_t* n_floats);

/* Step-size scalars: data sigma (scalar steps) of subset i, or the sigma of prior
 * block i - n_subsets, the probability p_i of block i and the operator norm used. */
int spdhg_block_info(const spdhg_ctx* ctx, int32_t i, double* sigma, double* p, double* norm);

/* Checkpoint: state = x, y, z, prior duals (TGV: also w, z_w) and the iteration counter (which fixes the
 * rest of the random block sequence).  spdhg_state_bytes gives the size; save writes it
 * to `dst` (device), load reads it back; both enqueue copies on `stream`. */
int spdhg_state_bytes(const spdhg_ctx* ctx, size_t* bytes);
int spdhg_save_state(spdhg_ctx* ctx, void* dst, size_t bytes, void* stream);
int spdhg_load_state(spdhg_ctx* ctx, const void* src, size_t bytes, void* stream);

/* Per-kernel timing of the iteration (HIP events recorded on the caller's stream around
 * each launch; adds no synchronisation inside spdhg_iterate).  spdhg_set_profiling turns
 * it on or off and clears the totals; spdhg_profile waits for the recorded events and
 * returns, per kernel kind (SPDHG_PROF_*), the summed milliseconds and launch counts. */
#define SPDHG_PROF_FWD 0   /* forward projection fused with the KL-dual prox          */
#define SPDHG_PROF_BWD 1   /* gather backprojection fused with the primal epilogue    */
#define SPDHG_PROF_PRIOR 2 /* prior dual update fused with its adjoint and epilogue    */
#define SPDHG_PROF_KINDS 3
int spdhg_set_profiling(spdhg_ctx* ctx, int32_t on);
int spdhg_profile(spdhg_ctx* ctx, double* ms, int64_t* launches);

/* Release the context (host memory only; caller memory is untouched). */
int spdhg_destroy(spdhg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SPDHG_H */
