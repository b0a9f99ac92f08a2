/*
 * tt.h -- C ABI of the MI355X tensor-tomography hot path.
 *
 * The library computes the linear forward model of SAXS/WAXS tensor
 * tomography of Nielsen et al. ("Mumott", section 2, Eqs. projection_matrix,
 * real_space_geom, projection_operator and forward_model),
 *
 *     I_sjkc = sum_xyz P_{sjk,xyz} sum_i B_{sc,i} c_xyzi        (I = A c),
 *
 * its exact adjoint, the squared loss with L2 regularisation of
 * Eq. opt_prob_general_form and its gradient, and an L-BFGS driver
 * (section 3.5, "Optimization"), all on one gfx950 GPU.
 *
 * Discretisation (the paper leaves it open): P_{sjk,xyz} is unit-step ray
 * sampling with trilinear weights and zero padding, samples at
 * x_n = u_jk + n * step * d_s for integer n, each weighted by step; voxel and
 * detector grids are centred on the rotation centre.  B_{sc,i} is the mean of
 * the real even-order spherical harmonic Y_i(R_s^T q(phi)) over n_sub
 * midpoint nodes of segment c, with the small-angle q(phi) of Eq. 1.
 *
 * Conventions for every call:
 *  - Layouts are row-major, float32 unless stated:
 *      coefficients c[nx][ny][nz][C],  C = (ell_max/2 + 1)(ell_max + 1),
 *      data / residual I[n_proj][nj][nk][n_seg],
 *      basis constants B[n_proj][n_seg][C] (float64, host).
 *    Coefficient index i(l, m) = l(l-1)/2 + l + m for even l, m = -l..l.
 *  - Pointers named *_dev are device pointers on the context's device; the
 *    caller allocates and owns them, work buffers included (tt_set_workspace,
 *    tt_lbfgs_create, tt_kappa, ...).  A context owns only its geometry tables
 *    (ray frames and basis constants, allocated once by tt_create); no call
 *    after tt_create allocates device memory.
 *  - Device work is enqueued on the context's stream (tt_set_stream) and is
 *    asynchronous unless stated otherwise.  A context must not be used from
 *    two host threads at once.
 *  - Every int-returning call returns TT_OK (0) or a negative TT_E* code and
 *    never aborts; tt_error_string() names the code and tt_last_error() gives
 *    the message of the most recent failure on the calling thread.
 */
#ifndef TT_H
#define TT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TT_OK = 0,
    TT_EINVAL = -1,       /* null pointer or out-of-range argument */
    TT_ESHAPE = -2,       /* inconsistent sizes */
    TT_ENOMEM = -3,       /* device or host allocation failed */
    TT_EHIP = -4,         /* a HIP runtime call failed */
    TT_ENONFINITE = -5,   /* a reduction produced NaN or Inf */
    TT_EUNSUPPORTED = -6  /* valid but not implemented (e.g. ell_max > 16) */
};

/* Precision of the coefficient-to-segment mapping. */
enum { TT_MAP_FP32 = 0, TT_MAP_BF16 = 1 };

/* Acquisition geometry (section 2, Table tab:geometry_vectors and
 * Eq. real_space_geom).  Angle and offset arrays are host pointers read
 * during tt_create only. */
typedef struct tt_geometry {
    int32_t nx, ny, nz;         /* volume shape, unit voxels (a = b = 1) */
    int32_t ell_max;            /* even, 0..16 (tt_create: 0..12) */
    int32_t n_proj;             /* number of goniometer settings s */
    int32_t nj, nk;             /* raster (detector pixel) grid */
    int32_t n_seg;              /* azimuthal detector segments, 1..64 */
    int32_t n_sub;              /* midpoint nodes per segment (>= 1) */
    int32_t map_precision;      /* TT_MAP_FP32 or TT_MAP_BF16 */
    double step;                /* ray sample spacing in voxels (> 0) */
    double seg_span;            /* angle covered by the segments: 2 pi (WAXS) or pi */
    const double *inner_angle;  /* alpha_s [rad], length n_proj */
    const double *outer_angle;  /* beta_s [rad], length n_proj */
    const double *j_offset;     /* delta j_s, length n_proj, or NULL for 0 */
    const double *k_offset;     /* delta k_s, or NULL */
    double p[3], j[3], k[3];    /* beam and raster directions, lab frame */
    double q0[3], q90[3];       /* detector azimuth origin and +90 deg */
    double alpha_axis[3];       /* inner (rotation) stage axis */
    double beta_axis[3];        /* outer (tilt) stage axis */
    /* Basis set of the per-voxel functions (sect. 3.3 "Basis sets"); zero
     * (TT_BASIS_SH) selects the real spherical harmonics up to ell_max.  The
     * kernel bases put one function on each of n_dirs grid directions
     * dirs[n_dirs][3] (host, normalised internally), C = n_dirs <= 96:
     *   TT_BASIS_GK: Gaussian kernels exp(-w^2 / (2 kernel_width^2)), w the
     *                angle between q and the nearer of +-dir (radians);
     *   TT_BASIS_NN: nearest neighbour, 1 on the directions q closer to +-dir
     *                than to any other grid direction (ties to the lower
     *                index), 0 elsewhere.
     * Both are antipodally symmetric.  ell_max is ignored for them. */
    int32_t basis;
    int32_t n_dirs;
    const double *dirs;
    double kernel_width;
} tt_geometry;

#define TT_BASIS_SH 0
#define TT_BASIS_GK 1
#define TT_BASIS_NN 2

typedef struct tt_ctx tt_ctx;

/* Build a context on the current HIP device: validates the geometry, computes
 * R_s = R_beta(beta_s) R_alpha(alpha_s), the ray frames and B_{sc,i} in
 * float64 on the host and uploads them as device tables (the only device
 * memory the library allocates).  Device computations need a workspace
 * (tt_set_workspace) first.  Synchronous.  On failure *out is NULL. */
/* TT_EUNSUPPORTED for ell_max > 12, more than 16 distinct segments, or a
 * projection image of 2^24 or more float4 groups (nj nk ceil(U/4) with U the
 * distinct segments rounded up to 4, 8 or 16). */
int tt_create(const tt_geometry *geom, tt_ctx **out);
/* Waits for the context's stream, then frees its tables and buffers. */
void tt_destroy(tt_ctx *ctx);

/* Stream for all later device work of this context (a hipStream_t; NULL is
 * the default stream). */
int tt_set_stream(tt_ctx *ctx, void *hip_stream);

/* Select TT_MAP_FP32 or TT_MAP_BF16 for tt_project / tt_adjoint. */
int tt_set_map_precision(tt_ctx *ctx, int precision);

/* Sparse fused forward (sect. "Pipelines": the sparse variant of the
 * asynchronous pipelines applies a sparse approximation of the
 * reciprocal-space map inside the ray-sum kernel, so the intermediate between
 * the two mappings is never stored; it saves memory rather than time unless
 * the map is very sparse).
 *   k = 0 (default): the exact constants B_{sc,i}; tt_project maps a batch of
 *     projections into the workspace (M_s = B_s c) and ray-sums it.
 *   k >= 1: in every row (projection s, segment c) of B only the k entries of
 *     largest magnitude are kept and the others set to zero (taken one at a
 *     time: the largest remaining magnitude m, then the lowest remaining basis
 *     index with |B| >= m - 1e-9 max|row|; k >= C keeps B whole); tt_project
 *     runs one fused kernel for all projections that forms the unique segment
 *     values sum_t B_{sc,i_t} c_{v,i_t} of each voxel while staging the
 *     coefficient volume for the ray sums (no mapped volumes in the
 *     workspace).  When no projection keeps more than 32 basis functions over
 *     its unique segments, tt_project first copies c channel-major into the
 *     workspace (C x nx ny nz floats) and the staging reads only the kept
 *     channels; otherwise it reads the coefficient records.  tt_adjoint,
 *     tt_loss_grad, the solver, tt_kappa and tt_basis_matrix use the same
 *     approximated constants, so the pair stays exactly adjoint.  The
 *     constants are rebuilt on the host and uploaded (synchronous; waits for
 *     the context's stream).  A call that changes the workspace layout
 *     (between k = 0 and k >= 1, or across the channel-major threshold)
 *     releases the attached workspace: attach one sized by tt_workspace_bytes
 *     in the new mode before computing.
 * Both projector models (tt_set_projector) run fused.  TT_EINVAL for k < 0;
 * TT_EUNSUPPORTED for k >= 1 with the bf16 map tier (and tt_set_map_precision
 * returns TT_EUNSUPPORTED for it while a sparse map is set). */
int tt_set_sparse_map(tt_ctx *ctx, int k);

/* Discretisation of the projection operator P_{sjk,xyz} (Eq. projection_operator):
 *   TT_PROJ_TRILINEAR (default): samples every `step` voxels along the ray,
 *     trilinear (tent) weights, each sample weighted by `step`;
 *   TT_PROJ_JOSEPH: Joseph's method, the paper's own projector (sect. 3.5):
 *     the ray is cut by every voxel-centre plane normal to its dominant axis A
 *     (ties within 1e-9 go to the lower axis), the field is interpolated
 *     bilinearly in the two other axes at each cut, and each cut is weighted
 *     by 1/|d_A|; `step` is not used.
 * tt_project, tt_adjoint, tt_loss_grad and the solver use the selection made
 * before they are called (exact transposes of each other in both models).
 * TT_EINVAL for another value. */
#define TT_PROJ_TRILINEAR 0
#define TT_PROJ_JOSEPH 1
int tt_set_projector(tt_ctx *ctx, int model);

/* Number of real even-order SH coefficients up to ell_max (or TT_EINVAL). */
int tt_num_coeffs(int ell_max);

/* Sizes of this context: out8 = {nx*ny*nz*C, n_proj*nj*nk*n_seg, C,
 * unique segments, projections per forward batch (0 before tt_set_workspace),
 * attached workspace bytes, bytes of the context's own tables, bytes of one
 * projection's mapped volume}. */
int tt_sizes(const tt_ctx *ctx, int64_t *out8);

/* Workspace of a context: float64 reduction partials, the antipodally folded
 * adjoint input (n_proj nj nk U floats), a data-sized residual scratch and
 * the coefficient-to-segment maps M_s = B_s c of one batch of projections
 * ((nx+2)(ny+2)(nz+2) U floats each, zero border).  The forward evaluates
 * Eq. forward_model batch by batch: a larger batch reads c fewer times.
 * tt_workspace_bytes gives the bytes for a batch of forward_batch projections
 * (rounded to what the map kernel accepts; forward_batch = 1 gives the
 * smallest valid workspace, >= n_proj the whole set in one batch;
 * forward_batch <= 0 gives the workspace without mapped volumes, which serves
 * only the fused forward of tt_set_sparse_map; with a sparse map of at most 32
 * kept basis functions per projection the workspace also holds a
 * channel-major copy of c, nx ny nz C floats).
 * tt_set_workspace attaches caller memory (device, 256-byte aligned) and
 * picks the largest batch that fits; TT_EINVAL below the smallest size (with
 * a sparse map set, below the size without mapped volumes).  The
 * memory must stay allocated and untouched by the caller while attached; the
 * zero border is written once, on the context's stream.  Calls that compute
 * (tt_project, tt_adjoint, tt_loss_grad, the solver, tt_kappa,
 * tt_voxel_preconditioner) return TT_EINVAL without a workspace. */
int64_t tt_workspace_bytes(const tt_ctx *ctx, int forward_batch);
int tt_set_workspace(tt_ctx *ctx, void *work_dev, size_t bytes);

/* Host-only: *out = the number of ray samples (trilinear model) or plane cuts
 * (Joseph's method) of all projections that touch the volume, i.e. the sample
 * positions whose trilinear (bilinear) stencil meets at least one voxel.  Each
 * touches up to 8 (4) voxels; the count sizes the arithmetic of the forward
 * ray sums and of the adjoint's gather. */
int tt_ray_samples(const tt_ctx *ctx, int64_t *out);

/* Copy B_{sc,i} (Eq. projection_matrix) to the host: B[n_proj][n_seg][C]. */
int tt_basis_matrix(const tt_ctx *ctx, double *B_host);

/* Host-only: B_{sc,i} for a geometry without creating a context (no device
 * work).  B_host[n_proj][n_seg][C]. */
int tt_geometry_basis(const tt_geometry *geom, double *B_host);

/* Host-side evaluation of the real even-order spherical harmonics (section
 * 3.2) at n directions dirs[n][3] (need not be unit length):
 * out[n][C].  No device work. */
int tt_sh_eval(int ell_max, int64_t n, const double *dirs, double *out);

/* Forward model (Eq. forward_model): I_dev = A c_dev.  Layouts as above.
 * Overwrites I_dev. */
int tt_project(tt_ctx *ctx, const float *c_dev, float *I_dev);

/* Adjoint: g_dev = A^T y_dev + beta * c_dev (c_dev may be NULL when
 * beta == 0).  y_dev has the data layout, g_dev and c_dev the coefficient
 * layout.  Overwrites g_dev. */
int tt_adjoint(tt_ctx *ctx, const float *y_dev, float *g_dev, float beta, const float *c_dev);

/* Squared loss with L2 regularisation (Eqs. opt_prob_general_form, residual):
 *   r = A c - I_data,  L = sum w r^2 + mu sum c^2,  grad = 2 A^T (w r) + 2 mu c.
 * w_dev may be NULL (all ones).  loss_dev receives L as one float64 on the
 * device; resid_dev (data layout) may be NULL (the residual then goes to the
 * workspace's scratch).  Overwrites grad_dev. */
int tt_loss_grad(tt_ctx *ctx, const float *c_dev, const float *data_dev, const float *w_dev,
                 double mu, double *loss_dev, float *grad_dev, float *resid_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * loss and gradient as tt_loss_grad, with the same arguments and results,
 * computed by the same kernels, but with its scratch (reduction partials,
 * folded residual, residual when resid_dev is NULL, the forward batch of
 * mapped volumes) in an array the library holds on each GPU from the first
 * tt_create there until the process ends, TT_NOALLOC_SCRATCH_BYTES long.
 * Needs no workspace (tt_set_workspace is not consulted) and allocates
 * nothing: no device or pinned memory, no events (timing is not recorded).
 * The forward batch is the largest that fits beside the other scratch;
 * TT_ENOMEM if even the smallest does not fit, with the needed size in
 * tt_last_error() (100^3 voxels at ell_max 8 with 240 projections of
 * 100x100 pixels x 8 segments fit; 128^3 with 300 projections of 128x128 x
 * 16 segments do not).
 * Every call on one GPU uses that GPU's single array and leaves its contents
 * there: calls that overlap in time on one GPU (other streams, other host
 * threads, other contexts) race and must be serialised by the caller. */
#define TT_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int tt_loss_grad_noalloc(tt_ctx *ctx, const float *c_dev, const float *data_dev, const float *w_dev,
                         double mu, double *loss_dev, float *grad_dev, float *resid_dev);

/* ------------------------------------------------------------------------ */
/* L-BFGS (section 3.5 "Optimization") on the loss above, with history m,    */
/* initial matrix gamma I (gamma = s^T y / y^T y of the newest pair), and    */
/* the exact line search of the quadratic loss                               */
/*   alpha = -g^T d / (2 (||A d||_w^2 + mu ||d||^2)).                        */
/* Pairs with s^T y <= 1e-12 ||s|| ||y|| are skipped.  All vectors stay on   */
/* the device in float32; dot products, curvature pairs and loss reductions  */
/* are float64.  The direction is formed from a float64 Gram matrix of the   */
/* history (same result as the two-loop recursion), so one iteration makes   */
/* two streaming passes over the history.                                    */
/* ------------------------------------------------------------------------ */
typedef struct tt_lbfgs tt_lbfgs;

/* Bytes of the solver workspace for history m (1..10): 2(m + 1) + 3
 * coefficient-sized float vectors (s and y slots, two gradients, the
 * direction), two data-sized float vectors (residual, A d), the float64 state
 * and reduction partials, each 256-byte aligned. */
int64_t tt_lbfgs_workspace_bytes(const tt_ctx *ctx, int m);
/* Create a solver on the caller's workspace (device, 256-byte aligned, at
 * least tt_lbfgs_workspace_bytes bytes; TT_EINVAL otherwise).  The history
 * slots are cleared on the context's stream.  The workspace and the data,
 * weight and coefficient buffers passed to tt_lbfgs_init must stay valid
 * while the solver is used.  The context needs its own workspace too. */
int tt_lbfgs_create(tt_ctx *ctx, int m, void *work_dev, size_t bytes, tt_lbfgs **out);
/* Waits for the context's stream, then frees the host-side solver state
 * (destroy it before its context; the workspace stays the caller's). */
void tt_lbfgs_destroy(tt_lbfgs *st);

/* Start from c_dev (read and updated in place): computes r, L and grad.
 * w_dev may be NULL.  Asynchronous. */
int tt_lbfgs_init(tt_lbfgs *st, float *c_dev, const float *data_dev, const float *w_dev,
                  double mu);

/* One iteration (direction, forward of d, line search, update, adjoint,
 * history update).  Asynchronous: no host synchronisation. */
int tt_lbfgs_step(tt_lbfgs *st);

/* One iteration along the caller's direction d_dev (coefficient layout)
 * instead of the two-loop direction: exact line search along d, update, and
 * the curvature pair (alpha d, g_new - g) enters the history.  Used to start
 * from zero along a predicted solution (a warm start whose scale the line
 * search chooses).  Asynchronous. */
int tt_lbfgs_step_direction(tt_lbfgs *st, const float *d_dev);

/* Synchronise and read the state: out4 = {loss, ||r||_2, ||I||_2,
 * accepted pairs}.  out4 may hold 4 doubles. */
int tt_lbfgs_query(tt_lbfgs *st, double *out4);

/* Recompute the residual from an explicit forward projection,
 * r = A c - I_data, and with it the loss and ||r|| that tt_lbfgs_query
 * reports (between iterations the solver updates r by r += alpha A d, which
 * accumulates float32 rounding).  Asynchronous. */
int tt_lbfgs_refresh(tt_lbfgs *st);

/* Run up to max_iter iterations, stopping once ||r|| / ||I|| <= rel_tol
 * (checked before each iteration, one host sync per iteration).  hist (host,
 * may be NULL) receives 2 doubles per iteration: loss and ||r||/||I||.
 * *iters_out gets the number of iterations done. */
int tt_lbfgs_run(tt_lbfgs *st, int max_iter, double rel_tol, double *hist, int *iters_out);

/* ------------------------------------------------------------------------ */
/* Learned warm start.  The paper's outlook (section 4) names simulated data */
/* for training machine-learning models; here a small 3-D convolutional      */
/* network maps the normalised backprojection A^T I to initial coefficients. */
/* Layers: y[v, co] = b[co] + sum_{d in {0,1,2}^3} sum_ci x[v + d - 1, ci]     */
/* w[d, ci, co], zero padding, tap index d = (dx*3 + dy)*3 + dz.  Layout is   */
/* channels-last x[n][X][Y][Z][c]; activations bf16 (uint16 bit patterns),    */
/* accumulation fp32 on bf16 MFMA.  ci, co must be 32 or 64.  All pointers    */
/* are device pointers owned by the caller; work is enqueued on `stream`.     */
/* ------------------------------------------------------------------------ */
enum { TT_CONV_RELU_BF16 = 0, TT_CONV_BIAS_F32 = 1, TT_CONV_MASK_BF16 = 2 };

/* bf16 elements of one MFMA-ordered weight copy for (ci, co). */
int64_t tt_conv3d_weight_elems(int ci, int co);
/* From fp32 masters w[27][ci][co]: wf (forward operand order) and wd (the
 * input-gradient operator w'[d][co][ci] = w[26 - d][ci][co], same order). */
int tt_conv3d_swizzle(const float *w, int ci, int co, uint16_t *wf, uint16_t *wd, void *stream);
/* y = conv(x, wf) with epilogue TT_CONV_RELU_BF16 (relu(. + bias), bf16 y),
 * TT_CONV_BIAS_F32 (. + bias, float y) or TT_CONV_MASK_BF16 (zero where
 * mask <= 0, bf16 y; with wd this is the input gradient through a ReLU whose
 * output is mask).  mask has co channels; bias may be NULL only for MASK. */
int tt_conv3d(int epilogue, int ci, int co, const uint16_t *x, const uint16_t *w_swizzled, const float *bias,
              const uint16_t *mask, void *y, int n, int X, int Y, int Z, void *stream);
/* Weight (and bias, if gb != NULL) gradients: gw[27][ci][co] =
 * sum_v x[v + d - 1, ci] gy[v, co], gb[co] = sum_v gy[v, co].  Deterministic
 * (split over voxels, partials summed in a fixed order).  work: float device
 * buffer of tt_conv3d_wgrad_work_bytes bytes. */
size_t tt_conv3d_wgrad_work_bytes(int ci, int co, int n, int X, int Y, int Z);
int tt_conv3d_wgrad(int ci, int co, const uint16_t *x, const uint16_t *gy, int n, int X, int Y, int Z, float *work,
                    size_t work_bytes, float *gw, float *gb, void *stream);
/* One Adam step (Kingma & Ba) on n fp32 parameters, step count t >= 1. */
int tt_adam(float *w, const float *g, float *m, float *v, int64_t n, int t, float lr, float beta1, float beta2,
            float eps, void *stream);
/* Mean-squared-error gradient: gy[v][c] = scale (y[v][c] - t[v][c]) for
 * c < creal (0 for creal <= c < cpad) in bf16 (gy may be NULL), and
 * loss[0] = sum (y - t)^2 in float64.  y is [nvox][cpad], t is
 * [nvox][creal]; work holds >= 1024 doubles. */
int tt_mse(const float *y, const float *t, int64_t nvox, int cpad, int creal, float scale, uint16_t *gy,
           double *loss, double *work, int64_t work_len, void *stream);
/* out[v][c] = bf16(scale[c] (pre_scale x[v][c] - shift[c])) for c < cin, 0
 * up to cpad (shift, scale may be NULL). */
int tt_pack_bf16(const float *x, int64_t nvox, int cin, int cpad, float pre_scale, const float *shift,
                 const float *scale, uint16_t *out, void *stream);

/* Patchwise inference on T^3 tiles at per-axis origins ox[ntx], oy[nty],
 * oz[ntz] (device int arrays; tile t = (ix nty + iy) ntz + iz).  Origins must
 * satisfy o + T <= volume size, tiles covering the whole volume.
 * tt_tile_gather: tiles t0 .. t0+nt-1 of vol[X][Y][Z][cv] (channels < cin),
 * scaled by pre_scale, standardised and packed to bf16
 * out[nt][T][T][T][cpad] as in tt_pack_bf16.
 * tt_tile_blend: out[X][Y][Z][cout] = sum_t w_t y_t / sum_t w_t on channels
 * < creal (0 above), y = all tiles' outputs [ntiles][T][T][T][cy] float,
 * w_t the product of per-axis linear ramps over `ramp` voxels on sides that
 * overlap a neighbouring tile. */
int tt_tile_gather(const float *vol, int X, int Y, int Z, int cv, int cin, int cpad, const int *ox, int ntx,
                   const int *oy, int nty, const int *oz, int ntz, int T, float pre_scale, const float *shift,
                   const float *scale, int t0, int nt, uint16_t *out, void *stream);

/* Normalisation of the network input of the learned warm start (the paper's
 * outlook on learned models, sect. 4): the backprojection A^T I is divided by
 * kappa, the lower median (element (n-1)/2 of the n sorted values) over the
 * voxels whose centre lies within `radius` of the volume centre of
 * (A^T A u)_{v,0}, u the unit isotropic field (u_{v,0} = 1, other
 * coefficients 0).  One forward and one adjoint on the context; the median is
 * an exact radix selection on the float bit patterns.  work: device, 256-byte
 * aligned, tt_normal_work_bytes bytes.  Synchronous; *kappa is a host double.
 * TT_ENONFINITE if no voxel centre lies inside the ball. */
int64_t tt_normal_work_bytes(const tt_ctx *ctx);
int tt_kappa(tt_ctx *ctx, double radius, void *work_dev, size_t work_bytes, double *kappa);
/* Per-channel standardisation statistics of y = pre_scale x over
 * x[nvox][cstride] (channels c < nch <= 64): shift[c] = mean, scale[c] =
 * 1 / max(unbiased standard deviation, 1e-12), as float.  Sums in float64
 * with fixed-order partials (run-to-run identical).  work: device float64
 * array of at least tt_channel_stats_work_len() elements.  Asynchronous. */
int64_t tt_channel_stats_work_len(void);
int tt_channel_stats(const float *x, int64_t nvox, int cstride, int nch, float pre_scale, float *shift, float *scale,
                     double *work, int64_t work_len, void *stream);
int tt_tile_blend(const float *y, int cy, int creal, int X, int Y, int Z, const int *ox, int ntx, const int *oy,
                  int nty, const int *oz, int ntz, int T, int ramp, int cout, float *out, void *stream);

#define TT_REDUCE_WORK 4096
/* ------------------------------------------------------------------------ */
/* Other objectives on the same operator (sect. 3.5, "Optimization"):       */
/* regularisers of the tensor field and fixed-step gradient descent with    */
/* optional Nesterov momentum.  Coefficient arrays are device float         */
/* [nx][ny][nz][C] (n = nx ny nz C elements).  Values accumulate in float64 */
/* without atomics: each block writes a partial sum into `partials` (device */
/* float64, at least TT_REDUCE_WORK elements, needed whenever a value is    */
/* requested) and one pass adds them in a fixed order, so repeated calls    */
/* give identical values.                                                   */
/* ------------------------------------------------------------------------ */
/* Laplacian regulariser lambda sum (Lap c)^2 with Lap the 7-point finite-
 * difference Laplacian of every coefficient channel, zero outside the volume:
 * grad += 2 lambda Lap(Lap c); value[0] += lambda sum (Lap c)^2 if value is
 * not NULL.  work: device float [n], holds Lap c on return.  c, work and grad
 * must not overlap.  TT_EUNSUPPORTED if C > 1024 or nx * ny * nz > 2^31 - 1
 * (z chunks of a row with their neighbours are staged in LDS). */
int tt_laplacian_reg(const float *c, int nx, int ny, int nz, int C, double lambda, float *work, float *grad,
                     double *value, double *partials, int64_t partials_len, void *stream);
/* Huber norm lambda sum h(c_e), h(x) = x^2 / (2 delta) for |x| <= delta and
 * |x| - delta / 2 otherwise (delta > 0): grad += lambda clamp(c / delta, -1, 1),
 * value[0] += lambda sum h if value is not NULL. */
int tt_huber_reg(const float *c, int64_t n, double delta, double lambda, float *grad, double *value, double *partials,
                 int64_t partials_len, void *stream);
/* Huber loss of the residual (robust regression, the paper's HuberLoss):
 * r = I - data, y = w clamp(r / delta, -1, 1) (pass y to tt_adjoint for the
 * gradient A^T y), value[0] += sum w h(r) if value is not NULL.  I, data, y
 * have n floats (data-shaped); w may be NULL (all ones). */
int tt_huber_loss(const float *I, const float *data, const float *w, int64_t n, double delta, float *y,
                  double *value, double *partials, int64_t partials_len, void *stream);
/* value[0] += scale * sum x^2 over n floats (float64 accumulation). */
int tt_sumsq(const float *x, int64_t n, double scale, double *value, double *partials, int64_t partials_len,
             void *stream);
/* One gradient step with momentum m on n floats, g = grad f(y):
 * c_new = y - step p g, y = c_new + m (c_new - c), c = c_new, with p an
 * optional diagonal preconditioner (n positive floats, NULL = 1; the paper's
 * loss functions "can be given a preconditioner to weight the gradient").
 * m = 0 is plain gradient descent (y then tracks c); Nesterov's schedule is
 * m_k = (k-1)/(k+2).  c, y, g and p must be distinct buffers. */
int tt_gd_step(float *c, float *y, const float *g, const float *precond, int64_t n, float step, float momentum,
               void *stream);
/* Diagonal preconditioner for tt_gd_step (the MITRA-style weighting of the
 * gradient, sect. 3.4): p[v][i] = 1 / max(d_v, floor_frac max_v d_v) for every
 * coefficient i of voxel v, with d_v = (A^T A u)_{v,0} the normal operator's
 * response to the unit isotropic field at voxel v.  p_dev has the coefficient
 * layout; work as for tt_kappa (tt_normal_work_bytes).  Asynchronous on the
 * context's stream. */
int tt_voxel_preconditioner(tt_ctx *ctx, double floor_frac, float *p_dev, void *work_dev, size_t work_bytes);

/* ------------------------------------------------------------------------ */
/* Derived per-voxel quantities (the paper's section on deriving standard    */
/* quantities from the output: mean intensity, second-moment tensor and its  */
/* eigendecomposition, fractional anisotropy; plus the spherical variance    */
/* and relative anisotropy that the basis-set properties list).              */
/* ------------------------------------------------------------------------ */
#define TT_PROP_FIELDS 22
/* c: device float [n_vox][C], C = tt_num_coeffs-style count for ell_max
 * (even, 0..16).  out: device float [n_vox][TT_PROP_FIELDS], per voxel:
 *   0 mean <f>, 1 variance <(f - <f>)^2>, 2 relative anisotropy sqrt(var)/mean,
 *   3..8 second-moment tensor M_ab = <q_a q_b f> as xx, yy, zz, xy, xz, yz,
 *   9..11 eigenvalues of M in descending order,
 *   12..20 the matching unit eigenvectors (x, y, z each), each with its
 *          largest-magnitude component positive,
 *   21 fractional anisotropy of the eigenvalues,
 * where f(q) = sum_i c_i Y_i(q) and <g> is the average over the unit sphere.
 * Sums and the eigensolver run in float64.  c and out must be 16-byte
 * aligned (TT_EINVAL otherwise); with n_vox = 0 nothing is accessed.
 * Asynchronous on `stream`. */
int tt_tensor_properties(const float *c, int64_t n_vox, int ell_max, float *out, void *stream);

/* ------------------------------------------------------------------------ */
/* Optional kernel timing: when enabled, every kernel launch of the context  */
/* is bracketed by HIP events on the context's stream, per kernel class.     */
/* ------------------------------------------------------------------------ */
enum {
    TT_K_MAP = 0,         /* coefficient-to-segment map (MFMA), forward */
    TT_K_MARCH = 1,       /* ray march, forward */
    TT_K_FOLD = 2,        /* antipodal fold of the adjoint input */
    TT_K_BACKPROJECT = 3, /* voxel-driven backprojection + MFMA map, adjoint */
    TT_K_RESIDUAL = 4,    /* residual, loss partials and fold */
    TT_K_VECTOR = 5,      /* L-BFGS streaming vector passes and reductions */
    TT_K_PLAN = 6,        /* L-BFGS float64 planner kernels */
    TT_K_FUSED = 7,       /* fused sparse map + ray march, forward (tt_set_sparse_map) */
    TT_K_COUNT = 8
};
int tt_timing_enable(tt_ctx *ctx, int on);
/* Synchronise, then ms_total[k] = summed duration and launches[k] = number of
 * launches of class k since the last read or enable; resets the counters. */
int tt_timing_read(tt_ctx *ctx, double *ms_total, int64_t *launches);

/* Last error message on this thread (never NULL). */
const char *tt_last_error(void);
const char *tt_error_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* TT_H */
