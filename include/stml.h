/*
 * stml.h -- C-ABI of the MI355X (gfx950) spatio-temporal multilevel (STML)
 * registration library, libstml.so.
 *
 * Method: Aggrawal & Modersitzki, "Accelerating the Registration of Image
 * Sequences by Spatio-temporal Multilevel Strategies" (arXiv 2001.06613).
 *   Sec. 2, eq. (1)  groupwise objective over a frame subset K,
 *                    J = sum_ij D(R_i o y_i, R_j o y_j) + S(Y) + P(Y),
 *                    with the penalty P on the mean transformation.
 *   Sec. 3, Fig. 1   temporal binary tree K_0 ... K_T.
 *   Sec. 3           coarse-level linear (midpoint) predictor, correction by
 *                    registering K_{q+1} from the prediction.
 *   Sec. 3, eq. (2)  least-squares temporal predictor on finer levels,
 *                    solved by the Thomas algorithm.
 *   Sec. 3, eq. (3)  optional stopping rule on the change of D.
 *   Sec. 4           spatial multilevel data, smoothed in space only.
 *
 * Instance computed here (the paper leaves the inner model open): every
 * frame k has a displacement u_k on a cell-centred grid, y_k = x + u_k;
 * D is the groupwise sum of squared differences normalised by 1/(2|K|)
 * (= h^d sum_k ||W_k - mean W||^2 with W_k the frame warped by bi/trilinear
 * interpolation, edge clamp); S = (alpha/2) h^d sum ||B u||^2 with B the
 * forward differences (diffusion) or the Neumann Laplacian (curvature);
 * P = lambda h^d ||mean_k u_k||^2.  The minimiser is Gauss-Newton with a
 * matrix-free Hessian, Jacobi-preconditioned CG, and an Armijo search.
 *
 * Conventions for every entry point
 *   - Pointers named *_dev are device pointers (HIP global memory on the
 *     context's device); all others are host pointers.
 *   - Images are float32, [n][extent...] with the last axis fastest
 *     (extent[0] slowest).  Displacements are float32 [n][dim][extent...]:
 *     component c is the displacement along axis c, in finest-level pixels.
 *   - The caller owns every buffer.  The context never allocates device
 *     memory: all device state lives in the caller's workspace, sized by
 *     stml_workspace_bytes().  Inputs are copied; outputs are written into
 *     caller buffers.
 *   - All work is enqueued on the stream given to stml_create(); every
 *     entry point returns with that stream synchronised.
 *   - Return value: 0 success, < 0 error (nothing further is valid for that
 *     call), > 0 warning (the call completed).  stml_last_error() gives a
 *     message.  One context must not be used by two threads at once.
 */
#ifndef STML_H
#define STML_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STML_OK            0
#define STML_EINVAL       -1  /* bad argument, shape, or non-finite input   */
#define STML_ENOMEM       -2  /* workspace too small                        */
#define STML_EDEVICE      -3  /* a HIP call failed                          */
#define STML_ESTATE       -4  /* call out of order (e.g. no sequence yet)   */
#define STML_EBREAKDOWN   -5  /* CG met p.Hp <= 0 (operator not SPD)        */
#define STML_WLINESEARCH   2  /* Armijo search found no step; u unchanged   */

#define STML_REG_DIFFUSION 0
#define STML_REG_CURVATURE 1

/* Registration model of a context (stml_opts.model).
 * FIELD : a displacement field per frame, groupwise SSD, diffusion or
 *         curvature regulariser, Gauss-Newton with Jacobi-PCG (the instance
 *         described at the top of this header).
 * AFFINE: the paper's experimental model (Sec. 2, Sec. 4): one affine-linear
 *         map per frame, u_k(x) = B_k xi(x) + b_k with xi(x) = (x - c) / R,
 *         c the centre of the finest grid and R half its largest side, so the
 *         p = dim^2 + dim parameters theta_k = (B_k row-major, b_k) are in
 *         pixels and mean the same map on every level; D is the pair sum of
 *         eq. (1) with the correlation-based distance 1 - rho_ij^2 (the SVD
 *         based SqN measure with q = 4, Sec. 2), no regulariser, the penalty
 *         P = lambda h^d sum_x |mean_k u_k(x)|^2 (Sec. 2), minimised by
 *         L-BFGS (Sec. 2) with the Armijo search; the temporal predictors
 *         and eq. (3) act on the parameters. */
#define STML_MODEL_FIELD  0
#define STML_MODEL_AFFINE 1

#define STML_MAX_FRAMES  256  /* frames per sequence supported by kernels   */

typedef struct stml_ctx stml_ctx;

/* Parameters.  stml_default_opts() fills the defaults listed here. */
typedef struct stml_opts {
  int dim;            /* 2 or 3                                     (2)      */
  int n_spatial;      /* number of spatial levels L >= 1            (2)      */
  int n_temporal;     /* number of temporal levels T + 1 >= 1       (2)      */
  int regulariser;    /* STML_REG_DIFFUSION or STML_REG_CURVATURE   (0)      */
  double alpha;       /* regulariser weight                         (1e-2)   */
  double lambda;      /* penalty weight of Sec. 2                   (1e-2)   */
  double beta;        /* eq. (2) weight                             (1e-5)   */
  double eps_stop;    /* eq. (3) tolerance epsilon; 0 = off         (0)      */
  int gn_max;         /* Gauss-Newton iterations per registration   (10)     */
  int cg_max;         /* CG iterations per Gauss-Newton step        (20)     */
  double cg_rtol;     /* CG stops at ||r|| <= cg_rtol ||r_0||       (0.1)    */
  int ls_max;         /* Armijo tries t = 1, 1/2, ..., 2^-ls_max    (10)     */
  double c1;          /* Armijo constant                            (1e-4)   */
  double tol_J;       /* GN stops when the relative decrease of J   (1e-3)   */
  double tol_u;       /*   and the root mean square of the accepted
                           step t delta (pixels) are below both     (1e-2)   */
  int predictor;      /* 0 = the paper's interpolation predictors;
                         1 = also reserve room for a learned predictor
                         (stml_set_predictor_net)                  (0)      */
  int parity_mode;    /* 1: exactly gn_max GN and cg_max CG iterations,
                         no convergence exits, eq. (3) off          (0)      */
  int stop_relative;  /* 0: eq. (3) as printed, |D_q - D_{q-1}| <= eps;
                         1: |D_q - D_{q-1}| <= eps |D_q|            (0)      */
  int model;          /* STML_MODEL_FIELD or STML_MODEL_AFFINE      (0)      */
  int lbfgs_mem;      /* AFFINE: L-BFGS pairs kept, 1..16 (gn_max is
                         the iteration cap; alpha, regulariser, cg_* and
                         predictor do not apply)                    (5)      */
} stml_opts;

/* Statistics of one registration call (GIR on one subset). */
typedef struct stml_gir_log {
  int level, q, n_frames;
  int gn_iterations;
  int status;             /* STML_OK, STML_WLINESEARCH or STML_EBREAKDOWN   */
  double J0, J;           /* objective before the first and after the last
                             accepted step                                   */
  double D, S, P;         /* parts of J at the last evaluation              */
  int cg_iterations[64];  /* per GN iteration (first 64)                    */
  double step[64];        /* accepted Armijo step t per GN iteration        */
  double J_iter[64];      /* objective after each accepted step             */
  double du_max[64];      /* max |t delta| (pixels) of each accepted step    */
  double du_rms[64];      /* root mean square of t delta (pixels)            */
  int predictor;          /* start guess: -1 none (q = 0: the spatial
                             prolongation), 0 the paper's temporal
                             predictor, 1 the learned one                   */
  double J_paper, J_learned;  /* objective on the subset at the two
                             candidate start guesses (NaN if not compared) */
} stml_gir_log;

void stml_default_opts(stml_opts* opts);

/* Bytes of device workspace a context for n frames of the given finest
 * extent (dim entries, slowest first) needs.  0 if the arguments are
 * invalid: n outside 1..STML_MAX_FRAMES, n dim N above 2e9 values, or
 * more than 8184 Hessian-product tiles at the finest level (2-D: 64 x 4
 * pixels, about 2 Mpx, e.g. 1448 x 1448; 3-D: columns of 16 x 16 x 16
 * voxels, about 33 M voxels). */
size_t stml_workspace_bytes(const stml_opts* opts, int n, const int* extent);

/* Create a context.  workspace_dev must stay valid, untouched by the caller,
 * until stml_destroy().  hip_stream is a hipStream_t (NULL = default).
 * Errors: EINVAL (opts or shape), ENOMEM (ws_bytes too small), EDEVICE. */
int stml_create(const stml_opts* opts, int n, const int* extent,
                void* hip_stream, void* workspace_dev, size_t ws_bytes,
                stml_ctx** out);

void stml_destroy(stml_ctx* ctx);

const char* stml_last_error(const stml_ctx* ctx);

/* Load the sequence R_1..R_n (Sec. 2) and build the spatial pyramid by
 * restriction in space only (Sec. 4): each coarser cell is the mean of the
 * 2^dim finer cells that exist (extents halve rounding up, as in Table 1).
 * frames_dev: [n][extent...] float32.  Resets every level's displacements
 * to 0.  Errors: EINVAL if any value is not finite. */
int stml_set_sequence(stml_ctx* ctx, const float* frames_dev);

/* Copy the pyramid image of `level` (0 = coarsest) into out_dev,
 * [n][extent_level...]. */
int stml_get_level_frames(const stml_ctx* ctx, int level, float* out_dev);

/* Extent of `level` (dim ints into out_extent). */
int stml_level_extent(const stml_ctx* ctx, int level, int* out_extent);

/* Frames of K_q (Sec. 3, Fig. 1), 0-based, ascending; returns |K_q| (or an
 * error) and writes at most `cap` indices to out_frames. */
int stml_temporal_set(const stml_ctx* ctx, int q, int* out_frames, int cap);

/* Predictor step (Sec. 3).  Sets the start guess z(level, q_next, all) of
 * every frame and makes it the current estimate y:
 *   q_next = 0, level = 0 : identity (u = 0);
 *   q_next = 0, level > 0 : prolongation of level-1's estimate;
 *   q_next > 0, level = 0 : linear interpolation from K_{q_next-1};
 *   q_next > 0, level > 0 : eq. (2), eta = current estimate on K_{q_next-1},
 *                           omega = the previous start guess, Thomas solve.
 * Errors: ESTATE (no sequence, or level-1 not registered), EINVAL. */
int stml_predict(stml_ctx* ctx, int level, int q_next);

/* Groupwise registration GIR(level, K_q) of eq. (1) from the current
 * estimate; frames outside K_q are unchanged.  Returns OK, or
 * STML_WLINESEARCH / STML_EBREAKDOWN (last good iterate kept). */
int stml_register_level(stml_ctx* ctx, int level, int q);

/* Correction step of Sec. 3: GIR(level, K_{q_next}) started from the
 * prediction; identical to stml_register_level(ctx, level, q_next). */
int stml_correct(stml_ctx* ctx, int level, int q_next);

/* Whole schedule of Sec. 3: levels coarse to fine, predictor-corrector over
 * K_0..K_T, eq. (3) when eps_stop > 0 and not in parity mode.
 * Eq. (3) (Sec. 3): after registering K_q and predicting every frame from
 * it, D is evaluated over all n frames at the estimate (the prediction,
 * with the frames of K_q as registered); from q = 1 on the level stops
 * when |D_q - D_{q-1}| <= eps_stop, and that estimate is the level's
 * result (K_{q+1}, ... are not registered). */
int stml_run(stml_ctx* ctx);

/* Eq. (3) record of the last stml_run for `level`: the all-frame D_q of
 * each q evaluated (at most `cap` into D_out, host), and in *stop_q (may be
 * NULL) the q at which the level stopped, -1 if it did not.  Returns the
 * number of D values recorded (0 when eq. (3) was off), or EINVAL. */
int stml_get_stop_trace(const stml_ctx* ctx, int level, double* D_out,
                        int cap, int* stop_q);

/* Objective targets for the registrations of the schedule (host array
 * J_targets[level * n_temporal + q], float64; -INFINITY for none; NULL
 * clears them): outside parity mode, GIR(level, K_q) also stops as soon as
 * its objective is at or below the target (before its first step if the
 * start already is).  Used to run a schedule to the objectives another run
 * reached (equal-objective comparisons).  Field model only; EINVAL for a
 * NaN. */
int stml_set_targets(stml_ctx* ctx, const double* J_targets);

/* Current estimate (y) of `level` into u_dev [n][dim][extent_level...]. */
int stml_get_displacements(const stml_ctx* ctx, int level, float* u_dev);
/* Overwrite the current estimate of `level` (resume or test). */
int stml_set_displacements(stml_ctx* ctx, int level, const float* u_dev);
/* Last start guess z of `level` (the omega reference of eq. (2)). */
int stml_get_prediction(const stml_ctx* ctx, int level, float* z_dev);
int stml_set_prediction(stml_ctx* ctx, int level, const float* z_dev);

/* Registration statistics: number of logged GIR calls since
 * stml_set_sequence, and entry i. */
int stml_log_count(const stml_ctx* ctx);
int stml_get_log(const stml_ctx* ctx, int i, stml_gir_log* out);

/* --- affine model (opts.model = STML_MODEL_AFFINE) -----------------------
 * Parameters are host arrays [n][p], p = dim^2 + dim, float64, rows
 * theta_k = (B_k row-major, b_k) in pixels (see STML_MODEL_AFFINE).  On an
 * affine context stml_get_displacements writes u_k(x) of every frame;
 * stml_set_displacements, stml_get/set_prediction, stml_eval,
 * stml_hessvec, stml_gn_direction, learned predictors and batches return
 * EINVAL; the schedule entry points (predict, register_level, correct,
 * run) act on the parameters. */

/* Current parameters of `level` into theta_out (host, [n][p]). */
int stml_get_params(const stml_ctx* ctx, int level, double* theta_out);
/* Overwrite the current parameters of `level` (resume or test). */
int stml_set_params(stml_ctx* ctx, int level, const double* theta);
/* Objective of the affine model at theta (host, [n][p]) over the frames K
 * (nk ascending indices): out_JDP = {J, D, P}; the gradient wrt the
 * parameters of the frames of K into grad_out (host, [nk][p], may be NULL).
 * Errors: EINVAL (also a frame without contrast after warping, whose
 * correlation is undefined). */
int stml_eval_params(stml_ctx* ctx, int level, const int* frames, int nk,
                     const double* theta, double* out_JDP, double* grad_out);

/* --- kernel-level entry points (same conventions) ------------------------
 * frames: host array of nk frame indices (distinct, ascending), the subset K.
 * u_dev : [n][dim][extent_level] displacement of all frames.
 * Compact outputs are [nk][dim][extent_level], in the order of frames.  */

/* Objective (eq. (1) instance) at u: out_JDSP = {J, D, S, P}; gradient
 * into grad_dev and dW/du into dW_dev (either may be NULL). */
int stml_eval(stml_ctx* ctx, int level, const int* frames, int nk,
              const float* u_dev, double* out_JDSP, float* grad_dev,
              float* dW_dev);

/* Gauss-Newton Hessian at u applied to v_dev (compact) into hv_dev
 * (compact); out_vHv (may be NULL) receives v.Hv. */
int stml_hessvec(stml_ctx* ctx, int level, const int* frames, int nk,
                 const float* u_dev, const float* v_dev, float* hv_dev,
                 double* out_vHv);

/* One Gauss-Newton direction at u: Jacobi-PCG on H delta = -g with the
 * context's cg_max / cg_rtol / parity_mode; delta into delta_dev
 * (compact), CG iterations into *out_cg.  Returns EBREAKDOWN on p.Hp <= 0
 * (delta = last iterate). */
int stml_gn_direction(stml_ctx* ctx, int level, const int* frames, int nk,
                      const float* u_dev, float* delta_dev, int* out_cg);
/* Test of the CG breakdown branch (p.Hp <= 0 never occurs with valid
 * options, Sec. 2's Gauss-Newton matrix being SPD): from now on CG step it
 * of every Gauss-Newton iteration of this context (single runs, not
 * batches) stops as if p.Hp <= 0, keeping the iterate of the steps before
 * it (x = 0 at it = 0) and reporting STML_EBREAKDOWN where a breakdown is
 * reported.  it = -1 turns this off.  EINVAL for it < -1. */
int stml_force_cg_breakdown(stml_ctx* ctx, int it);

/* --- evaluation without allocation --------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * objective, gradient and dW/du of stml_eval (same kernels, same results)
 * on frames the caller holds, without a context or workspace.  Its scratch
 * (the evaluation's float64 partials, the objective scalars and the frame
 * list) is one static device array of STML_NOALLOC_SCRATCH_BYTES that each
 * GPU holds from the first call on it until the process ends.  Calls that
 * overlap on one GPU (two host threads, or two streams in flight) share
 * that array and race; each call returns with its stream synchronised.
 *   opts      : dim, regulariser, alpha, lambda are read (host).
 *   n, extent : frames and their extent (dim ints, slowest first; host).
 *   h         : grid spacing of this level (finest = 1).
 *   frames_dev: [n][extent...] float32 images (device).
 *   frames    : nk ascending frame indices, the subset K (host).
 *   u_dev     : [n][dim][extent...] displacements (device).
 *   out_JDSP  : host, {J, D, S, P}.
 *   grad_dev, dW_dev: [nk][dim][extent...] outputs (device, required).
 *   hip_stream: hipStream_t (NULL = default).
 * Errors: EINVAL (null pointer, options, shape, frame list), ENOMEM (n
 * above STML_MAX_FRAMES, or an evaluation grid above the scratch's 512
 * blocks: cannot happen for valid shapes), EDEVICE; the message is in
 * stml_noalloc_last_error() (per host thread).  Calls no hipMalloc,
 * hipFree or other allocating routine. */
#define STML_NOALLOC_SCRATCH_BYTES 66816
int stml_eval_noalloc(const stml_opts* opts, int n, const int* extent,
                      double h, const float* frames_dev, const int* frames,
                      int nk, const float* u_dev, double* out_JDSP,
                      float* grad_dev, float* dW_dev, void* hip_stream);
const char* stml_noalloc_last_error(void);

/* --- kernel timing (measurement only) -----------------------------------
 * Each launch of a timed kernel class on the context's stream is bracketed
 * by two HIP events; durations, launch counts and the voxel-frames each
 * launch covers (|K| x voxels of the level, or n x voxels for
 * whole-sequence kernels) accumulate per (class, level).  Timing adds two
 * event records per timed launch. */
#define STML_K_EVAL        0  /* warp + distance + gradient                 */
#define STML_K_HESSVEC     1  /* Gauss-Newton Hessian product (CG and test;
                                 volumes: with the direction's voxel sums) */
#define STML_K_CG_UPDATE   2  /* r, z update, x every second step, r.z       */
#define STML_K_CG_PUPDATE  3  /* p = z + beta p                              */
#define STML_K_TRIAL       4  /* objective at the Armijo trial steps         */
#define STML_K_CG_INIT     5  /* CG start scalars (r, z: by the evaluation)  */
#define STML_K_ACCEPT      6  /* u += t delta                                */
#define STML_K_PREDICT     7  /* prolongation and temporal predictors        */
#define STML_K_RESTRICT    8  /* spatial restriction                         */
#define STML_K_COUNT       9
#define STML_K_ALL       0x1ff  /* mask of every class                     */

/* Launch shape of the kernels (autotuned by the caller; every value a
 * multiple of 8): blocks per registration for the objective and trial
 * kernels (8..1024, default 512) and for the voxel-major CG updates
 * (8..1024, default 512), and the block target of the Hessian product
 * (8..8192, default 2048).  Results depend on them only through the order
 * of float64 sums.  EINVAL when out of range. */
typedef struct stml_tuning {
  int tile_blocks;
  int vox_blocks;
  int hv_blocks;
} stml_tuning;
int stml_set_tuning(stml_ctx* ctx, const stml_tuning* tuning);
int stml_get_tuning(const stml_ctx* ctx, stml_tuning* tuning);

/* mask != 0: clear the accumulators and time the classes whose bit
 * (1 << STML_K_...) is set; mask = 0: stop timing.  Each timed launch is
 * bracketed by its dispatch's own start/end timestamps (or an event pair);
 * the records are resolved when read, never inside a solve. */
int stml_timing(stml_ctx* ctx, int mask);
/* As stml_timing, but time only every period-th launch of each class
 * (period >= 1; counting restarts here): a timestamped dispatch costs a few
 * microseconds of issue time, so a sample keeps a timed run close to an
 * untimed one.  Totals then cover the sampled launches only. */
int stml_timing_every(stml_ctx* ctx, int mask, int period);
/* Totals of one kernel class at one level (level = -1: all levels):
 * time, launches, voxel-frames, and algorithmic HBM bytes (every input
 * field read once, every output field written once, float32). */
int stml_timing_get(stml_ctx* ctx, int kernel, int level, double* total_ms,
                    long long* launches, double* voxel_frames,
                    double* bytes);

/* --- learned temporal predictor -----------------------------------------
 * A convolutional encoder-decoder that refines the linear interpolation of
 * a frame t between its registered neighbours l < t < r (Sec. 3 predicts
 * such frames by interpolation; the network adds a learned correction).
 * For images (dim 2) and volumes (dim 3; D = dim components).  Input
 * channels: frame_l, frame_t, frame_r, u_l / h, u_r / h (3 + 2D channels;
 * displacements in pixels of the level, h = cell width); output: the
 * D-channel correction c, u_t = w_l u_l + w_r u_r + h c with the linear
 * weights w_l = (r - t) / (r - l), w_r = (t - l) / (r - l).  Encoder 3^dim
 * convolutions 32/64/128/128 with ReLU and 2^dim average pooling, decoder
 * with nearest upsampling and skip concatenation, 1x1 head.  Parameters are
 * one float32 vector (layer by layer W[tap][c_out][c_in] then b[c_out], the
 * taps in row-major order of their offsets); kernels use bfloat16 weights
 * and activations with float32 accumulation (MFMA), float32 gradients, Adam
 * on the float32 master copy.  Extents (H, W in 2-D; Z, H, W in 3-D, W
 * fastest) must be multiples of 8, W at most 256.  The net is sized for
 * max_batch frames of max_extent; a batch may hold any number B of frames
 * of any extent with B times its voxels <= max_batch times the voxels of
 * max_extent.  All buffers: caller-owned device memory; the net keeps the
 * last assembled batch until the next one.  Errors: STML_EINVAL (shapes,
 * null pointers, triples not l < t < r), STML_ESTATE (no batch yet),
 * STML_EDEVICE. */
typedef struct stml_net stml_net;

int stml_net_param_count(int dim);
size_t stml_net_workspace_bytes(int dim, int max_batch,
                                const int* max_extent);
int stml_net_create(int dim, int max_batch, const int* max_extent,
                    void* hip_stream, void* workspace_dev, size_t ws_bytes,
                    stml_net** out);
void stml_net_destroy(stml_net* net);
/* Float32 parameters in and out (setting them also resets Adam). */
int stml_net_set_params(stml_net* net, const float* params_dev);
int stml_net_get_params(const stml_net* net, float* params_dev);
/* A batch from planar float32 channels x [batch][channels][extent] and,
 * optionally, the target correction [batch][extent][D]. */
int stml_net_set_input(stml_net* net, const float* x_dev, int channels,
                       const float* target_dev, int batch, const int* extent);
/* A batch of frames (triples[3b] = t, l, r with 0 <= l < t < r < n_frames)
 * from level frames [n_frames][extent] and displacements
 * [n_frames][D][extent]; with_target: the target correction
 * (u_t - linear interpolation) / h from the same field. */
int stml_net_assemble(stml_net* net, const float* frames_dev,
                      const float* u_dev, int n_frames, const int* extent,
                      double h, const int* triples, int batch,
                      int with_target);
/* Forward pass; out_dev (may be NULL) receives [batch][extent][32] floats
 * whose first D channels are the correction. */
int stml_net_forward(stml_net* net, float* out_dev);
/* u_t = linear interpolation + h * correction into u_dev
 * [n_frames][D][extent] (n_frames and extent as last assembled) for the
 * frames of the last assembled batch (after stml_net_forward). */
int stml_net_emit(stml_net* net, double h, float* u_dev);
/* Mean squared error of the correction and its gradient wrt the
 * parameters (no update). */
int stml_net_gradient(stml_net* net, float* grad_dev, double* loss);
/* Forward, loss, backward and one Adam step (lr > 0). */
int stml_net_train_step(stml_net* net, double lr, double* loss);
/* Use net for the prediction of the frames of K_{q+1} \ K_q (each from its
 * nearest registered neighbours in K_q) on every level whose extents are
 * multiples of 8 and fit the net (NULL: the paper's predictors only).  The
 * predictor of Sec. 3 (linear interpolation, eq. (2) on finer levels) stays
 * the fallback: per prediction step both start guesses are evaluated on
 * K_{q+1} and the one with the lower objective is kept (a tie keeps the
 * paper's); the log of the following registration records the choice.
 * The context must have been created with opts.predictor = 1 (ESTATE
 * otherwise) and have the net's dimension (EINVAL otherwise); the net runs
 * on its own stream and must outlive its use. */
int stml_set_predictor_net(stml_ctx* ctx, stml_net* net);

/* --- batching: several sequences in shared launches ----------------------
 * A batch registers the sequences of several contexts together: each
 * Gauss-Newton iteration of a stage (level, q) runs as one launch per
 * kernel over the tiles of every sequence (a persistent grid whose blocks
 * are dealt to the sequences in fixed shares, so every sequence gets the
 * blocks, and hence the float64 sums, it gets alone: batched results equal
 * per-sequence results bit for bit).  Per-sequence scalars and stop flags
 * stay on the device; one iteration is captured in a HIP graph and
 * replayed.  The contexts keep their own workspaces, sequences, logs and
 * displacements (read them with stml_get_displacements / stml_get_log).
 * All contexts: the same dim (2 or 3), the same numbers of levels,
 * regulariser, gn_max, cg_max, cg_rtol, ls_max, c1, tol_J, tol_u and
 * parity_mode; eq. (3) off
 * (eps_stop = 0) unless in parity mode; at most one batch per context at a
 * time.  The batch only borrows the contexts (they must outlive it).
 * Workspace: caller-owned device memory of stml_batch_workspace_bytes().
 * Errors: STML_EINVAL (mismatched contexts, bad level/q), STML_ESTATE (a
 * context without a sequence), STML_ENOMEM, STML_EDEVICE; warnings as for
 * the single-sequence calls (the worst over the sequences). */
typedef struct stml_batch stml_batch;

size_t stml_batch_workspace_bytes(int count);
int stml_batch_create(stml_ctx* const* ctxs, int count, void* hip_stream,
                      void* workspace_dev, size_t ws_bytes,
                      stml_batch** out);
void stml_batch_destroy(stml_batch* batch);
const char* stml_batch_last_error(const stml_batch* batch);
/* on = 0: enqueue every iteration's launches directly instead of replaying
 * a captured graph (the default; same results). */
int stml_batch_set_graph(stml_batch* batch, int on);
/* stml_predict(level, q_next) of every sequence. */
int stml_batch_predict(stml_batch* batch, int level, int q_next);
/* stml_register_level(level, q) of every sequence, batched. */
int stml_batch_register_level(stml_batch* batch, int level, int q);
/* The schedule of Sec. 3 for every sequence (levels coarse to fine,
 * predictor-corrector over K_0..K_T), each registration batched. */
int stml_batch_run(stml_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* STML_H */
