// Host-side launchers of the STML kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "stml_dev.h"

struct stml_net;

namespace stml {

// Partial-sum slots of the reductions: one region per producing kernel, so
// a consumer can read its producer's slots after the next kernel wrote its
// own.  A region holds up to 20 values x 1024 blocks (a trial sweep of
// kTrialSteps steps writes kTrialSteps + 9 values per block).
constexpr size_t kRegionSlots = (size_t)20 * 1024;
static_assert(kTrialSteps + 9 <= 20, "trial partials exceed a region");
// Line-search sweeps: sweep 0 in kRegTrial, later sweeps alternate between
// kRegTrialOdd and kRegTrialEven, so that a sweep can read its
// predecessor's slots while it writes its own.
enum {
  kRegEval,
  kRegHv,
  kRegUpdate,
  kRegTrial,
  kRegTrialOdd,
  kRegTrialEven,
  kRegTest,
  kRegCount
};
__host__ __device__ inline int trial_region(int p) {
  return p == 0 ? kRegTrial : (p & 1) ? kRegTrialOdd : kRegTrialEven;
}
constexpr size_t kRedSlots = kRegionSlots * kRegCount;
struct RedBuf {
  double* part;         // kRedSlots doubles
  __host__ __device__ double* region(int r) const {
    return part + (size_t)r * kRegionSlots;
  }
};

// Temporal-predictor tables of one subset K_q (device pointers).
struct LinTab {            // per frame k: z_k = wl y_left + wr y_right
  int* left;
  int* right;
  double* wl;
  double* wr;
};
struct ThomasTab {         // factorisation of M + beta D^T D for one K_q
  double* invp;            // 1 / pivot_k
  double* cp;              // c'_k (super-diagonal after elimination)
  int* mask;               // 1 if k in K_q
};

Geom make_geom(int dim, const int* ext, double h);
Model make_model(int dim, double h, int nK, double alpha, double lambda,
                 int reg);

int tile_blocks(const Geom& g);
int tile_threads(int dim, int nK);
int eval_threads(int dim, int nK);

hipError_t launch_fill(float* p, size_t count, float v, hipStream_t s);
hipError_t launch_check_finite(const float* p, size_t count, Scal* sc,
                               hipStream_t s);
hipError_t launch_restrict(int dim, const float* fine, float* coarse, int n,
                           const Geom& gf, const Geom& gc, hipStream_t s);
hipError_t launch_prolong(int dim, const float* coarse, float* fine,
                          int fields, const Geom& gc, const Geom& gf,
                          hipStream_t s);

// Start of the Jacobi-PCG, formed by the evaluation from the gradient it
// writes: r = -g, z = M^-1 r and the per-voxel sums S_z ([N]) and V_z
// ([D][N]).
struct CgStart {
  float* r;
  float* z;
  double* Sz;
  float* Vz;
};
// finalize = false leaves the partials for the CG start to reduce.
// gn_it: Gauss-Newton iteration this launch belongs to (ignored when
// finalize is set); the kernel does nothing if gn_it >= sc->gn_stop.
// cs (needs grad): the evaluation also forms the CG start; its partials
// then hold r.z and r.r after D, S, P.
hipError_t launch_eval(int dim, const float* T, const float* u, const int* K,
                       const Geom& g, const Model& md, float* grad,
                       float* dW, RedBuf rb, Scal* sc, hipStream_t s,
                       bool finalize, int gn_it,
                       const CgStart* cs = nullptr);

// Line-search sweep p of iteration gn_it (see sweep_t): objective at
// u + t delta for the sweep's steps, g.delta, max |delta| and sum delta^2.
// A sweep p >= 1 runs only if sweep p - 1 ran and accepted no step (every
// block decides that from the partials itself).
hipError_t launch_trial(int dim, const float* T, const float* u,
                        const float* delta, const float* grad, const int* K,
                        const Geom& g, const Model& md, int p, int ls_max,
                        double c1, RedBuf rb, Scal* sc, hipStream_t s,
                        int gn_it, GNLog* log);
// Armijo decision after the sweeps: the first accepted step of the last
// sweep that ran; u[K[j]] += t delta_j, the log entry and the Gauss-Newton
// stop tests.  No step: status 1 and the iteration ends the registration.
hipError_t launch_ls_accept(float* u, const float* delta, const int* K,
                            const Geom& g, const Model& md, int ls_max,
                            double c1, int fixed, double tol_J, double tol_u,
                            RedBuf rb, int gn_it, Scal* sc, GNLog* log,
                            hipStream_t s);
// J_target: the registration stops once J <= J_target (not in parity
// mode); -inf for none.
hipError_t launch_gn_reset(Scal* sc, GNLog* log, int n, hipStream_t s,
                           double J_target = -INFINITY);
// One block: objective and CG start scalars from the partials of an
// evaluation that formed the CG start (ev_nb blocks).
hipError_t launch_finalize_start(RedBuf rb, int ev_nb, const Model& md,
                                 Scal* sc, int gn_it, GNLog* log,
                                 hipStream_t s);
hipError_t launch_finalize_vhv(const double* part, int nb, Scal* sc,
                               hipStream_t s);

// --- CG with per-voxel cross-frame sums (cg_tiles.hip) -------------------
// Per-voxel sums, accumulated in float64: S = sum_k dW_k . v_k ([N],
// stored float64: the data term subtracts its mean from each s_k) and
// V = sum_k v_k ([D][N], stored float32: it only feeds the penalty term) of
// z, and of the CG directions (ping-pong by CG iteration).
struct CgSums {
  double* Sz;
  float* Vz;
  double* Sp[2];
  float* Vp[2];
};
struct CgTiles {             // launch shape of the Hessian product
  int nreal, nfg, fpg, grid, vox_grid;
};
// Launch shape of the Hessian product (2-D: 64 x 4 tiles, 3-D: columns of
// kHv3X x kHv3Y x kHv3Z) and of the voxel-major updates
CgTiles cg_tiles(const Geom& g, int nK, int dim);
int cg_tile_count(const Geom& g, int dim);
// ev0/ev1 (optional): timed by the dispatch's own start/end timestamps
// x: the CG solution, to which a step that finds convergence after an even
// step adds that step's term (unused at it = 0).
hipError_t launch_cgt_hvp(int it, const float* z, const float* p_old,
                          float* p_new, const float* dW, const Geom& g,
                          const Model& md, float* q, float* x, CgSums sums,
                          int fixed, double rtol, RedBuf rb, Scal* sc,
                          hipStream_t s, int gn_it, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr);
// At it = 0 it also forms the Gauss-Newton iteration's start scalars from
// the evaluation's partials (and writes log[gn_it].J).  p_prev: the
// direction of step it - 1 (the other buffer of the pair); x is written by
// cg_x_mode(it, cg_max).  brk: a step that takes the breakdown branch as if
// p.Hp <= 0 (-1: none).
hipError_t launch_cgv_update(int dim, int it, int cg_max, int brk,
                             const float* p,
                             const float* p_prev, const float* q,
                             const float* dW, const Geom& g, const Model& md,
                             float* x, float* r, float* z, CgSums sums,
                             RedBuf rb, Scal* sc, hipStream_t s, int gn_it,
                             GNLog* log, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr);
// Test entry: H v for a stored v through the tiled Hessian product;
// v is copied to vcopy on the way.
hipError_t launch_hessvec_tiled(const float* v, const float* dW,
                                const Geom& g, const Model& md, float* hv,
                                float* vcopy, CgSums sums, RedBuf rb,
                                Scal* sc, hipStream_t s);

hipError_t launch_linear_predict(const float* Y, float* Z, float* Yout,
                                 LinTab tab, int n, int dim, long long N,
                                 hipStream_t s);
hipError_t launch_ls_predict(float* Y, float* Z, ThomasTab tab, int n,
                             int dim, long long N, double beta,
                             hipStream_t s);

// ------------------------------------------------------------- batching
//
// One problem of a batched launch: the subset K of one sequence at one
// level, with that sequence's own solver vectors, reduction slots, scalars
// and log.  Every kernel of a Gauss-Newton iteration has a batched form that
// serves all problems (all 2-D or all 3-D) in one launch: the blocks of a launch are
// dealt to the problems in order (first[c][j] .. first[c][j+1] for kernel
// class c), each problem getting exactly the blocks (and hence the sums) it
// gets alone.  The iteration index is read from the problem's scalars
// (gn_cur), so one captured iteration can be replayed.
struct Job {
  const float* T;        // level frames [n][N]
  float* u;              // displacements [n][D][N]
  const int* K;          // frames of the subset
  Geom g;
  Model md;
  float *grad, *dW, *x, *r, *z, *q, *P0, *P1;
  CgSums sums;
  RedBuf rb;
  Scal* sc;
  GNLog* log;
  long long count;       // |K| D N
  int nb_tile, nb_vox, nb_elem;
  CgTiles ct;
};
enum { kClsTile, kClsVox, kClsHv, kClsOne, kClsElem, kClsCount };
struct JobSet {
  const Job* jobs;
  const int* first;      // [kClsCount][n + 1] block offsets
  int n;
};
// Blocks of each kernel class for a problem (shares start at multiples of
// kXCD); fills job.nb_* and job.ct.
void job_shape(Job* job);
int elem_grid(long long count);
hipError_t batch_gn_reset(const JobSet& js, int gn_max, hipStream_t s);
hipError_t batch_eval(const JobSet& js, int nblocks, int dim, int reg,
                      hipStream_t s);
// objective and CG start scalars of every running job (one block each)
hipError_t batch_finalize_start(const JobSet& js, hipStream_t s);
// x = 0 for every running job (CG with no iteration: cg_max = 0)
hipError_t batch_zero_x(const JobSet& js, int nvox, int dim, hipStream_t s);
hipError_t batch_cg_hvp(const JobSet& js, int nhv, int nvox, int dim, int reg,
                        int it, int fixed, double rtol, hipStream_t s);
hipError_t batch_cg_update(const JobSet& js, int nvox, int dim, int it,
                           int cg_max, hipStream_t s);
hipError_t batch_trial(const JobSet& js, int ntile, int dim, int reg, int p,
                       int ls_max, double c1, hipStream_t s);
hipError_t batch_accept(const JobSet& js, int nelem, int ls_max, double c1,
                        int fixed, double tol_J, double tol_u, hipStream_t s);
hipError_t batch_advance(const JobSet& js, int* stop_out, hipStream_t s);

// ------------------------------------------------ affine model (affine.hip)
//
// Affine-linear maps per frame with the SqN distance (Sec. 2, Sec. 4):
// u_k(x) = B_k xi(x) + b_k, xi(x) = (x - c) / R on a level's cell centres.
struct AffGeom {
  Geom g;
  double h, hd, inv_R;
  double c[3];
  int d;
};
// Objective of the last first-pass evaluation (J = D + P) and a flag for a
// frame without contrast after warping (zero variance).
struct AffScal {
  double J, D, P;
  int bad, pad;
};
// L-BFGS state of one registration (device).
struct AffState {
  double J, Jt, slope, t;
  double rho[16];
  int npairs, head, iters, accepted, stop, bad;
};
// Device buffers of one evaluation.
struct AffBufs {
  double* part;     // Gram partials [nb][E]
  double* tot;      // Gram totals [E]
  double* mu;       // frame means [|K|]
  double* Rc;       // dD/dW coefficients [|K|][|K|]
  double* gpen;     // penalty gradient wrt the mean parameters [p]
  float* r;         // dD/dW_i per voxel [|K|][N]
  float* W;         // warped frames of the last Gram pass [|K|][N]
  double* gpart;    // parameter-gradient partials [|K|][p][nb]
  double* gout;     // gradient [|K|][p]
  AffScal* sc;
};
constexpr int kAffGramBlocks = 512;    // Gram partials per evaluation
constexpr int kAffGramTiles = 12;      // 16 x 16 Gram tiles per wave
constexpr int kAffResidRows = 3;       // 16-row tiles of dD/dW per wave
constexpr int kAffPgradBlocks = 64;    // gradient partials per frame
struct AffShape {
  int groups, E, nb_gram, nb_resid, nb_pgrad;
  size_t lds_gram, lds_resid;
};
AffShape aff_shape(const AffGeom& ag, int nk);
// J (and with grad the gradient into b.gout) at x + t dv (dv may be null:
// at x) for the frames K; reuse_gram skips the first pass, whose totals
// (b.tot) are then those of the same point.
hipError_t launch_aff_objective(const float* T, const int* K, int nk,
                                const double* x, const double* dv, double t,
                                const AffGeom& ag, double lam, AffBufs b,
                                bool grad, bool reuse_gram, hipStream_t s);
hipError_t launch_aff_state_init(AffState* st, const AffScal* sc,
                                 hipStream_t s);
hipError_t launch_aff_direction(AffState* st, const double* g, double* d,
                                const double* S, const double* Y, int nP,
                                int mem, hipStream_t s);
hipError_t launch_aff_accept(AffState* st, const AffScal* sc, double t,
                             double c1, hipStream_t s);
hipError_t launch_aff_update(AffState* st, double* x, const double* d,
                             double* g, const double* gn, double* S,
                             double* Y, int nP, int mem, double tol_J,
                             double tol_u, hipStream_t s);
hipError_t launch_aff_gather(double* x, const double* theta, const int* K,
                             int nk, int P, bool scatter, hipStream_t s);
hipError_t launch_aff_linear_predict(double* Y, double* Z, LinTab tab, int n,
                                     int P, hipStream_t s);
hipError_t launch_aff_ls_predict(double* Y, double* Z, ThomasTab tab, int n,
                                 int P, double beta, double* dp,
                                 hipStream_t s);
hipError_t launch_aff_field(const double* theta, int n, const AffGeom& ag,
                            float* u, hipStream_t s);

// Capacity of a learned-predictor net (cnn.hip): the batch it was created
// for and the pixels a batch may hold in total (frames x pixels per frame).
void net_capacity(const stml_net* n, int* max_batch, long long* max_pixels);
int net_dim(const stml_net* n);
// 3-D Hessian-product columns: x, y tile and planes marched in z
constexpr int kHv3X = 32, kHv3Y = 16, kHv3Z = 16;
constexpr int kMaxNetWidth = 256;   // widest frame row the net accepts

}  // namespace stml
