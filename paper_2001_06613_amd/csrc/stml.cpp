// Host side of libstml: context, workspace layout, the Gauss-Newton / PCG
// driver, the spatio-temporal multilevel schedule and the C-ABI of stml.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/stml.h"
#include "launch.h"

using namespace stml;

static_assert(STML_MAX_FRAMES == kMaxFrames,
              "the kernels size per-frame LDS tables by kMaxFrames");

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct LevelBufs {
  float* T;      // [n][N]
  float* Y;      // [n][D][N] current estimate
  float* Z;      // [n][D][N] last start guess (omega of eq. (2))
};

struct QTabs {
  int* K;            // device: frames of K_q
  LinTab lin;
  ThomasTab thomas;
};

// Workspace carve-up; the same walk sizes and assigns it.
struct Layout {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    size_t o = off;
    off = align_up(off + count * sizeof(T));
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

}  // namespace

struct stml_ctx {
  stml_opts o;
  int n = 0, d = 2, L = 1, T1 = 1;
  std::vector<std::vector<int>> ext;    // per level, coarse first
  std::vector<long long> N;
  std::vector<double> h;
  hipStream_t stream = nullptr;
  std::vector<LevelBufs> lv;
  std::vector<QTabs> qt;
  std::vector<std::vector<int>> K;      // host copies of K_q
  // solver scratch, compact [nK][D][N_finest]
  float *g = nullptr, *dW = nullptr, *x = nullptr, *r = nullptr,
        *z = nullptr, *q = nullptr;
  float* P[2] = {nullptr, nullptr};      // CG directions, ping-pong
  int cg_break = -1;                     // CG step forced to break down
  CgSums sums{};                         // per-voxel cross-frame sums
  RedBuf rb{};
  Scal* sc = nullptr;
  int* kbuf = nullptr;                  // device frame list for test calls
  Scal* hsc = nullptr;                  // pinned host mirror of sc
  GNLog* gnlog = nullptr;               // device: one entry per GN iteration
  GNLog* hlog = nullptr;                // pinned host mirror
  int* hk = nullptr;                    // pinned host staging of frame lists
  bool have_seq = false;
  stml_tuning tune{kMaxTileBlocks, kMaxTileBlocks, kHvBlocks};
  stml_net* net = nullptr;               // learned predictor (optional)
  float* ureg = nullptr;                 // registered estimate kept for it
  struct Pick {
    int used = -1;
    double Jp = NAN, Jl = NAN;
  } pick;                                // start guess of the next GIR
  // affine model: parameters [n][P] per level (estimate Y, start guess Z),
  // the evaluation's buffers and the L-BFGS state and vectors ([n P])
  int npar = 0;
  struct AffLevel {
    double* Y;
    double* Z;
  };
  std::vector<AffLevel> alv;
  AffBufs ab{};
  double *ax = nullptr, *agr = nullptr, *ad = nullptr, *agn = nullptr,
         *aS = nullptr, *aY = nullptr, *aest = nullptr, *anow = nullptr,
         *adp = nullptr;
  AffState* ast = nullptr;
  AffState* hast = nullptr;             // pinned host mirrors
  AffScal* hasc = nullptr;
  std::vector<stml_gir_log> logs;
  // objective targets per (level, q) (-inf: none), see stml_set_targets
  std::vector<double> targets;
  // eq. (3) of the last stml_run: D over all frames per q, and the q at
  // which each level stopped (-1: not stopped)
  std::vector<std::vector<double>> stop_trace;
  std::vector<int> stop_q;
  std::string err;
  // kernel timing
  struct Rec {
    int kernel, level;
    double vf, bytes;
    hipEvent_t a, b;
  };
  struct KStat {
    double ms = 0.0, vf = 0.0, bytes = 0.0;
    long long n = 0;
  };
  unsigned timing = 0;                  // bit k: time kernel class k
  int tperiod = 1;                      // time every tperiod-th launch
  long long tcount[STML_K_COUNT] = {};  // launches seen per class
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  std::map<std::pair<int, int>, KStat> kstats;
};

namespace {

int fail(stml_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIP_OK(call)                                                       \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess)                                                  \
      return fail(c, STML_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

bool opts_valid(const stml_opts* o) {
  return o && (o->dim == 2 || o->dim == 3) && o->n_spatial >= 1 &&
         o->n_spatial <= 16 && o->n_temporal >= 1 && o->n_temporal <= 16 &&
         (o->regulariser == STML_REG_DIFFUSION ||
          o->regulariser == STML_REG_CURVATURE) &&
         o->alpha >= 0 && o->lambda >= 0 && o->beta >= 0 &&
         o->eps_stop >= 0 && o->gn_max >= 0 && o->cg_max >= 0 &&
         o->ls_max >= 0 && o->ls_max <= 60 &&
         (o->stop_relative == 0 || o->stop_relative == 1) &&
         (o->model == STML_MODEL_FIELD ||
          (o->model == STML_MODEL_AFFINE && o->predictor == 0 &&
           o->lbfgs_mem >= 1 && o->lbfgs_mem <= 16)) &&
         (o->predictor == 0 || o->predictor == 1);
}

std::vector<std::vector<int>> level_extents(int dim, const int* extent,
                                            int L) {
  std::vector<std::vector<int>> e(L);
  e[L - 1].assign(extent, extent + dim);
  for (int l = L - 2; l >= 0; --l) {
    e[l].resize(dim);
    for (int a = 0; a < dim; ++a) e[l][a] = (e[l + 1][a] + 1) / 2;
  }
  return e;
}

// K_q = {k : k mod 2^(T-q) = 0} u {n-1} (Sec. 3, Fig. 1).
std::vector<std::vector<int>> temporal_sets(int n, int T1) {
  std::vector<std::vector<int>> K(T1);
  int T = T1 - 1;
  for (int q = 0; q < T1; ++q) {
    long long step = 1LL << (T - q);
    for (int k = 0; k < n; ++k)
      if (k % step == 0 || k == n - 1) K[q].push_back(k);
  }
  return K;
}

long long voxels(const std::vector<int>& e) {
  long long v = 1;
  for (int m : e) v *= m;
  return v;
}

// Walk the workspace: returns the byte size; assigns pointers if base.
size_t layout_affine(stml_ctx* c, Layout& lo) {
  const int n = c->n, P = c->npar;
  const size_t nP = (size_t)n * P;
  c->alv.resize(c->L);
  for (int l = 0; l < c->L; ++l) {
    c->lv[l].T = lo.take<float>((size_t)n * c->N[l]);
    c->lv[l].Y = c->lv[l].Z = nullptr;
    c->alv[l].Y = lo.take<double>(nP);
    c->alv[l].Z = lo.take<double>(nP);
  }
  const size_t E = (size_t)(n + 1) * (n + 2) / 2;
  c->ab.part = lo.take<double>((size_t)kAffGramBlocks * E);
  c->ab.tot = lo.take<double>(E);
  c->ab.mu = lo.take<double>(n);
  c->ab.Rc = lo.take<double>((size_t)n * n);
  c->ab.gpen = lo.take<double>(16);
  c->ab.r = lo.take<float>((size_t)n * c->N[c->L - 1]);
  c->ab.W = lo.take<float>((size_t)n * c->N[c->L - 1]);
  c->ab.gpart = lo.take<double>(nP * kAffPgradBlocks);
  c->ab.gout = nullptr;                      // set per evaluation
  c->ab.sc = lo.take<AffScal>(1);
  c->ax = lo.take<double>(nP);
  c->agr = lo.take<double>(nP);
  c->ad = lo.take<double>(nP);
  c->agn = lo.take<double>(nP);
  c->aest = lo.take<double>(nP);
  c->anow = lo.take<double>(nP);
  c->adp = lo.take<double>(nP);
  c->aS = lo.take<double>(nP * c->o.lbfgs_mem);
  c->aY = lo.take<double>(nP * c->o.lbfgs_mem);
  c->ast = lo.take<AffState>(1);
  return lo.off;
}

size_t layout(stml_ctx* c, char* base) {
  Layout lo;
  lo.base = base;
  const int n = c->n, D = c->d;
  c->lv.resize(c->L);
  if (c->o.model == STML_MODEL_AFFINE) {
    layout_affine(c, lo);
    c->sc = lo.take<Scal>(1);
    c->gnlog = lo.take<GNLog>(1);
    c->kbuf = lo.take<int>(STML_MAX_FRAMES);
    c->qt.resize(c->T1);
    for (int q = 0; q < c->T1; ++q) {
      c->qt[q].K = lo.take<int>(n);
      c->qt[q].lin.left = lo.take<int>(n);
      c->qt[q].lin.right = lo.take<int>(n);
      c->qt[q].lin.wl = lo.take<double>(n);
      c->qt[q].lin.wr = lo.take<double>(n);
      c->qt[q].thomas.invp = lo.take<double>(n);
      c->qt[q].thomas.cp = lo.take<double>(n);
      c->qt[q].thomas.mask = lo.take<int>(n);
    }
    return lo.off;
  }
  for (int l = 0; l < c->L; ++l) {
    size_t NL = (size_t)c->N[l];
    c->lv[l].T = lo.take<float>((size_t)n * NL);
    c->lv[l].Y = lo.take<float>((size_t)n * D * NL);
    c->lv[l].Z = lo.take<float>((size_t)n * D * NL);
  }
  size_t vec = (size_t)n * D * (size_t)c->N[c->L - 1];
  c->g = lo.take<float>(vec);
  c->dW = lo.take<float>(vec);
  c->x = lo.take<float>(vec);
  c->r = lo.take<float>(vec);
  c->P[0] = lo.take<float>(vec);
  c->P[1] = lo.take<float>(vec);
  c->z = lo.take<float>(vec);
  c->q = lo.take<float>(vec);
  if (c->o.predictor == 1) c->ureg = lo.take<float>(vec);
  {
    size_t NF = (size_t)c->N[c->L - 1];
    c->sums.Sz = lo.take<double>(NF);
    c->sums.Vz = lo.take<float>(NF * D);
    for (int i = 0; i < 2; ++i) {
      c->sums.Sp[i] = lo.take<double>(NF);
      c->sums.Vp[i] = lo.take<float>(NF * D);
    }
  }
  c->rb.part = lo.take<double>(kRedSlots);
  c->sc = lo.take<Scal>(1);
  c->gnlog = lo.take<GNLog>(c->o.gn_max > 0 ? c->o.gn_max : 1);
  c->kbuf = lo.take<int>(STML_MAX_FRAMES);
  c->qt.resize(c->T1);
  for (int q = 0; q < c->T1; ++q) {
    c->qt[q].K = lo.take<int>(n);
    c->qt[q].lin.left = lo.take<int>(n);
    c->qt[q].lin.right = lo.take<int>(n);
    c->qt[q].lin.wl = lo.take<double>(n);
    c->qt[q].lin.wr = lo.take<double>(n);
    c->qt[q].thomas.invp = lo.take<double>(n);
    c->qt[q].thomas.cp = lo.take<double>(n);
    c->qt[q].thomas.mask = lo.take<int>(n);
  }
  return lo.off;
}

bool setup_dims(stml_ctx* c, const stml_opts* o, int n, const int* extent) {
  if (!opts_valid(o) || n < 1 || n > STML_MAX_FRAMES || !extent) return false;
  for (int a = 0; a < o->dim; ++a)
    if (extent[a] < 1) return false;
  c->o = *o;
  c->n = n;
  c->d = o->dim;
  c->L = o->n_spatial;
  c->T1 = o->n_temporal;
  c->ext = level_extents(o->dim, extent, c->L);
  c->N.resize(c->L);
  c->h.resize(c->L);
  for (int l = 0; l < c->L; ++l) {
    c->N[l] = voxels(c->ext[l]);
    c->h[l] = std::ldexp(1.0, c->L - 1 - l);
  }
  // compact vectors index elements with 64-bit offsets, but the element
  // kernels decode the frame index from 32-bit rows
  if ((double)n * o->dim * (double)c->N[c->L - 1] > 2.0e9) return false;
  c->npar = o->dim * o->dim + o->dim;
  // the Hessian product runs one block per 64 x 4 tile (3-D: per column of
  // kHv3X x kHv3Y x kHv3Z) at least, and its partials must fit one
  // reduction region
  if (o->model == STML_MODEL_FIELD) {
    const std::vector<int>& e = c->ext[c->L - 1];
    long long tiles =
        o->dim == 2
            ? (long long)((e[1] + 63) / 64) * ((e[0] + 3) / 4)
            : (long long)((e[2] + kHv3X - 1) / kHv3X) *
                  ((e[1] + kHv3Y - 1) / kHv3Y) * ((e[0] + kHv3Z - 1) / kHv3Z);
    if (tiles > (long long)kRegionSlots - 8192 - 8) return false;
  }
  c->K = temporal_sets(n, c->T1);
  return true;
}

Geom geom_of(const stml_ctx* c, int level) {
  Geom g = make_geom(c->d, c->ext[level].data(), c->h[level]);
  g.tile_cap = c->tune.tile_blocks;
  g.vox_cap = c->tune.vox_blocks;
  g.hv_target = c->tune.hv_blocks;
  return g;
}

Model model_of(const stml_ctx* c, int level, int nK) {
  return make_model(c->d, c->h[level], nK, c->o.alpha, c->o.lambda,
                    c->o.regulariser);
}

// --- kernel timing: event pairs around launches, resolved at sync points
hipEvent_t pooled_event(stml_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void tresolve(stml_ctx* c);

// Pending records are resolved when read (stml_timing_get), when timing is
// switched, or when this many accumulate: resolving waits for the events,
// so it is kept out of the solve.
constexpr size_t kMaxPending = 1 << 15;

// Whether this launch of class kernel is timed (every tperiod-th one).
bool timed_now(stml_ctx* c, int kernel) {
  if (!((c->timing >> kernel) & 1u)) return false;
  return c->tcount[kernel]++ % c->tperiod == 0;
}

bool tbegin(stml_ctx* c, int kernel, int level, double vf, double bytes) {
  if (!timed_now(c, kernel)) return false;
  if (c->pending.size() >= kMaxPending) tresolve(c);
  stml_ctx::Rec r{kernel, level, vf, bytes, pooled_event(c),
                  pooled_event(c)};
  if (!r.a || !r.b) return false;
  (void)hipEventRecord(r.a, c->stream);
  c->pending.push_back(r);
  return true;
}

// Timing by the dispatch itself: a pending record whose events the
// launcher passes to hipExtLaunchKernelGGL (no separate event packets).
void tdispatch(stml_ctx* c, int kernel, int level, double vf, double bytes,
               hipEvent_t* ev0, hipEvent_t* ev1) {
  *ev0 = *ev1 = nullptr;
  if (!timed_now(c, kernel)) return;
  if (c->pending.size() >= kMaxPending) tresolve(c);
  stml_ctx::Rec r{kernel, level, vf, bytes, pooled_event(c),
                  pooled_event(c)};
  if (!r.a || !r.b) return;
  *ev0 = r.a;
  *ev1 = r.b;
  c->pending.push_back(r);
}

void tend(stml_ctx* c) {
  if (!c->pending.empty())
    (void)hipEventRecord(c->pending.back().b, c->stream);
}

void tresolve(stml_ctx* c) {
  for (auto& r : c->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess ||
        hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      (void)hipGetLastError();   // an unrecorded pair: not an error here
    } else {
      auto& st = c->kstats[{r.kernel, r.level}];
      st.ms += ms;
      st.vf += r.vf;
      st.bytes += r.bytes;
      st.n += 1;
    }
    c->pool.push_back(r.a);
    c->pool.push_back(r.b);
  }
  c->pending.clear();
}

int read_scal(stml_ctx* c) {
  HIP_OK(hipMemcpyAsync(c->hsc, c->sc, sizeof(Scal), hipMemcpyDeviceToHost,
                        c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  return STML_OK;
}

// Algorithmic HBM bytes per voxel-frame of each kernel class (float32
// fields of D components): what the kernel must read and write once.
double alg_bytes(int kernel, int D, int cg_it, int cg_max) {
  switch (kernel) {
    case STML_K_EVAL: return 4.0 + 20.0 * D;      // T; u; dW, g, r, z
    case STML_K_HESSVEC:                          // z (+p_old), dW; p, q
      return cg_it > 0 ? 20.0 * D : 16.0 * D;
    case STML_K_CG_UPDATE: {                      // q, dW, r; r, z; x terms
      // x by cg_x_mode: none; x (+)= a p; x += a' p' + a p; x = a' p' + a p
      const int xm = cg_x_mode(cg_it, cg_max);
      const double xb = xm == kXNone  ? 0.0
                        : xm == kXOne ? (cg_it > 0 ? 12.0 : 8.0)
                        : xm == kXTwo ? 16.0
                                      : 12.0;
      return (20.0 + xb) * D;
    }
    case STML_K_CG_INIT: return 0.0;              // scalars only
    case STML_K_TRIAL: return 4.0 + 12.0 * D;     // T; u, delta, g
    case STML_K_ACCEPT: return 12.0 * D;          // u, delta; u
    case STML_K_PREDICT: return 16.0 * D;         // read y, z; write z, y
    case STML_K_RESTRICT: return 4.0 * (1 << D) + 4.0;  // per coarse voxel
    default: return 0.0;
  }
}

#define TIMED(KERNEL, LEVEL, VF, CALL) TIMED_IT(KERNEL, LEVEL, VF, 0, CALL)
// CALL names the events ev0_, ev1_ it passes to its launcher
#define TIMED_DISPATCH(KERNEL, LEVEL, VF, CGIT, CALL)                   \
  do {                                                                  \
    hipEvent_t ev0_, ev1_;                                              \
    tdispatch(c, KERNEL, LEVEL, VF,                                     \
              (VF) * alg_bytes(KERNEL, c->d, CGIT, c->o.cg_max), &ev0_, \
              &ev1_);                                                   \
    HIP_OK(CALL);                                                       \
  } while (0)
#define TIMED_IT(KERNEL, LEVEL, VF, CGIT, CALL)                        \
  do {                                                                 \
    const bool tr_ =                                                   \
        tbegin(c, KERNEL, LEVEL, VF,                                    \
               (VF) * alg_bytes(KERNEL, c->d, CGIT, c->o.cg_max));     \
    hipError_t te_ = (CALL);           \
    if (tr_) tend(c);                  \
    HIP_OK(te_);                       \
  } while (0)

int upload_tables(stml_ctx* c) {
  const int n = c->n;
  const double beta = c->o.beta;
  for (int q = 0; q < c->T1; ++q) {
    const std::vector<int>& Kq = c->K[q];
    std::vector<int> left(n), right(n), mask(n, 0);
    std::vector<double> wl(n), wr(n), invp(n), cp(n);
    for (int k : Kq) mask[k] = 1;
    for (int k = 0; k < n; ++k) {
      if (mask[k]) {
        left[k] = right[k] = k;
        wl[k] = 1.0;
        wr[k] = 0.0;
        continue;
      }
      int l = 0, r = n - 1;
      for (int z : Kq) {
        if (z < k) l = z;
        if (z > k) {
          r = z;
          break;
        }
      }
      left[k] = l;
      right[k] = r;
      wl[k] = (double)(r - k) / (r - l);
      wr[k] = (double)(k - l) / (r - l);
    }
    // Thomas factorisation of M + beta D^T D (shared by every component)
    double prev_cp = 0.0;
    for (int k = 0; k < n; ++k) {
      int ndiff = (n == 1) ? 0 : ((k == 0 || k == n - 1) ? 1 : 2);
      double diag = mask[k] + beta * ndiff;
      double den = (k == 0) ? diag : diag + beta * prev_cp;  // -sub*cp, sub=-beta
      invp[k] = 1.0 / den;
      cp[k] = (k == n - 1) ? 0.0 : -beta / den;
      prev_cp = cp[k];
    }
    QTabs& t = c->qt[q];
    HIP_OK(hipMemcpyAsync(t.K, Kq.data(), Kq.size() * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(t.lin.left, left.data(), n * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(t.lin.right, right.data(), n * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(t.lin.wl, wl.data(), n * sizeof(double),
                          hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(t.lin.wr, wr.data(), n * sizeof(double),
                          hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(t.thomas.invp, invp.data(), n * sizeof(double),
                          hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(t.thomas.cp, cp.data(), n * sizeof(double),
                          hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(t.thomas.mask, mask.data(), n * sizeof(int),
                          hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
  }
  return STML_OK;
}

int check_level(stml_ctx* c, int level) {
  if (level < 0 || level >= c->L)
    return fail(c, STML_EINVAL, "level %d outside [0, %d)", level, c->L);
  return STML_OK;
}

// Frames list from the caller into the device staging buffer.
int stage_frames(stml_ctx* c, const int* frames, int nk) {
  if (!frames || nk < 1 || nk > c->n)
    return fail(c, STML_EINVAL, "frame list: need 1..%d frames", c->n);
  for (int i = 0; i < nk; ++i) {
    if (frames[i] < 0 || frames[i] >= c->n || (i && frames[i] <= frames[i - 1]))
      return fail(c, STML_EINVAL, "frame list must be ascending in [0,%d)",
                  c->n);
    c->hk[i] = frames[i];
  }
  HIP_OK(hipMemcpyAsync(c->kbuf, c->hk, nk * sizeof(int),
                        hipMemcpyHostToDevice, c->stream));
  return STML_OK;
}

// The CG start the evaluation forms along with the gradient (r, z and the
// per-voxel sums of z).
CgStart cg_start(stml_ctx* c) {
  return CgStart{c->r, c->z, c->sums.Sz, c->sums.Vz};
}

// Jacobi-PCG for H delta = -g at the evaluation just made (g, dW, and the
// CG start r, z in scratch), as part of Gauss-Newton iteration gn_it.
// Enqueued only; the scalars stay on the device.  The first CG update forms
// the iteration's start scalars; without CG steps a one-block kernel does.
int enqueue_pcg(stml_ctx* c, int level, const Geom& g, const Model& md,
                int gn_it) {
  const int D = c->d;
  const double vf = (double)md.nK * g.N;
  if (c->o.cg_max == 0) {   // no CG step: the direction is x0 = 0
    TIMED(STML_K_CG_INIT, level, vf,
          launch_finalize_start(c->rb, tile_blocks(g), md, c->sc, gn_it,
                                c->gnlog, c->stream));
    HIP_OK(launch_fill(c->x, (size_t)md.nK * D * g.N, 0.0f, c->stream));
  }
  for (int it = 0; it < c->o.cg_max; ++it) {
    float* pn = c->P[it & 1];
    const float* po = c->P[(it + 1) & 1];
    TIMED_DISPATCH(STML_K_HESSVEC, level, vf, it,
                   launch_cgt_hvp(it, c->z, po, pn, c->dW, g, md, c->q,
                                  c->x, c->sums, c->o.parity_mode,
                                  c->o.cg_rtol,
                                  c->rb, c->sc, c->stream, gn_it, ev0_,
                                  ev1_));
    TIMED_DISPATCH(STML_K_CG_UPDATE, level, vf, it,
                   launch_cgv_update(D, it, c->o.cg_max, c->cg_break, pn, po,
                                     c->q, c->dW, g, md, c->x,
                                     c->r, c->z, c->sums, c->rb, c->sc,
                                     c->stream, gn_it, c->gnlog, ev0_,
                                     ev1_));
  }
  return STML_OK;
}

int gn_log(stml_ctx* c, int nK, long long N, stml_gir_log* log);

// Gauss-Newton on the frames Kdev (nK of them) of `level`, updating u in
// place; mirrors the oracle's gauss_newton step for step.  Every decision
// (CG stop, Armijo step, Gauss-Newton stop) is taken on the device, so the
// iterations are enqueued without host round trips; in parity mode the
// host synchronises once at the end, otherwise after every iteration so
// that no launches are spent after the stopping rule fired.
int gauss_newton(stml_ctx* c, int level, const int* Kdev, int nK, float* u,
                 stml_gir_log* log, double J_target = -INFINITY) {
  const stml_opts& o = c->o;
  const int D = c->d;
  const Geom g = geom_of(c, level);
  const Model md = model_of(c, level, nK);
  const float* T = c->lv[level].T;
  const double vf = (double)nK * g.N;
  // Armijo: every sweep is enqueued (a sweep whose predecessor accepted a
  // step exits at once), then one decision
  const int sweeps = sweep_count(o.ls_max);
  HIP_OK(launch_gn_reset(c->sc, c->gnlog, o.gn_max, c->stream,
                         o.parity_mode ? -INFINITY : J_target));
  const CgStart cs = cg_start(c);
  for (int it = 0; it < o.gn_max; ++it) {
    TIMED(STML_K_EVAL, level, vf,
          launch_eval(D, T, u, Kdev, g, md, c->g, c->dW, c->rb, c->sc,
                      c->stream, false, it, &cs));
    int rc = enqueue_pcg(c, level, g, md, it);
    if (rc) return rc;
    for (int p = 0; p < sweeps; ++p)
      TIMED(STML_K_TRIAL, level, vf,
            launch_trial(D, T, u, c->x, c->g, Kdev, g, md, p, o.ls_max, o.c1,
                         c->rb, c->sc, c->stream, it, c->gnlog));
    TIMED(STML_K_ACCEPT, level, vf,
          launch_ls_accept(u, c->x, Kdev, g, md, o.ls_max, o.c1,
                           o.parity_mode, o.tol_J, o.tol_u, c->rb, it, c->sc,
                           c->gnlog, c->stream));
    if (!o.parity_mode) {
      rc = read_scal(c);
      if (rc) return rc;
      if (c->hsc->gn_stop <= it + 1) break;
    }
  }
  return gn_log(c, nK, g.N, log);
}

// Statistics of the registration that just ran on c (device log and
// scalars) for nK frames of N voxels.
int gn_log(stml_ctx* c, int nK, long long N, stml_gir_log* log) {
  const stml_opts& o = c->o;
  const int D = c->d;
  HIP_OK(hipMemcpyAsync(c->hlog, c->gnlog, o.gn_max * sizeof(GNLog),
                        hipMemcpyDeviceToHost, c->stream));
  int rc = read_scal(c);
  if (rc) return rc;
  int status = STML_OK;
  std::memset(log, 0, sizeof *log);
  log->n_frames = nK;
  log->J0 = log->J = NAN;
  // the start's objective, also when no step was taken (a target met)
  if (o.gn_max > 0) log->J0 = log->J = c->hlog[0].J;
  for (int it = 0; it < o.gn_max; ++it) {
    const GNLog& L = c->hlog[it];
    if (L.status < 0) break;
    if (it == 0) log->J0 = log->J = L.J;
    if (it < 64) log->cg_iterations[it] = L.cg;
    if (L.status == 1) {
      status = STML_WLINESEARCH;
      break;
    }
    if (it < 64) {
      log->step[it] = L.t;
      log->J_iter[it] = L.Jacc;
      log->du_max[it] = L.t * L.maxd;
      log->du_rms[it] = L.t * std::sqrt(L.ssqd / ((double)nK * D * N));
    }
    log->gn_iterations += 1;
    log->J = L.Jacc;
    if (L.status == 2) {
      status = STML_EBREAKDOWN;
      break;
    }
  }
  log->D = c->hsc->D;
  log->S = c->hsc->S;
  log->P = c->hsc->P;
  log->status = status;
  return status;
}

// Objective of GIR(level, K_q) at the field U (no gradient).
int objective_on(stml_ctx* c, int level, int q, const float* U, double* J) {
  const Geom g = geom_of(c, level);
  const Model md = model_of(c, level, (int)c->K[q].size());
  HIP_OK(launch_eval(c->d, c->lv[level].T, U, c->qt[q].K, g, md, nullptr,
                     nullptr, c->rb, c->sc, c->stream, true, 0));
  int rc = read_scal(c);
  if (rc) return rc;
  *J = c->hsc->J;
  return STML_OK;
}

bool net_fits(const stml_ctx* c, int level) {
  if (!c->net || !c->ureg || net_dim(c->net) != c->d) return false;
  int maxB = 0;
  long long maxpix = 0;
  net_capacity(c->net, &maxB, &maxpix);
  const std::vector<int>& e = c->ext[level];
  for (int a = 0; a < c->d; ++a)
    if (e[a] % 8 || e[a] < 8) return false;
  return e[c->d - 1] <= kMaxNetWidth && c->N[level] <= maxpix;
}

// Learned start guess for the frames of K_{q_next} \ K_{q_next-1}: the
// network refines the linear interpolation between each frame's nearest
// registered neighbours (kept in ureg); the paper's prediction, already in
// Y and Z, is kept unless the learned one has the lower objective on
// K_{q_next}.  Both predictors leave Z equal to Y, so the candidate is
// written into Z and the loser is overwritten by the winner.
int learned_predict(stml_ctx* c, int level, int q_next) {
  const std::vector<int>& Kq = c->K[q_next - 1];
  const std::vector<int>& Kn = c->K[q_next];
  LevelBufs& b = c->lv[level];
  std::vector<int> tri;
  for (int t : Kn) {
    if (std::binary_search(Kq.begin(), Kq.end(), t)) continue;
    auto it = std::upper_bound(Kq.begin(), Kq.end(), t);
    if (it == Kq.begin() || it == Kq.end()) continue;   // K_q holds 0, n-1
    tri.push_back(t);
    tri.push_back(*(it - 1));
    tri.push_back(*it);
  }
  const int nt = (int)tri.size() / 3;
  if (nt == 0) return STML_OK;
  double Jp = NAN, Jl = NAN;
  int rc = objective_on(c, level, q_next, b.Y, &Jp);
  if (rc) return rc;
  int maxB = 0;
  long long maxpix = 0;
  net_capacity(c->net, &maxB, &maxpix);
  const int* e = c->ext[level].data();
  const double h = c->h[level];
  const int per = (int)std::min<long long>(nt, maxpix / c->N[level]);
  for (int s = 0; s < nt; s += per) {
    int B = std::min(per, nt - s);
    rc = stml_net_assemble(c->net, b.T, c->ureg, c->n, e, h,
                           tri.data() + 3 * s, B, 0);
    if (!rc) rc = stml_net_forward(c->net, nullptr);
    if (!rc) rc = stml_net_emit(c->net, h, b.Z);
    if (rc) return fail(c, rc, "learned predictor failed at level %d", level);
  }
  rc = objective_on(c, level, q_next, b.Z, &Jl);
  if (rc) return rc;
  const bool use = Jl < Jp;
  const size_t cnt = (size_t)c->n * c->d * c->N[level];
  HIP_OK(hipMemcpyAsync(use ? b.Y : b.Z, use ? b.Z : b.Y, cnt * sizeof(float),
                        hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  c->pick.used = use ? 1 : 0;
  c->pick.Jp = Jp;
  c->pick.Jl = Jl;
  return STML_OK;
}

// ------------------------------------------------------------ affine model

AffGeom aff_geom(const stml_ctx* c, int level) {
  AffGeom ag;
  ag.g = geom_of(c, level);
  ag.h = c->h[level];
  ag.d = c->d;
  ag.hd = c->d == 3 ? ag.h * ag.h * ag.h : ag.h * ag.h;
  const std::vector<int>& ef = c->ext[c->L - 1];
  int mx = 0;
  for (int a = 0; a < 3; ++a) ag.c[a] = 0.0;
  for (int a = 0; a < c->d; ++a) {
    ag.c[a] = ef[a] / 2.0;
    mx = std::max(mx, ef[a]);
  }
  ag.inv_R = 1.0 / (mx / 2.0);
  return ag;
}

int read_aff(stml_ctx* c) {
  HIP_OK(hipMemcpyAsync(c->hast, c->ast, sizeof(AffState),
                        hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipMemcpyAsync(c->hasc, c->ab.sc, sizeof(AffScal),
                        hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  return STML_OK;
}

// Objective (and gradient into gout) of the frames Kdev at x + t dv.
int aff_objective(stml_ctx* c, int level, const int* Kdev, int nk,
                  const double* x, const double* dv, double t, double* gout,
                  bool reuse_gram) {
  AffBufs b = c->ab;
  b.gout = gout;
  HIP_OK(launch_aff_objective(c->lv[level].T, Kdev, nk, x, dv, t,
                              aff_geom(c, level), c->o.lambda, b,
                              gout != nullptr, reuse_gram, c->stream));
  return STML_OK;
}

// GIR(level, K_q) of the affine model: L-BFGS on the parameters of K_q,
// every decision on the device; the host waits once per trial step.
int aff_register(stml_ctx* c, int level, int q, stml_gir_log* log) {
  const stml_opts& o = c->o;
  const int nk = (int)c->K[q].size(), P = c->npar, nP = nk * P;
  const int* Kd = c->qt[q].K;
  const int mem = o.lbfgs_mem;
  double* theta = c->alv[level].Y;
  std::memset(log, 0, sizeof *log);
  log->n_frames = nk;
  HIP_OK(launch_aff_gather(c->ax, theta, Kd, nk, P, false, c->stream));
  int rc = aff_objective(c, level, Kd, nk, c->ax, nullptr, 0.0, c->agr,
                         false);
  if (rc) return rc;
  HIP_OK(launch_aff_state_init(c->ast, c->ab.sc, c->stream));
  rc = read_aff(c);
  if (rc) return rc;
  if (c->hast->bad)
    return fail(c, STML_EINVAL, "a frame has no contrast after warping");
  log->J0 = log->J = c->hast->J;
  int status = STML_OK;
  for (int it = 0; it < o.gn_max; ++it) {
    HIP_OK(launch_aff_direction(c->ast, c->agr, c->ad, c->aS, c->aY, nP, mem,
                                c->stream));
    bool accepted = false;
    double t = 1.0;
    for (int ti = 0; ti <= o.ls_max; ++ti) {
      t = std::ldexp(1.0, -ti);
      rc = aff_objective(c, level, Kd, nk, c->ax, c->ad, t, nullptr, false);
      if (rc) return rc;
      HIP_OK(launch_aff_accept(c->ast, c->ab.sc, t, o.c1, c->stream));
      rc = read_aff(c);
      if (rc) return rc;
      if (c->hast->bad)
        return fail(c, STML_EINVAL, "a frame has no contrast after warping");
      if (c->hast->accepted) {
        accepted = true;
        break;
      }
    }
    if (!accepted) {
      status = STML_WLINESEARCH;
      break;
    }
    rc = aff_objective(c, level, Kd, nk, c->ax, c->ad, t, c->agn, true);
    if (rc) return rc;
    HIP_OK(launch_aff_update(c->ast, c->ax, c->ad, c->agr, c->agn, c->aS,
                             c->aY, nP, mem, o.tol_J, o.tol_u, c->stream));
    rc = read_aff(c);
    if (rc) return rc;
    if (it < 64) {
      log->step[it] = t;
      log->J_iter[it] = c->hast->J;
    }
    log->gn_iterations += 1;
    log->J = c->hast->J;
    if (!o.parity_mode && c->hast->stop) break;
  }
  HIP_OK(launch_aff_gather(c->ax, theta, Kd, nk, P, true, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  log->D = c->hasc->D;
  log->P = c->hasc->P;
  log->S = 0.0;
  log->status = status;
  log->predictor = q > 0 ? 0 : -1;
  return status;
}

int aff_predict(stml_ctx* c, int level, int q_next) {
  const int n = c->n, P = c->npar;
  const size_t bytes = (size_t)n * P * sizeof(double);
  stml_ctx::AffLevel& a = c->alv[level];
  if (q_next == 0) {
    if (level == 0)
      HIP_OK(hipMemsetAsync(a.Z, 0, bytes, c->stream));
    else   // the same parameters mean the same map on every level
      HIP_OK(hipMemcpyAsync(a.Z, c->alv[level - 1].Y, bytes,
                            hipMemcpyDeviceToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(a.Y, a.Z, bytes, hipMemcpyDeviceToDevice,
                          c->stream));
  } else if (level == 0) {
    HIP_OK(launch_aff_linear_predict(a.Y, a.Z, c->qt[q_next - 1].lin, n, P,
                                     c->stream));
  } else {
    HIP_OK(launch_aff_ls_predict(a.Y, a.Z, c->qt[q_next - 1].thomas, n, P,
                                 c->o.beta, c->adp, c->stream));
  }
  HIP_OK(hipStreamSynchronize(c->stream));
  return STML_OK;
}

// D over all frames at the parameters U ([n][P], device).
int aff_all_frame_D(stml_ctx* c, int level, const double* U, double* out) {
  const int T = c->T1 - 1;
  int rc = aff_objective(c, level, c->qt[T].K, c->n, U, nullptr, 0.0,
                         nullptr, false);
  if (rc) return rc;
  rc = read_aff(c);
  if (rc) return rc;
  if (c->hasc->bad)
    return fail(c, STML_EINVAL, "a frame has no contrast after warping");
  *out = c->hasc->D;
  return STML_OK;
}

int do_predict(stml_ctx* c, int level, int q_next) {
  if (c->o.model == STML_MODEL_AFFINE) return aff_predict(c, level, q_next);
  const int n = c->n, D = c->d;
  LevelBufs& b = c->lv[level];
  const size_t cnt = (size_t)n * D * c->N[level];
  const double vf = (double)n * c->N[level];
  c->pick = stml_ctx::Pick{};
  const bool learned = q_next > 0 && net_fits(c, level);
  if (learned)
    HIP_OK(hipMemcpyAsync(c->ureg, b.Y, cnt * sizeof(float),
                          hipMemcpyDeviceToDevice, c->stream));
  if (q_next == 0) {
    if (level == 0) {
      HIP_OK(launch_fill(b.Z, cnt, 0.0f, c->stream));
    } else {
      Geom gc = geom_of(c, level - 1), gf = geom_of(c, level);
      TIMED(STML_K_PREDICT, level, vf,
            launch_prolong(D, c->lv[level - 1].Y, b.Z, n * D, gc, gf,
                           c->stream));
    }
    HIP_OK(hipMemcpyAsync(b.Y, b.Z, cnt * sizeof(float),
                          hipMemcpyDeviceToDevice, c->stream));
  } else if (level == 0) {
    TIMED(STML_K_PREDICT, level, vf,
          launch_linear_predict(b.Y, b.Z, b.Y, c->qt[q_next - 1].lin, n, D,
                                c->N[level], c->stream));
  } else {
    TIMED(STML_K_PREDICT, level, vf,
          launch_ls_predict(b.Y, b.Z, c->qt[q_next - 1].thomas, n, D,
                            c->N[level], c->o.beta, c->stream));
  }
  HIP_OK(hipStreamSynchronize(c->stream));
  if (q_next > 0) c->pick.used = 0;
  if (learned) return learned_predict(c, level, q_next);
  return STML_OK;
}

int record_gir(stml_ctx* c, int level, int q, int rc, stml_gir_log& log);

int do_register(stml_ctx* c, int level, int q) {
  stml_gir_log log;
  if (c->o.model == STML_MODEL_AFFINE) {
    int rc = aff_register(c, level, q, &log);
    return record_gir(c, level, q, rc, log);
  }
  const double target = c->targets.empty()
                            ? -INFINITY
                            : c->targets[(size_t)level * c->T1 + q];
  int rc = gauss_newton(c, level, c->qt[q].K, (int)c->K[q].size(),
                        c->lv[level].Y, &log, target);
  return record_gir(c, level, q, rc, log);
}

// Keep the log of GIR(level, K_q) and turn its status into the return code.
int record_gir(stml_ctx* c, int level, int q, int rc, stml_gir_log& log) {
  if (rc < 0 && rc != STML_EBREAKDOWN) return rc;
  log.level = level;
  log.q = q;
  log.predictor = c->pick.used;
  log.J_paper = c->pick.Jp;
  log.J_learned = c->pick.Jl;
  c->pick = stml_ctx::Pick{};
  c->logs.push_back(log);
  if (rc == STML_EBREAKDOWN) return fail(c, rc, "CG breakdown (p.Hp <= 0)");
  if (rc == STML_WLINESEARCH)
    return fail(c, rc, "Armijo search found no step at level %d q %d", level,
                q);
  return STML_OK;
}

// D over all frames at an all-frame estimate U (eq. (3) test).
int all_frame_D(stml_ctx* c, int level, const float* U, double* out) {
  const int T = c->T1 - 1;
  const Geom g = geom_of(c, level);
  const Model md = model_of(c, level, c->n);
  HIP_OK(launch_eval(c->d, c->lv[level].T, U, c->qt[T].K, g, md, nullptr,
                     nullptr, c->rb, c->sc, c->stream, true, 0));
  int rc = read_scal(c);
  if (rc) return rc;
  *out = c->hsc->D;
  return STML_OK;
}

}  // namespace

// ================================================================= C-ABI

extern "C" {

void stml_default_opts(stml_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->dim = 2;
  o->n_spatial = 2;
  o->n_temporal = 2;
  o->regulariser = STML_REG_DIFFUSION;
  o->alpha = 1e-2;
  o->lambda = 1e-2;
  o->beta = 1e-5;
  o->eps_stop = 0.0;
  o->gn_max = 10;
  o->cg_max = 20;
  o->cg_rtol = 0.1;
  o->ls_max = 10;
  o->c1 = 1e-4;
  o->tol_J = 1e-3;
  o->tol_u = 1e-2;
  o->predictor = 0;
  o->parity_mode = 0;
  o->stop_relative = 0;
  o->model = STML_MODEL_FIELD;
  o->lbfgs_mem = 5;
}

size_t stml_workspace_bytes(const stml_opts* o, int n, const int* extent) {
  stml_ctx tmp;
  if (!setup_dims(&tmp, o, n, extent)) return 0;
  return layout(&tmp, nullptr);
}

int stml_create(const stml_opts* o, int n, const int* extent, void* stream,
                void* ws, size_t ws_bytes, stml_ctx** out) {
  if (!out) return STML_EINVAL;
  *out = nullptr;
  stml_ctx* c = new stml_ctx();
  if (!setup_dims(c, o, n, extent)) {
    delete c;
    return STML_EINVAL;
  }
  size_t need = layout(c, nullptr);
  if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign)) {
    delete c;
    return ws && ws_bytes < need ? STML_ENOMEM : STML_EINVAL;
  }
  layout(c, static_cast<char*>(ws));
  c->stream = static_cast<hipStream_t>(stream);
  if (hipHostMalloc((void**)&c->hsc, sizeof(Scal), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&c->hk, STML_MAX_FRAMES * sizeof(int),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->hlog,
                    (o->gn_max > 0 ? o->gn_max : 1) * sizeof(GNLog),
                    hipHostMallocDefault) != hipSuccess ||
      (o->model == STML_MODEL_AFFINE &&
       (hipHostMalloc((void**)&c->hast, sizeof(AffState),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->hasc, sizeof(AffScal),
                      hipHostMallocDefault) != hipSuccess))) {
    stml_destroy(c);
    return STML_EDEVICE;
  }
  if (hipMemsetAsync(c->sc, 0, sizeof(Scal), c->stream) != hipSuccess ||
      upload_tables(c) != STML_OK) {
    stml_destroy(c);
    return STML_EDEVICE;
  }
  *out = c;
  return STML_OK;
}

void stml_destroy(stml_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  tresolve(c);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  if (c->hsc) (void)hipHostFree(c->hsc);
  if (c->hk) (void)hipHostFree(c->hk);
  if (c->hlog) (void)hipHostFree(c->hlog);
  if (c->hast) (void)hipHostFree(c->hast);
  if (c->hasc) (void)hipHostFree(c->hasc);
  delete c;
}

const char* stml_last_error(const stml_ctx* c) {
  return c ? c->err.c_str() : "null context";
}

int stml_set_sequence(stml_ctx* c, const float* frames_dev) {
  if (!c) return STML_EINVAL;
  if (!frames_dev) return fail(c, STML_EINVAL, "null frames");
  const int n = c->n, D = c->d, L = c->L;
  size_t cnt = (size_t)n * c->N[L - 1];
  HIP_OK(hipMemsetAsync(&c->sc->bad, 0, sizeof(int), c->stream));
  HIP_OK(launch_check_finite(frames_dev, cnt, c->sc, c->stream));
  HIP_OK(hipMemcpyAsync(c->lv[L - 1].T, frames_dev, cnt * sizeof(float),
                        hipMemcpyDeviceToDevice, c->stream));
  for (int l = L - 1; l > 0; --l) {
    Geom gf = geom_of(c, l), gc = geom_of(c, l - 1);
    TIMED(STML_K_RESTRICT, l - 1, (double)n * gc.N,
          launch_restrict(D, c->lv[l].T, c->lv[l - 1].T, n, gf, gc,
                          c->stream));
  }
  for (int l = 0; l < L; ++l) {
    if (c->o.model == STML_MODEL_AFFINE) {
      size_t pc = (size_t)n * c->npar * sizeof(double);
      HIP_OK(hipMemsetAsync(c->alv[l].Y, 0, pc, c->stream));
      HIP_OK(hipMemsetAsync(c->alv[l].Z, 0, pc, c->stream));
      continue;
    }
    size_t vc = (size_t)n * D * c->N[l];
    HIP_OK(launch_fill(c->lv[l].Y, vc, 0.0f, c->stream));
    HIP_OK(launch_fill(c->lv[l].Z, vc, 0.0f, c->stream));
  }
  int rc = read_scal(c);
  if (rc) return rc;
  if (c->hsc->bad) {
    c->have_seq = false;
    return fail(c, STML_EINVAL, "%d non-finite frame values", c->hsc->bad);
  }
  c->have_seq = true;
  c->logs.clear();
  return STML_OK;
}

int stml_get_level_frames(const stml_ctx* cc, int level, float* out) {
  stml_ctx* c = const_cast<stml_ctx*>(cc);
  if (!c) return STML_EINVAL;
  int rc = check_level(c, level);
  if (rc) return rc;
  if (!c->have_seq) return fail(c, STML_ESTATE, "no sequence");
  HIP_OK(hipMemcpyAsync(out, c->lv[level].T,
                        (size_t)c->n * c->N[level] * sizeof(float),
                        hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  return STML_OK;
}

int stml_level_extent(const stml_ctx* cc, int level, int* out_extent) {
  stml_ctx* c = const_cast<stml_ctx*>(cc);
  if (!c || !out_extent) return STML_EINVAL;
  int rc = check_level(c, level);
  if (rc) return rc;
  for (int a = 0; a < c->d; ++a) out_extent[a] = c->ext[level][a];
  return STML_OK;
}

int stml_temporal_set(const stml_ctx* cc, int q, int* out, int cap) {
  stml_ctx* c = const_cast<stml_ctx*>(cc);
  if (!c) return STML_EINVAL;
  if (q < 0 || q >= c->T1) return fail(c, STML_EINVAL, "q %d out of range", q);
  const std::vector<int>& Kq = c->K[q];
  for (int i = 0; i < (int)Kq.size() && i < cap; ++i) out[i] = Kq[i];
  return (int)Kq.size();
}

int stml_predict(stml_ctx* c, int level, int q_next) {
  if (!c) return STML_EINVAL;
  int rc = check_level(c, level);
  if (rc) return rc;
  if (q_next < 0 || q_next >= c->T1)
    return fail(c, STML_EINVAL, "q_next %d out of range", q_next);
  if (!c->have_seq) return fail(c, STML_ESTATE, "no sequence");
  return do_predict(c, level, q_next);
}

int stml_register_level(stml_ctx* c, int level, int q) {
  if (!c) return STML_EINVAL;
  int rc = check_level(c, level);
  if (rc) return rc;
  if (q < 0 || q >= c->T1) return fail(c, STML_EINVAL, "q %d out of range", q);
  if (!c->have_seq) return fail(c, STML_ESTATE, "no sequence");
  return do_register(c, level, q);
}

int stml_correct(stml_ctx* c, int level, int q_next) {
  return stml_register_level(c, level, q_next);
}

int stml_run(stml_ctx* c) {
  if (!c) return STML_EINVAL;
  if (!c->have_seq) return fail(c, STML_ESTATE, "no sequence");
  const int T = c->T1 - 1;
  const bool eq3 = c->o.eps_stop > 0 && !c->o.parity_mode;
  int warn = STML_OK;
  c->stop_trace.assign(c->L, std::vector<double>());
  c->stop_q.assign(c->L, -1);
  for (int level = 0; level < c->L; ++level) {
    int rc = do_predict(c, level, 0);
    if (rc < 0) return rc;
    rc = do_register(c, level, 0);
    if (rc < 0) return rc;
    if (rc > 0) warn = rc;
    bool have_prev = false;
    double D_prev = 0.0;
    const size_t cnt = (size_t)c->n * c->d * c->N[level];
    for (int q = 0; q < T; ++q) {
      if (c->o.model == STML_MODEL_AFFINE) {
        stml_ctx::AffLevel& a = c->alv[level];
        const size_t pb = (size_t)c->n * c->npar * sizeof(double);
        if (eq3)
          HIP_OK(hipMemcpyAsync(c->anow, a.Y, pb, hipMemcpyDeviceToDevice,
                                c->stream));
        rc = do_predict(c, level, q + 1);
        if (rc < 0) return rc;
        if (eq3) {
          // estimate = prediction, with the frames of K_q as registered
          const int nq = (int)c->K[q].size();
          HIP_OK(hipMemcpyAsync(c->aest, a.Y, pb, hipMemcpyDeviceToDevice,
                                c->stream));
          HIP_OK(launch_aff_gather(c->ax, c->anow, c->qt[q].K, nq, c->npar,
                                   false, c->stream));
          HIP_OK(launch_aff_gather(c->ax, c->aest, c->qt[q].K, nq, c->npar,
                                   true, c->stream));
          double Dq;
          rc = aff_all_frame_D(c, level, c->aest, &Dq);
          if (rc) return rc;
          c->stop_trace[level].push_back(Dq);
          const double tol =
              c->o.eps_stop * (c->o.stop_relative ? std::fabs(Dq) : 1.0);
          if (have_prev && std::fabs(Dq - D_prev) <= tol) {
            HIP_OK(hipMemcpyAsync(a.Y, c->aest, pb, hipMemcpyDeviceToDevice,
                                  c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
            c->stop_q[level] = q;
            break;
          }
          D_prev = Dq;
          have_prev = true;
        }
        rc = do_register(c, level, q + 1);
        if (rc < 0) return rc;
        if (rc > 0) warn = rc;
        continue;
      }
      LevelBufs& b = c->lv[level];
      if (eq3) {
        // keep the registered frames of K_q for the all-frame estimate
        HIP_OK(hipMemcpyAsync(c->x, b.Y, cnt * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream));
      }
      rc = do_predict(c, level, q + 1);
      if (rc < 0) return rc;
      if (eq3) {
        // estimate = prediction, with the frames of K_q as registered
        HIP_OK(hipMemcpyAsync(c->r, b.Y, cnt * sizeof(float),
                              hipMemcpyDeviceToDevice, c->stream));
        size_t fr = (size_t)c->d * c->N[level];
        for (int k : c->K[q])
          HIP_OK(hipMemcpyAsync(c->r + k * fr, c->x + k * fr,
                                fr * sizeof(float), hipMemcpyDeviceToDevice,
                                c->stream));
        double Dq;
        rc = all_frame_D(c, level, c->r, &Dq);
        if (rc) return rc;
        c->stop_trace[level].push_back(Dq);
        // eq. (3) as printed: |D_q - D_{q-1}| <= eps (relative on request)
        const double tol =
            c->o.eps_stop * (c->o.stop_relative ? std::fabs(Dq) : 1.0);
        if (have_prev && std::fabs(Dq - D_prev) <= tol) {
          HIP_OK(hipMemcpyAsync(b.Y, c->r, cnt * sizeof(float),
                                hipMemcpyDeviceToDevice, c->stream));
          HIP_OK(hipStreamSynchronize(c->stream));
          c->stop_q[level] = q;
          break;
        }
        D_prev = Dq;
        have_prev = true;
      }
      rc = do_register(c, level, q + 1);
      if (rc < 0) return rc;
      if (rc > 0) warn = rc;
    }
  }
  return warn;
}

int stml_get_stop_trace(const stml_ctx* cc, int level, double* D_out,
                        int cap, int* stop_q) {
  stml_ctx* c = const_cast<stml_ctx*>(cc);
  if (!c) return STML_EINVAL;
  int rc = check_level(c, level);
  if (rc) return rc;
  if (cap < 0 || (cap > 0 && !D_out))
    return fail(c, STML_EINVAL, "D_out must hold cap values");
  if ((int)c->stop_trace.size() != c->L) {
    if (stop_q) *stop_q = -1;
    return 0;
  }
  const std::vector<double>& tr = c->stop_trace[level];
  for (int i = 0; i < (int)tr.size() && i < cap; ++i) D_out[i] = tr[i];
  if (stop_q) *stop_q = c->stop_q[level];
  return (int)tr.size();
}

static int copy_field(stml_ctx* c, int level, float* dst, const float* src) {
  int rc = check_level(c, level);
  if (rc) return rc;
  if (!dst || !src) return fail(c, STML_EINVAL, "null pointer");
  HIP_OK(hipMemcpyAsync(dst, src, (size_t)c->n * c->d * c->N[level] *
                                      sizeof(float),
                        hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  return STML_OK;
}

static int field_only(stml_ctx* c) {
  if (c->o.model != STML_MODEL_FIELD)
    return fail(c, STML_EINVAL, "not available for the affine model");
  return STML_OK;
}

int stml_get_displacements(const stml_ctx* cc, int level, float* u) {
  stml_ctx* c = const_cast<stml_ctx*>(cc);
  if (!c) return STML_EINVAL;
  if (check_level(c, level)) return STML_EINVAL;
  if (c->o.model == STML_MODEL_AFFINE) {
    if (!u) return fail(c, STML_EINVAL, "null pointer");
    HIP_OK(launch_aff_field(c->alv[level].Y, c->n, aff_geom(c, level), u,
                            c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    return STML_OK;
  }
  return copy_field(c, level, u, c->lv[level].Y);
}

int stml_set_displacements(stml_ctx* c, int level, const float* u) {
  if (!c) return STML_EINVAL;
  if (check_level(c, level)) return STML_EINVAL;
  if (field_only(c)) return STML_EINVAL;
  return copy_field(c, level, c->lv[level].Y, u);
}

int stml_get_prediction(const stml_ctx* cc, int level, float* z) {
  stml_ctx* c = const_cast<stml_ctx*>(cc);
  if (!c) return STML_EINVAL;
  if (check_level(c, level)) return STML_EINVAL;
  if (field_only(c)) return STML_EINVAL;
  return copy_field(c, level, z, c->lv[level].Z);
}

int stml_set_prediction(stml_ctx* c, int level, const float* z) {
  if (!c) return STML_EINVAL;
  if (check_level(c, level)) return STML_EINVAL;
  if (field_only(c)) return STML_EINVAL;
  return copy_field(c, level, c->lv[level].Z, z);
}

int stml_set_targets(stml_ctx* c, const double* J_targets) {
  if (!c) return STML_EINVAL;
  if (!J_targets) {
    c->targets.clear();
    return STML_OK;
  }
  if (c->o.model != STML_MODEL_FIELD)
    return fail(c, STML_EINVAL, "targets apply to the field model");
  const size_t cnt = (size_t)c->L * c->T1;
  for (size_t i = 0; i < cnt; ++i)
    if (std::isnan(J_targets[i]))
      return fail(c, STML_EINVAL, "target %zu is NaN", i);
  c->targets.assign(J_targets, J_targets + cnt);
  return STML_OK;
}

int stml_get_params(const stml_ctx* cc, int level, double* theta) {
  stml_ctx* c = const_cast<stml_ctx*>(cc);
  if (!c) return STML_EINVAL;
  if (check_level(c, level)) return STML_EINVAL;
  if (c->o.model != STML_MODEL_AFFINE)
    return fail(c, STML_EINVAL, "parameters exist for the affine model only");
  if (!theta) return fail(c, STML_EINVAL, "null pointer");
  HIP_OK(hipMemcpyAsync(theta, c->alv[level].Y,
                        (size_t)c->n * c->npar * sizeof(double),
                        hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  return STML_OK;
}

int stml_set_params(stml_ctx* c, int level, const double* theta) {
  if (!c) return STML_EINVAL;
  if (check_level(c, level)) return STML_EINVAL;
  if (c->o.model != STML_MODEL_AFFINE)
    return fail(c, STML_EINVAL, "parameters exist for the affine model only");
  if (!theta) return fail(c, STML_EINVAL, "null pointer");
  for (size_t i = 0; i < (size_t)c->n * c->npar; ++i)
    if (!std::isfinite(theta[i]))
      return fail(c, STML_EINVAL, "non-finite parameter");
  HIP_OK(hipMemcpyAsync(c->alv[level].Y, theta,
                        (size_t)c->n * c->npar * sizeof(double),
                        hipMemcpyHostToDevice, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  return STML_OK;
}

int stml_eval_params(stml_ctx* c, int level, const int* frames, int nk,
                     const double* theta, double* out, double* grad) {
  if (!c) return STML_EINVAL;
  int rc = check_level(c, level);
  if (rc) return rc;
  if (c->o.model != STML_MODEL_AFFINE)
    return fail(c, STML_EINVAL, "parameters exist for the affine model only");
  if (!c->have_seq) return fail(c, STML_ESTATE, "no sequence");
  if (!theta || !out) return fail(c, STML_EINVAL, "null pointer");
  rc = stage_frames(c, frames, nk);
  if (rc) return rc;
  const int P = c->npar;
  std::vector<double> xk((size_t)nk * P);
  for (int j = 0; j < nk; ++j)
    for (int i = 0; i < P; ++i) {
      const double v = theta[(size_t)frames[j] * P + i];
      if (!std::isfinite(v)) return fail(c, STML_EINVAL, "non-finite parameter");
      xk[(size_t)j * P + i] = v;
    }
  HIP_OK(hipMemcpyAsync(c->ax, xk.data(), xk.size() * sizeof(double),
                        hipMemcpyHostToDevice, c->stream));
  rc = aff_objective(c, level, c->kbuf, nk, c->ax, nullptr, 0.0,
                     grad ? c->agr : nullptr, false);
  if (rc) return rc;
  if (grad)
    HIP_OK(hipMemcpyAsync(grad, c->agr, xk.size() * sizeof(double),
                          hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipMemcpyAsync(c->hasc, c->ab.sc, sizeof(AffScal),
                        hipMemcpyDeviceToHost, c->stream));
  HIP_OK(hipStreamSynchronize(c->stream));
  if (c->hasc->bad)
    return fail(c, STML_EINVAL, "a frame has no contrast after warping");
  out[0] = c->hasc->J;
  out[1] = c->hasc->D;
  out[2] = c->hasc->P;
  return STML_OK;
}

int stml_log_count(const stml_ctx* c) {
  return c ? (int)c->logs.size() : STML_EINVAL;
}

int stml_get_log(const stml_ctx* c, int i, stml_gir_log* out) {
  if (!c || !out || i < 0 || i >= (int)c->logs.size()) return STML_EINVAL;
  *out = c->logs[i];
  return STML_OK;
}

int stml_eval(stml_ctx* c, int level, const int* frames, int nk,
              const float* u, double* out, float* grad, float* dW) {
  if (!c) return STML_EINVAL;
  if (field_only(c)) return STML_EINVAL;
  int rc = check_level(c, level);
  if (rc) return rc;
  if (!c->have_seq) return fail(c, STML_ESTATE, "no sequence");
  if (!u || !out) return fail(c, STML_EINVAL, "null pointer");
  rc = stage_frames(c, frames, nk);
  if (rc) return rc;
  Geom g = geom_of(c, level);
  Model md = model_of(c, level, nk);
  HIP_OK(launch_eval(c->d, c->lv[level].T, u, c->kbuf, g, md,
                     grad ? grad : c->g, dW ? dW : c->dW, c->rb, c->sc,
                     c->stream, true, 0));
  rc = read_scal(c);
  if (rc) return rc;
  out[0] = c->hsc->J;
  out[1] = c->hsc->D;
  out[2] = c->hsc->S;
  out[3] = c->hsc->P;
  return STML_OK;
}

int stml_hessvec(stml_ctx* c, int level, const int* frames, int nk,
                 const float* u, const float* v, float* hv, double* vHv) {
  if (!c) return STML_EINVAL;
  if (field_only(c)) return STML_EINVAL;
  int rc = check_level(c, level);
  if (rc) return rc;
  if (!c->have_seq) return fail(c, STML_ESTATE, "no sequence");
  if (!u || !v || !hv) return fail(c, STML_EINVAL, "null pointer");
  rc = stage_frames(c, frames, nk);
  if (rc) return rc;
  Geom g = geom_of(c, level);
  Model md = model_of(c, level, nk);
  HIP_OK(launch_eval(c->d, c->lv[level].T, u, c->kbuf, g, md, c->g, c->dW,
                     c->rb, c->sc, c->stream, true, 0));
  TIMED(STML_K_HESSVEC, level, (double)nk * g.N,
        launch_hessvec_tiled(v, c->dW, g, md, hv, c->P[0], c->sums, c->rb,
                             c->sc, c->stream));
  rc = read_scal(c);
  if (rc) return rc;
  if (vHv) *vHv = c->hsc->vHv;
  return STML_OK;
}

int stml_gn_direction(stml_ctx* c, int level, const int* frames, int nk,
                      const float* u, float* delta, int* out_cg) {
  if (!c) return STML_EINVAL;
  if (field_only(c)) return STML_EINVAL;
  int rc = check_level(c, level);
  if (rc) return rc;
  if (!c->have_seq) return fail(c, STML_ESTATE, "no sequence");
  if (!u || !delta) return fail(c, STML_EINVAL, "null pointer");
  rc = stage_frames(c, frames, nk);
  if (rc) return rc;
  Geom g = geom_of(c, level);
  Model md = model_of(c, level, nk);
  HIP_OK(launch_gn_reset(c->sc, c->gnlog, 1, c->stream));
  const CgStart cs = cg_start(c);
  HIP_OK(launch_eval(c->d, c->lv[level].T, u, c->kbuf, g, md, c->g, c->dW,
                     c->rb, c->sc, c->stream, false, 0, &cs));
  rc = enqueue_pcg(c, level, g, md, 0);
  if (rc) return rc;
  HIP_OK(hipMemcpyAsync(delta, c->x, (size_t)nk * c->d * g.N * sizeof(float),
                        hipMemcpyDeviceToDevice, c->stream));
  rc = read_scal(c);
  if (rc) return rc;
  if (out_cg) *out_cg = c->hsc->iters;
  if (c->hsc->done == 2) return fail(c, STML_EBREAKDOWN, "CG breakdown");
  return STML_OK;
}

int stml_force_cg_breakdown(stml_ctx* c, int it) {
  if (!c || it < -1) return STML_EINVAL;
  c->cg_break = it;
  return STML_OK;
}

int stml_set_predictor_net(stml_ctx* c, stml_net* net) {
  if (!c) return STML_EINVAL;
  if (field_only(c)) return STML_EINVAL;
  if (net && net_dim(net) != c->d)
    return fail(c, STML_EINVAL, "learned predictor of another dimension");
  if (net && !c->ureg)
    return fail(c, STML_ESTATE, "create the context with predictor = 1");
  c->net = net;
  return STML_OK;
}

int stml_set_tuning(stml_ctx* c, const stml_tuning* t) {
  if (!c || !t) return STML_EINVAL;
  auto ok = [](int v, int hi) { return v >= 8 && v <= hi && v % 8 == 0; };
  if (!ok(t->tile_blocks, 1024) || !ok(t->vox_blocks, 1024) ||
      !ok(t->hv_blocks, 8192))
    return fail(c, STML_EINVAL, "tuning out of range");
  c->tune = *t;
  return STML_OK;
}

int stml_get_tuning(const stml_ctx* c, stml_tuning* t) {
  if (!c || !t) return STML_EINVAL;
  *t = c->tune;
  return STML_OK;
}

int stml_timing_every(stml_ctx* c, int mask, int period) {
  if (!c || mask < 0 || period < 1) return STML_EINVAL;
  HIP_OK(hipStreamSynchronize(c->stream));
  tresolve(c);
  if (mask) c->kstats.clear();
  c->timing = (unsigned)mask & ((1u << STML_K_COUNT) - 1u);
  c->tperiod = period;
  for (long long& n : c->tcount) n = 0;
  return STML_OK;
}

int stml_timing(stml_ctx* c, int mask) { return stml_timing_every(c, mask, 1); }

int stml_timing_get(stml_ctx* c, int kernel, int level, double* ms,
                    long long* n, double* vf, double* bytes) {
  if (!c || kernel < 0 || kernel >= STML_K_COUNT) return STML_EINVAL;
  HIP_OK(hipStreamSynchronize(c->stream));
  tresolve(c);
  double tms = 0.0, tvf = 0.0, tb = 0.0;
  long long tn = 0;
  for (auto& kv : c->kstats) {
    if (kv.first.first != kernel) continue;
    if (level >= 0 && kv.first.second != level) continue;
    tms += kv.second.ms;
    tvf += kv.second.vf;
    tb += kv.second.bytes;
    tn += kv.second.n;
  }
  if (ms) *ms = tms;
  if (n) *n = tn;
  if (vf) *vf = tvf;
  if (bytes) *bytes = tb;
  return STML_OK;
}

}  // extern "C"

// ============================================================ batching

struct stml_batch {
  std::vector<stml_ctx*> c;
  hipStream_t user = nullptr;     // caller's stream
  hipStream_t stream = nullptr;   // internal (graphs are captured on it)
  Job* djobs = nullptr;
  int* dfirst = nullptr;
  int* dstop = nullptr;
  Job* hjobs = nullptr;           // pinned staging
  int* hfirst = nullptr;
  int* hstop = nullptr;
  bool graph = true;               // replay a captured iteration
  std::string err;
};

namespace {

int bfail(stml_batch* b, int code, const char* fmt, ...) {
  if (b) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b->err = buf;
  }
  return code;
}

#define BHIP_OK(call)                                                       \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess)                                                   \
      return bfail(b, STML_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t batch_layout(int count, char* base, stml_batch* b) {
  Layout lo;
  lo.base = base;
  Job* j = lo.take<Job>(count);
  int* f = lo.take<int>((size_t)kClsCount * (count + 1));
  int* st = lo.take<int>(count);
  if (b) {
    b->djobs = j;
    b->dfirst = f;
    b->dstop = st;
  }
  return lo.off;
}

// One Gauss-Newton iteration of every problem of js.
hipError_t batch_iteration(const JobSet& js, const int* tot, int dim,
                           int reg, const stml_opts& o, int* dstop,
                           hipStream_t s) {
  // the evaluation also forms the CG start (r, z, sums of z); the first CG
  // update its scalars (without CG steps a one-block kernel per job does)
  hipError_t e = batch_eval(js, tot[kClsTile], dim, reg, s);
  if (e == hipSuccess && o.cg_max == 0) e = batch_finalize_start(js, s);
  if (e == hipSuccess && o.cg_max == 0) e = batch_zero_x(js, tot[kClsVox], dim, s);
  for (int it = 0; e == hipSuccess && it < o.cg_max; ++it) {
    e = batch_cg_hvp(js, tot[kClsHv], tot[kClsVox], dim, reg, it,
                     o.parity_mode, o.cg_rtol, s);
    if (e == hipSuccess)
      e = batch_cg_update(js, tot[kClsVox], dim, it, o.cg_max, s);
  }
  const int sweeps = sweep_count(o.ls_max);
  for (int p = 0; e == hipSuccess && p < sweeps; ++p)
    e = batch_trial(js, tot[kClsTile], dim, reg, p, o.ls_max, o.c1, s);
  if (e == hipSuccess)
    e = batch_accept(js, tot[kClsElem], o.ls_max, o.c1, o.parity_mode,
                     o.tol_J, o.tol_u, s);
  if (e == hipSuccess) e = batch_advance(js, dstop, s);
  return e;
}

// GIR(level, K_q) of every sequence of the batch, in shared launches.
int batch_register(stml_batch* b, int level, int q) {
  const int S = (int)b->c.size();
  const stml_opts& o = b->c[0]->o;
  int tot[kClsCount] = {};
  for (int cl = 0; cl < kClsCount; ++cl) b->hfirst[cl * (S + 1)] = 0;
  for (int j = 0; j < S; ++j) {
    stml_ctx* c = b->c[j];
    Job& J = b->hjobs[j];
    J.T = c->lv[level].T;
    J.u = c->lv[level].Y;
    J.K = c->qt[q].K;
    J.g = geom_of(c, level);
    J.md = model_of(c, level, (int)c->K[q].size());
    J.grad = c->g;
    J.dW = c->dW;
    J.x = c->x;
    J.r = c->r;
    J.z = c->z;
    J.q = c->q;
    J.P0 = c->P[0];
    J.P1 = c->P[1];
    J.sums = c->sums;
    J.rb = c->rb;
    J.sc = c->sc;
    J.log = c->gnlog;
    job_shape(&J);
    const int nb[kClsCount] = {J.nb_tile, J.nb_vox, J.ct.grid, 1, J.nb_elem};
    for (int cl = 0; cl < kClsCount; ++cl) {
      tot[cl] += nb[cl];
      b->hfirst[cl * (S + 1) + j + 1] = tot[cl];
    }
  }
  BHIP_OK(hipMemcpyAsync(b->djobs, b->hjobs, S * sizeof(Job),
                         hipMemcpyHostToDevice, b->stream));
  BHIP_OK(hipMemcpyAsync(b->dfirst, b->hfirst,
                         (size_t)kClsCount * (S + 1) * sizeof(int),
                         hipMemcpyHostToDevice, b->stream));
  const JobSet js{b->djobs, b->dfirst, S};
  const int reg = o.regulariser;
  const int dim = b->c[0]->d;
  BHIP_OK(batch_gn_reset(js, o.gn_max, b->stream));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (b->graph && o.gn_max > 0) {
    BHIP_OK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = batch_iteration(js, tot, dim, reg, o, b->dstop,
                                   b->stream);
    hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return bfail(b, STML_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    }
  }
  hipError_t e = hipSuccess;
  for (int it = 0; it < o.gn_max && e == hipSuccess; ++it) {
    e = exec ? hipGraphLaunch(exec, b->stream)
             : batch_iteration(js, tot, dim, reg, o, b->dstop, b->stream);
    if (e != hipSuccess || o.parity_mode) continue;
    e = hipMemcpyAsync(b->hstop, b->dstop, S * sizeof(int),
                       hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    bool all = true;
    for (int j = 0; j < S && all; ++j) all = b->hstop[j] != 0;
    if (all) break;
  }
  hipError_t es = hipStreamSynchronize(b->stream);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (e == hipSuccess) e = es;
  if (e != hipSuccess)
    return bfail(b, STML_EDEVICE, "batched iteration: %s",
                 hipGetErrorString(e));
  int worst = STML_OK;
  for (int j = 0; j < S; ++j) {
    stml_ctx* c = b->c[j];
    stml_gir_log log;
    int rc = gn_log(c, (int)c->K[q].size(), c->N[level], &log);
    rc = record_gir(c, level, q, rc, log);
    if (rc < 0 && worst >= 0) {
      worst = rc;
      b->err = "sequence " + std::to_string(j) + ": " + c->err;
    } else if (rc > 0 && worst == STML_OK) {
      worst = rc;
    }
  }
  return worst;
}

int batch_check(stml_batch* b, int level) {
  for (size_t j = 0; j < b->c.size(); ++j) {
    stml_ctx* c = b->c[j];
    if (!c->have_seq)
      return bfail(b, STML_ESTATE, "sequence %zu: no sequence set", j);
    if (level < 0 || level >= c->L)
      return bfail(b, STML_EINVAL, "level %d out of range", level);
  }
  if (b->user) BHIP_OK(hipStreamSynchronize(b->user));
  return STML_OK;
}

}  // namespace

extern "C" {

size_t stml_batch_workspace_bytes(int count) {
  if (count < 1) return 0;
  return batch_layout(count, nullptr, nullptr);
}

int stml_batch_create(stml_ctx* const* ctxs, int count, void* stream,
                      void* ws, size_t ws_bytes, stml_batch** out) {
  if (!out) return STML_EINVAL;
  *out = nullptr;
  if (!ctxs || count < 1) return STML_EINVAL;
  const stml_ctx* a = ctxs[0];
  if (!a) return STML_EINVAL;
  for (int j = 0; j < count; ++j) {
    const stml_ctx* c = ctxs[j];
    if (!c || c->o.model != STML_MODEL_FIELD || c->d != a->d ||
        c->L != a->L || c->T1 != a->T1 ||
        c->o.regulariser != a->o.regulariser || c->o.gn_max != a->o.gn_max ||
        c->o.cg_max != a->o.cg_max || c->o.ls_max != a->o.ls_max ||
        c->o.parity_mode != a->o.parity_mode || c->o.c1 != a->o.c1 ||
        c->o.cg_rtol != a->o.cg_rtol || c->o.tol_J != a->o.tol_J ||
        c->o.tol_u != a->o.tol_u ||
        (c->o.eps_stop > 0 && !c->o.parity_mode))
      return STML_EINVAL;
    for (int i = 0; i < j; ++i)
      if (ctxs[i] == c) return STML_EINVAL;
  }
  const size_t need = batch_layout(count, nullptr, nullptr);
  if (!ws || ws_bytes < need || ((uintptr_t)ws % kAlign))
    return ws && ws_bytes < need ? STML_ENOMEM : STML_EINVAL;
  stml_batch* b = new stml_batch();
  b->c.assign(ctxs, ctxs + count);
  b->user = static_cast<hipStream_t>(stream);
  batch_layout(count, static_cast<char*>(ws), b);
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) !=
          hipSuccess ||
      hipHostMalloc((void**)&b->hjobs, count * sizeof(Job),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->hfirst,
                    (size_t)kClsCount * (count + 1) * sizeof(int),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->hstop, count * sizeof(int),
                    hipHostMallocDefault) != hipSuccess) {
    stml_batch_destroy(b);
    return STML_EDEVICE;
  }
  *out = b;
  return STML_OK;
}

void stml_batch_destroy(stml_batch* b) {
  if (!b) return;
  if (b->stream) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipStreamDestroy(b->stream);
  }
  if (b->hjobs) (void)hipHostFree(b->hjobs);
  if (b->hfirst) (void)hipHostFree(b->hfirst);
  if (b->hstop) (void)hipHostFree(b->hstop);
  delete b;
}

const char* stml_batch_last_error(const stml_batch* b) {
  return b ? b->err.c_str() : "null batch";
}

int stml_batch_set_graph(stml_batch* b, int on) {
  if (!b) return STML_EINVAL;
  b->graph = on != 0;
  return STML_OK;
}

int stml_batch_predict(stml_batch* b, int level, int q_next) {
  if (!b) return STML_EINVAL;
  int rc = batch_check(b, level);
  if (rc) return rc;
  for (size_t j = 0; j < b->c.size(); ++j) {
    stml_ctx* c = b->c[j];
    if (q_next < 0 || q_next >= c->T1)
      return bfail(b, STML_EINVAL, "q_next %d out of range", q_next);
    rc = do_predict(c, level, q_next);
    if (rc < 0)
      return bfail(b, rc, "sequence %zu: %s", j, c->err.c_str());
  }
  return STML_OK;
}

int stml_batch_register_level(stml_batch* b, int level, int q) {
  if (!b) return STML_EINVAL;
  int rc = batch_check(b, level);
  if (rc) return rc;
  if (q < 0 || q >= b->c[0]->T1)
    return bfail(b, STML_EINVAL, "q %d out of range", q);
  return batch_register(b, level, q);
}

int stml_batch_run(stml_batch* b) {
  if (!b) return STML_EINVAL;
  int rc = batch_check(b, 0);
  if (rc) return rc;
  const int L = b->c[0]->L, T = b->c[0]->T1 - 1;
  int warn = STML_OK;
  for (int level = 0; level < L; ++level) {
    for (int q = 0; q <= T; ++q) {
      rc = stml_batch_predict(b, level, q);
      if (rc < 0) return rc;
      rc = batch_register(b, level, q);
      if (rc < 0) return rc;
      if (rc > 0) warn = rc;
    }
  }
  return warn;
}

}  // extern "C"
