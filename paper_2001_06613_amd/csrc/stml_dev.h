// Device-side shared definitions for the STML kernels (gfx950, wave64).
//
// Layout in HBM: images [n][N], displacement-like fields [frames][D][N],
// N = voxels of one level, last axis fastest.  Compact solver vectors hold
// the |K| frames of the subset being registered, in the order of K.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stml {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kMaxFPT = 16;        // max frames one thread keeps in registers
constexpr int kMaxChunks = 16;     // waves per block -> |K| <= 256
constexpr int kMaxFrames = 256;    // frames of a sequence (the C-ABI maximum)
constexpr int kTrialSteps = 10;    // Armijo steps of a sweep after the first
constexpr int kXCD = 8;            // MI355X: 8 accelerator complex dies
constexpr int kCUs = 256;          // compute units (32 per die)
constexpr int kMaxTileBlocks = 512;    // default block caps
constexpr int kHvBlocks = 2048;
constexpr int kMaxElemBlocks = 1024;

// Level geometry.  D = 2 uses m[0] (slow) and m[1] (fast); D = 3 uses all.
struct Geom {
  int m[3];
  long long s[3];      // strides (elements) of each axis
  long long N;         // voxels
  double inv_h;        // 1 / cell width (finest-pixel units)
  // launch shape (host side only): block caps of the tile and voxel-major
  // kernels, and the block target of the 2-D Hessian product
  int tile_cap, vox_cap, hv_target;
};

__host__ __device__ inline int geom_dim(const Geom& g) {
  return g.s[2] == 1 ? 3 : 2;
}

// Constants of the model on one level and subset.
struct Model {
  double hd;           // h^D
  double data_c;       // 2 h^D
  double mdiag_c;      // 2 h^D (1 - 1/|K|)
  double alpha_hd;     // alpha h^D
  double half_alpha_hd;
  double lam_hd;       // lambda h^D
  double lam_c;        // 2 lambda h^D / |K|
  double pen_diag;     // 2 lambda h^D / |K|^2
  double reg_scale;    // 1/h^2 (diffusion) or 1/h^4 (curvature)
  double inv_nK;
  int reg;             // 0 diffusion, 1 curvature
  int nK;
};

// Device-resident scalars of one Gauss-Newton step.  Written only by the
// last block of a kernel, read by later kernels.
struct Scal {
  double J, D, S, P;          // objective at the evaluation point
  double rzh[2];              // r.z of CG iteration it in slot it & 1
  double r0, a, beta;         // CG scalars
  double pq, rr;
  double vHv;
  int done;                   // 0 running, 1 converged, 2 breakdown
  int iters;                  // CG iterations taken
  int bad;                    // non-finite input count
  int gn_stop;                // Gauss-Newton iterations >= gn_stop do nothing
  int gn_cur;                 // iteration of batched (graph) launches
  double J_target;            // stop once J <= J_target (-inf: no target)
  double ah[2];               // CG step length of iteration it in slot it & 1
};

// One Gauss-Newton iteration as decided on the device.
struct GNLog {
  double J;                   // objective at the evaluation
  double J0t;                 // objective at t = 0 in the trial sweep
  double Jacc;                // objective at the accepted step
  double t;                   // accepted step
  double slope, maxd;         // g . delta and max |delta|
  double ssqd;                // sum of delta^2
  int cg;                     // CG iterations
  int status;                 // -1 not run, 0 accepted, 1 no step found,
                              // 2 accepted after a CG breakdown
  int next_pass;              // last line-search sweep that ran
  int pad;
};

// Terms of the CG solution x = sum_i a_i p_i that the update of CG step it
// (of cg_max) writes.  An even step other than the last leaves x alone; the
// odd step after it adds both steps' terms, p of the previous step being
// still in the other buffer of the direction pair, so x is read and written
// every second step only; the last step completes x.  A CG that stops after
// an even step (convergence found by the next step's first kernel, or a
// breakdown at the next update) has that kernel add the pending term.
enum CgXMode {
  kXNone = 0,      // x untouched
  kXOne = 1,       // x += a p (x = a p at step 0)
  kXTwo = 2,       // x += a' p' + a p
  kXTwoFirst = 3,  // x = a' p' + a p (step 1)
};
__host__ __device__ inline int cg_x_mode(int it, int cg_max) {
  if (it & 1) return it == 1 ? kXTwoFirst : kXTwo;
  return it == cg_max - 1 ? kXOne : kXNone;
}

// Armijo schedule of one Gauss-Newton iteration, t = 2^-e for e = 0, 1,
// ..., ls_max, in sweeps: sweep 0 evaluates t = 0 (the reference value,
// taken by the same formula as the steps) and t = 1; sweep p >= 1
// evaluates kTrialSteps steps, e = 1 + kTrialSteps (p - 1) + s (entries
// past ls_max repeat 2^-ls_max and are not tested).
constexpr int kSweep0Steps = 2;
__host__ __device__ inline int sweep_steps(int p) {
  return p == 0 ? kSweep0Steps : kTrialSteps;
}
__host__ __device__ inline int sweep_count(int ls_max) {
  return 1 + (ls_max + kTrialSteps - 1) / kTrialSteps;
}
// exponent of step s of sweep p; -1 for t = 0
__host__ __device__ inline int sweep_exp(int p, int s) {
  return p == 0 ? s - 1 : 1 + kTrialSteps * (p - 1) + s;
}
__host__ __device__ inline bool sweep_tests(int p, int s, int ls_max) {
  const int e = sweep_exp(p, s);
  return e >= 0 && e <= ls_max;
}
__host__ __device__ inline double sweep_t(int p, int s, int ls_max) {
  const int e = sweep_exp(p, s);
  return e < 0 ? 0.0 : ldexp(1.0, -(e <= ls_max ? e : ls_max));
}

// ---------------------------------------------------------------- helpers

// Voxel coordinates and its index inside one [N] plane.  Planes hold at
// most 2^30 voxels, so in-plane offsets are 32-bit: loads then use a
// wave-uniform plane base (scalar registers) plus a 32-bit lane offset.
template <int D>
struct Pos {
  int c[D];
  unsigned idx;
};

template <int D>
__device__ __forceinline__ Pos<D> make_pos(const Geom& g, long long x) {
  Pos<D> p;
  p.idx = (unsigned)x;
  if (D == 2) {
    int c0 = (int)(x / g.m[1]);
    p.c[0] = c0;
    p.c[1] = (int)(x - (long long)c0 * g.m[1]);
  } else {
    long long plane = (long long)g.m[1] * g.m[2];
    int c0 = (int)(x / plane);
    long long rem = x - (long long)c0 * plane;
    int c1 = (int)(rem / g.m[2]);
    p.c[0] = c0;
    p.c[1] = c1;
    p.c[D - 1] = (int)(rem - (long long)c1 * g.m[2]);
  }
  return p;
}

// Regulariser stencils.  Neighbours outside the grid are replaced by the
// voxel itself (replicate padding), which turns the plain Laplacian into the
// Neumann graph Laplacian L.  All arithmetic is float64 on float32 loads.

// Field accessor of a stored float32 plane.
struct Src1 {
  const float* __restrict__ a;
  __device__ __forceinline__ float ld(unsigned i) const { return a[i]; }
  __device__ __forceinline__ double operator()(unsigned i) const {
    return (double)a[i];
  }
};
// Offsets (in elements) of the clamped neighbours at -2, -1, +1, +2 along
// every axis, and whether the -1 / +1 neighbour exists.
template <int D>
struct Nbr {
  int m1[D], p1[D], m2[D], p2[D];
  bool hm[D], hp[D];
};

template <int D>
__device__ __forceinline__ Nbr<D> neighbours(const Pos<D>& p, const Geom& g) {
  Nbr<D> n;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int c = p.c[a], m = g.m[a];
    int s = (int)g.s[a];
    n.hm[a] = c > 0;
    n.hp[a] = c < m - 1;
    n.m1[a] = n.hm[a] ? -s : 0;
    n.p1[a] = n.hp[a] ? s : 0;
    n.m2[a] = c >= 2 ? -2 * s : n.m1[a];
    n.p2[a] = c <= m - 3 ? 2 * s : n.p1[a];
  }
  return n;
}

// (L v)(x) from the 2D face neighbours.
template <int D, class F>
__device__ __forceinline__ double lap_c(const F& v, unsigned idx,
                                        const Nbr<D>& nb) {
  double c = v(idx);
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
    s += (v(idx + nb.m1[a]) - c) + (v(idx + nb.p1[a]) - c);
  return s;
}

// Stencil points: 0 = the voxel; 1 + 2a (+0 / +1) = its -1 / +1 neighbour
// along axis a; 1 + 2D + 2a (+0 / +1) = the -2 / +2 neighbour; then for
// every pair a < b the four diagonal neighbours (sa, sb) in {-1,+1}^2.
// Offsets are clamped per axis (replicate padding).
template <int D>
struct StencilPts {
  static constexpr int kFace = 1 + 2 * D;          // diffusion
  static constexpr int kAll = 1 + 4 * D + 2 * D * (D - 1);  // curvature
};

template <int D, int NP>
__device__ __forceinline__ void stencil_offsets(const Nbr<D>& nb, int* off) {
  off[0] = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    off[1 + 2 * a] = nb.m1[a];
    off[2 + 2 * a] = nb.p1[a];
  }
  if (NP > 1 + 2 * D) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      off[1 + 2 * D + 2 * a] = nb.m2[a];
      off[2 + 2 * D + 2 * a] = nb.p2[a];
    }
    int k = 1 + 4 * D;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = a + 1; b < D; ++b) {
        off[k++] = nb.m1[a] + nb.m1[b];
        off[k++] = nb.m1[a] + nb.p1[b];
        off[k++] = nb.p1[a] + nb.m1[b];
        off[k++] = nb.p1[a] + nb.p1[b];
      }
  }
}

// Index of the diagonal point (a, sa, b, sb) in the curvature stencil.
template <int D>
__device__ __forceinline__ constexpr int diag_index(int a, int sa, int b,
                                                    int sb) {
  // pairs (a < b) in order (0,1), (0,2), (1,2)
  int lo = a < b ? a : b, hi = a < b ? b : a;
  int slo = a < b ? sa : sb, shi = a < b ? sb : sa;
  int pair = (D == 2) ? 0 : (lo == 0 ? hi - 1 : 2);
  return 1 + 4 * D + 4 * pair + 2 * slo + shi;
}

// B^T B v at p (without the 1/h^2 or 1/h^4 factor), this voxel's share of
// ||B v||^2 and v at p: diffusion (REG 0) -> (-L v, forward-face
// differences squared); curvature (REG 1) -> (L (L v), (L v)^2).  In two
// parts, so that a caller can issue the loads of several stencils before
// the arithmetic of any: reg_load issues the stencil's loads, reg_eval does
// the float64 arithmetic on them.
template <int D, int REG>
struct RegPts {
  static constexpr int kN = REG ? StencilPts<D>::kAll : StencilPts<D>::kFace;
};
template <int D, int REG, class F>
__device__ __forceinline__ void reg_load(const F& f, const Pos<D>& p,
                                         const Nbr<D>& nb,
                                         float (&v)[RegPts<D, REG>::kN]) {
  constexpr int NP = RegPts<D, REG>::kN;
  int off[NP];
  stencil_offsets<D, NP>(nb, off);
#pragma unroll
  for (int i = 0; i < NP; ++i) v[i] = f.ld(p.idx + off[i]);
}
template <int D, int REG>
__device__ __forceinline__ void reg_eval(const float (&v)[RegPts<D, REG>::kN],
                                         const Nbr<D>& nb, double& btb,
                                         double& energy, double& centre) {
  const double c = (double)v[0];
  centre = c;
  double vm[D], vp[D], Lc = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    vm[a] = (double)v[1 + 2 * a];
    vp[a] = (double)v[2 + 2 * a];
    Lc += (vm[a] - c) + (vp[a] - c);
  }
  if (REG == 0) {
    double e = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) e += (vp[a] - c) * (vp[a] - c);
    btb = -Lc;
    energy = e;
    return;
  }
  double LL = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int sa = 0; sa < 2; ++sa) {
      bool has = sa ? nb.hp[a] : nb.hm[a];
      double vn = sa ? vp[a] : vm[a];
      double far = (double)v[1 + 2 * D + 2 * a + sa];
      double Ln = (far - vn) + (c - vn);
#pragma unroll
      for (int b = 0; b < D; ++b) {
        if (b == a) continue;
        Ln += ((double)v[diag_index<D>(a, sa, b, 0)] - vn) +
              ((double)v[diag_index<D>(a, sa, b, 1)] - vn);
      }
      LL += has ? (Ln - Lc) : 0.0;
    }
  btb = LL;
  energy = Lc * Lc;
}
// Both parts for one stencil; all its loads are issued first.
template <int D, int REG, class F>
__device__ __forceinline__ void reg_terms(const F& f, const Pos<D>& p,
                                          const Geom& g, double& btb,
                                          double& energy, double& centre) {
  const Nbr<D> nb = neighbours<D>(p, g);
  float v[RegPts<D, REG>::kN];
  reg_load<D, REG>(f, p, nb, v);
  // keep the loads together: interleaved with their uses they would wait
  // for each other one by one
  __builtin_amdgcn_sched_barrier(0);
  reg_eval<D, REG>(v, nb, btb, energy, centre);
}

// Shares of ||B u||^2, <B u, B w>, ||B w||^2 at p (quadratic expansion of S).
template <int D, int REG>
__device__ __forceinline__ void reg_cross(const float* __restrict__ uptr,
                                          const float* __restrict__ wptr,
                                          const Pos<D>& p, const Geom& g,
                                          double& uu, double& uw,
                                          double& ww) {
  const Src1 u{uptr}, w{wptr};
  const Nbr<D> nb = neighbours<D>(p, g);
  const unsigned i = p.idx;
  if (REG == 0) {
    double cu = u(i), cw = w(i);
    double a_uu = 0, a_uw = 0, a_ww = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double du = u(i + nb.p1[a]) - cu;
      double dw = w(i + nb.p1[a]) - cw;
      a_uu += du * du;
      a_uw += du * dw;
      a_ww += dw * dw;
    }
    uu = a_uu;
    uw = a_uw;
    ww = a_ww;
  } else {
    double lu = lap_c<D>(u, i, nb);
    double lw = lap_c<D>(w, i, nb);
    uu = lu * lu;
    uw = lu * lw;
    ww = lw * lw;
  }
}

// diag(B^T B) at p (unscaled).
template <int D>
__device__ __forceinline__ double reg_diag_at(const Pos<D>& p, const Geom& g,
                                              int reg) {
  int deg = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    deg += (p.c[a] > 0) + (p.c[a] < g.m[a] - 1);
  }
  double dd = (double)deg;
  return reg == 0 ? dd : dd * dd + dd;
}

// Jacobi diagonal factor of voxel p without the data term.
template <int D>
__device__ __forceinline__ double jacobi_rest(const Pos<D>& p, const Geom& g,
                                              const Model& md) {
  return md.alpha_hd * md.reg_scale * reg_diag_at<D>(p, g, md.reg) +
         md.pen_diag;
}

// Bi/trilinear sample of one frame at x + u(x) with d/du, float64.
template <int D>
__device__ __forceinline__ void warp_sample(const float* __restrict__ T,
                                            const Geom& g, const Pos<D>& p,
                                            const double* uv, double& W,
                                            double* dW) {
  int i0[D], i1[D];
  double f[D];
  bool inside[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int m = g.m[a];
    double q = (double)p.c[a] + uv[a] * g.inv_h;
    inside[a] = (q >= 0.0) && (q <= (double)(m - 1));
    double qc = fmin(fmax(q, 0.0), (double)(m - 1));
    // m = 1: qc = 0 gives i0 = i1 = 0, f = 0
    int fl = (int)floor(qc);
    i0[a] = max(min(fl, m - 2), 0);
    i1[a] = min(i0[a] + 1, m - 1);
    f[a] = qc - (double)i0[a];
  }
  if (D == 2) {
    unsigned r0 = (unsigned)i0[0] * (unsigned)g.s[0];
    unsigned r1 = (unsigned)i1[0] * (unsigned)g.s[0];
    double t00 = T[r0 + i0[1]], t01 = T[r0 + i1[1]];
    double t10 = T[r1 + i0[1]], t11 = T[r1 + i1[1]];
    double a0 = (1.0 - f[1]) * t00 + f[1] * t01;   // row i0
    double a1 = (1.0 - f[1]) * t10 + f[1] * t11;   // row i1
    double b0 = (1.0 - f[0]) * t00 + f[0] * t10;   // column i0
    double b1 = (1.0 - f[0]) * t01 + f[0] * t11;   // column i1
    W = (1.0 - f[0]) * a0 + f[0] * a1;
    dW[0] = inside[0] ? (a1 - a0) * g.inv_h : 0.0;
    dW[1] = inside[1] ? (b1 - b0) * g.inv_h : 0.0;
  } else {
    double t[2][2][2];
#pragma unroll
    for (int z = 0; z < 2; ++z)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          unsigned o = (unsigned)(z ? i1[0] : i0[0]) * (unsigned)g.s[0] +
                       (unsigned)(y ? i1[1] : i0[1]) * (unsigned)g.s[1] +
                       (unsigned)(x ? i1[2] : i0[2]);
          t[z][y][x] = T[o];
        }
    double w0[2] = {1.0 - f[0], f[0]};
    double w1[2] = {1.0 - f[1], f[1]};
    double w2[2] = {1.0 - f[2], f[2]};
    double val = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
    for (int z = 0; z < 2; ++z)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          double tv = t[z][y][x];
          val += w0[z] * w1[y] * w2[x] * tv;
          d0 += (z ? 1.0 : -1.0) * w1[y] * w2[x] * tv;
          d1 += (y ? 1.0 : -1.0) * w0[z] * w2[x] * tv;
          d2 += (x ? 1.0 : -1.0) * w0[z] * w1[y] * tv;
        }
    W = val;
    dW[0] = inside[0] ? d0 * g.inv_h : 0.0;
    dW[1] = inside[1] ? d1 * g.inv_h : 0.0;
    dW[2] = inside[2] ? d2 * g.inv_h : 0.0;
  }
}

// Value only (trial evaluations).
template <int D>
__device__ __forceinline__ double warp_value(const float* __restrict__ T,
                                             const Geom& g, const Pos<D>& p,
                                             const double* uv) {
  double W, dW[D];
  warp_sample<D>(T, g, p, uv, W, dW);
  return W;
}

// Index of this thread's wave in the block, as a wave-uniform value (the
// compiler cannot prove threadIdx.x / 64 uniform; readfirstlane lets loop
// bounds and plane pointers that depend on it live in scalar registers).
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

// Wave-level reductions by DPP lane moves (register-only, a few cycles
// each; a shuffle goes through the LDS crossbar): inclusive scan within
// 16-lane rows (shifts by 1, 2, 4, 8), then row 0's total into row 1 and
// rows 0-1's into rows 2-3 (row broadcasts of lanes 15 and 31), so lane 63
// ends with the total, which every lane reads back.  Lanes a move cannot
// reach contribute the identity.  The order of the float64 operations is
// fixed, so results are deterministic.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v, double identity) {
  const long long b = __double_as_longlong(v);
  const long long id = __double_as_longlong(identity);
  const int lo = __builtin_amdgcn_update_dpp((int)id, (int)b, CTRL, ROW_MASK,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(id >> 32), (int)(b >> 32),
                                             CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) |
                              (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_lane63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) |
                              (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0x111, 0xf>(v, 0.0);     // row_shr:1
  v += dpp_f64<0x112, 0xf>(v, 0.0);     // row_shr:2
  v += dpp_f64<0x114, 0xf>(v, 0.0);     // row_shr:4
  v += dpp_f64<0x118, 0xf>(v, 0.0);     // row_shr:8
  v += dpp_f64<0x142, 0xa>(v, 0.0);     // row_bcast:15 into rows 1, 3
  v += dpp_f64<0x143, 0xc>(v, 0.0);     // row_bcast:31 into rows 2, 3
  return wave_lane63(v);
}

__device__ __forceinline__ double wave_max(double v) {
  const double ninf = -__builtin_inf();
  v = fmax(v, dpp_f64<0x111, 0xf>(v, ninf));
  v = fmax(v, dpp_f64<0x112, 0xf>(v, ninf));
  v = fmax(v, dpp_f64<0x114, 0xf>(v, ninf));
  v = fmax(v, dpp_f64<0x118, 0xf>(v, ninf));
  v = fmax(v, dpp_f64<0x142, 0xa>(v, ninf));
  v = fmax(v, dpp_f64<0x143, 0xc>(v, ninf));
  return wave_lane63(v);
}

// A block's index and the block count within its own problem: the grid of
// a single-problem launch, or one problem's share of a batched launch
// (whose shares start at multiples of kXCD, so b % kXCD is still the XCD).
struct Blk {
  int id, n;
};
__device__ __forceinline__ Blk grid_blk() {
  return Blk{(int)blockIdx.x, (int)gridDim.x};
}

// Tile index of the i-th tile a block processes.  Blocks are dealt to the 8
// XCDs round-robin by the hardware; this gives every XCD one contiguous
// range of tiles so that stencil neighbours share that XCD's L2.
__device__ __forceinline__ long long xcd_tile(long long ntiles, int i,
                                              Blk blk) {
  int b = blk.id;
  int nb = blk.n;                // a multiple of kXCD
  int xcd = b % kXCD;
  int local = b / kXCD;
  int per_xcd_blocks = nb / kXCD;
  long long lo = ntiles * xcd / kXCD;
  long long hi = ntiles * (xcd + 1) / kXCD;
  long long t = lo + local + (long long)i * per_xcd_blocks;
  return t < hi ? t : -1;
}
__device__ __forceinline__ long long xcd_tile(long long ntiles, int i) {
  return xcd_tile(ntiles, i, grid_blk());
}

// Tile order of the volume sweeps whose regulariser stencils reach the
// neighbouring z-lines (evaluation and trial steps).  A tile is 64 voxels
// of one z-line when the z-extent is a multiple of 64; in index order the
// lines at x +- 1 and x +- 2 come m1 and 2 m1 tiles later and have left the
// L2 by then.  Ordered instead in bands of kLineBand y-lines (x slower
// within a band), they come kLineBand and 2 kLineBand tiles later, in the
// same round of a die's blocks; with m1 = 8 kLineBand every die's range of
// tiles (xcd_tile) is one band.  t: position in the order; returns the
// index of the tile.  Other shapes keep index order.
constexpr unsigned kLineBand = 16;
template <int D>
__device__ __forceinline__ long long stencil_tile(const Geom& g, long long t) {
  if (D != 3 || g.m[2] % kWave != 0) return t;
  const unsigned nz = (unsigned)g.m[2] / kWave;
  const unsigned m0 = (unsigned)g.m[0], m1 = (unsigned)g.m[1];
  const unsigned tt = (unsigned)t;
  const unsigned band = kLineBand * m0 * nz;  // tiles of a full band
  const unsigned b = tt / band;
  const unsigned r = tt - b * band;
  const unsigned y0 = b * kLineBand;
  const unsigned bw = (m1 - y0 < kLineBand ? m1 - y0 : kLineBand) * nz;
  const unsigned i0 = r / bw;  // x of the line
  // the rest, r - i0 bw, is (y - y0) nz + the tile within the line
  return ((long long)i0 * m1 + y0) * nz + (r - i0 * bw);
}

}  // namespace stml
