// Conjugate-gradient kernels of the Gauss-Newton step (images and volumes).
//
// The Gauss-Newton Hessian couples the frames of a voxel only through two
// per-voxel sums, S = sum_k dW_k . v_k and V = sum_k v_k.  The CG direction
// is p = z + beta p_old, so S and V of p follow from those of z (summed
// by the kernel that writes z) and of p_old (kept from the previous
// product): S_p = S_z + beta S_pold.  The Hessian product therefore needs
// no sweep over frames and runs as a plain stencil kernel, parallel over
// (frame, spatial tile): in 2-D each block stages p = z + beta p_old of a
// 64 x 4 tile with a 2-cell halo in LDS, forms L p once per point and
// L (L p) from LDS; in 3-D a block marches a 32 x 16 column through the
// planes with rings of planes in LDS.  The vector updates are voxel-major
// (the waves of a block split the frames of a 64-voxel tile) so that they
// can sum S_z and V_z per voxel; the Jacobi diagonal is recomputed there
// from dW/du instead of being stored.
#include <hip/hip_ext.h>
#include <math.h>

#include "launch.h"
#include "reduce.h"

namespace stml {

constexpr int kTX = 64;            // tile width (x, fastest axis)
constexpr int kTY = 4;             // tile height (y)
constexpr int kHX = kTX + 4;       // with a 2-cell halo
constexpr int kHY = kTY + 4;
constexpr int kLX = kTX + 2;       // L p on a 1-cell halo
constexpr int kLY = kTY + 2;
// 3-D columns: 16 (x) x 16 (y) points marched through 16 planes in z
constexpr int kT3X = kHv3X, kT3Y = kHv3Y, kT3Z = kHv3Z;
// threads of a Hessian-product block: one per tile point
constexpr int kHv2Threads = kTX * kTY;
constexpr int kHv3Threads = kT3X * kT3Y;

// Frames of a voxel-major tile handled by this wave.
__device__ __forceinline__ void wave_frames(int nK, int& j0, int& j1) {
  int G = blockDim.x / kWave;
  int w = wave_id();
  int per = (nK + G - 1) / G;
  j0 = w * per;
  j1 = j0 + per < nK ? j0 + per : nK;
}

// Combine the per-wave sums of S (1) and V (D) of every voxel of the tile
// and store them (float64).
template <int D>
__device__ __forceinline__ void store_voxel_sums(double s, const double* v,
                                                 long long x, bool valid,
                                                 long long N,
                                                 double* __restrict__ S,
                                                 float* __restrict__ V) {
  __shared__ double xs[kMaxChunks][kWave][1 + D];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = wave_id();
  const int G = blockDim.x / kWave;
  xs[w][lane][0] = s;
#pragma unroll
  for (int a = 0; a < D; ++a) xs[w][lane][1 + a] = v[a];
  __syncthreads();
  // wave k sums value k (S, then the D components of V) over the waves
  if (w <= D && valid) {
    double t = 0.0;
    for (int c = 0; c < G; ++c) t += xs[c][lane][w];
    if (w == 0) S[x] = t;
    else V[(size_t)(w - 1) * N + x] = t;
  }
  __syncthreads();
}

// x = 0 over this block's tiles: the CG solution when no step is taken
// (r.z = 0 at the start, or p.q <= 0 at the first step), as CG from x0 = 0
// leaves it; without this the Gauss-Newton step would read whatever x held.
template <int D>
__device__ __forceinline__ void cg_zero_x(float* __restrict__ x,
                                          const Geom& g, const Model& md,
                                          Blk blk) {
  int j0, j1;
  wave_frames(md.nK, j0, j1);
  const int lane = threadIdx.x & (kWave - 1);
  const long long N = g.N;
  const long long ntiles = (N + kWave - 1) / kWave;
  for (int tt = 0;; ++tt) {
    long long tile = xcd_tile(ntiles, tt, blk);
    if (tile < 0) break;
    long long xv = tile * kWave + lane;
    if (xv >= N) continue;
    for (int j = j0; j < j1; ++j)
#pragma unroll
      for (int a = 0; a < D; ++a)
        x[((size_t)j * D + a) * N + (size_t)xv] = 0.f;
  }
}

// x = (zero ? 0 : x) + a p over this block's tiles (voxel-major, every
// frame): the pending term of a CG that stopped after an even step.
template <int D>
__device__ __forceinline__ void cg_fold_x(float* __restrict__ x,
                                          const float* __restrict__ p,
                                          double a, bool zero, const Geom& g,
                                          const Model& md, Blk blk) {
  int j0, j1;
  wave_frames(md.nK, j0, j1);
  const int lane = threadIdx.x & (kWave - 1);
  const long long N = g.N;
  const long long ntiles = (N + kWave - 1) / kWave;
  for (int tt = 0;; ++tt) {
    long long tile = xcd_tile(ntiles, tt, blk);
    if (tile < 0) break;
    long long xv = tile * kWave + lane;
    if (xv >= N) continue;
    for (int j = j0; j < j1; ++j)
#pragma unroll
      for (int a2 = 0; a2 < D; ++a2) {
        const size_t o = ((size_t)j * D + a2) * N + (size_t)xv;
        x[o] = (float)((zero ? 0.0 : (double)x[o]) + a * (double)p[o]);
      }
  }
}

// CG step, part 2: a = rz / p.q (stop on p.q <= 0); r -= a q, z = M^-1 r;
// per-voxel S_z, V_z; partials r.z, r.r; x by XM (cg_x_mode): nothing at an
// even step other than the last, x += a' p' + a p at an odd one (p' and a'
// of the previous step: the other buffer of the direction pair and the step
// length history), x += a p at a last even step.  A frame's loads (both
// components) issue before its stores, which would otherwise hold the next
// component's loads back.  At it = 0 a CG that stops before its first step
// sets x = 0; a breakdown at an odd step adds the previous step's term.
// FIRST with ev_part: the step also forms the start scalars of the
// Gauss-Newton iteration from the evaluation's five partials (J = D + S +
// P, r.z, r.r; the log's J) and takes their decisions: r.z = 0 ends the CG
// with x = 0, and a start at or below the objective target takes no step.
template <int D, bool FIRST, bool PRE, int XM>
__device__ __forceinline__ void cgv_update_body(
    int it, const float* __restrict__ p, const float* __restrict__ p_prev,
    const float* __restrict__ q, const float* __restrict__ dW, const Geom& g,
    const Model& md, float* __restrict__ x, float* __restrict__ r,
    float* __restrict__ z, double* __restrict__ Sz, float* __restrict__ Vz,
    const double* __restrict__ hv_part, int hv_nb, double* __restrict__ part,
    Scal* __restrict__ sc, int gn_it, const double* __restrict__ ev_part,
    int ev_nb, GNLog* __restrict__ log, int brk, Blk blk) {
  static_assert(!FIRST || XM == kXNone || XM == kXOne, "x mode");
  constexpr bool kP = XM != kXNone;                    // reads p
  constexpr bool kPP = XM == kXTwo || XM == kXTwoFirst; // reads p'
  constexpr bool kXR = (XM == kXOne && !FIRST) || XM == kXTwo;  // reads x
  const int stop = sc->gn_stop;
  int done = sc->done;
  double rz_it = sc->rzh[it & 1];
  const double a_prev = (!FIRST && (it & 1)) ? sc->ah[(it - 1) & 1] : 0.0;
  int j0, j1;
  wave_frames(md.nK, j0, j1);
  const int lane = threadIdx.x & (kWave - 1);
  const long long N = g.N;
  const long long ntiles = (N + kWave - 1) / kWave;
  // one frame's loads and its update (x, r, z stored, sums accumulated)
  struct Fr {
    float p[D], pp[D], d[D], x[D], r[D], q[D];
  };
  auto load = [&](size_t base, Fr& f) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const size_t o = base + (size_t)a * N;
      f.p[a] = kP ? p[o] : 0.f;
      f.pp[a] = kPP ? p_prev[o] : 0.f;
      f.d[a] = dW[o];
      f.x[a] = kXR ? x[o] : 0.f;
      f.r[a] = r[o];
      f.q[a] = q[o];
    }
  };
  // PRE (grids of at most one block per compute unit, latency-bound): the
  // first frame of the first tile is requested together with the control
  // scalars and the product's partials (four frames ahead measured slower:
  // the registers they hold cost more than the round trips they save)
  const long long tile0 = xcd_tile(ntiles, 0, blk);
  const long long xv0 = tile0 * kWave + lane;
  const bool pre = PRE && tile0 >= 0 && xv0 < N;
  Fr f0;
  if (pre && j0 < j1) load((size_t)j0 * D * N + (size_t)xv0, f0);
  if (gn_it >= stop) return;
  if (FIRST && ev_part) {
    // (the flags other blocks read at their start, done and gn_stop, are
    // only written in ways that leave such a block's work unchanged)
    double e[5];
    reduce_partials<5>(ev_part, ev_nb, 0u, e);
    const double Dv = md.hd * e[0];
    const double Sv = md.half_alpha_hd * md.reg_scale * e[1];
    const double Pv = md.lam_hd * e[2];
    const double Jv = Dv + Sv + Pv;
    rz_it = e[3];
    done = e[3] == 0.0 ? 1 : 0;
    const bool no_step = gn_it == 0 && Jv <= sc->J_target;
    if (blk.id == 0 && threadIdx.x == 0) {
      sc->D = Dv;
      sc->S = Sv;
      sc->P = Pv;
      sc->J = Jv;
      sc->rzh[0] = e[3];
      sc->r0 = sqrt(e[4]);
      sc->rr = e[4];
      sc->iters = 0;
      sc->done = done;
      if (log) log[gn_it].J = Jv;
      if (no_step) sc->gn_stop = 0;
    }
    if (no_step) return;
  }
  if (done) {
    if (FIRST) cg_zero_x<D>(x, g, md, blk);
    return;
  }
  double t[1];
  reduce_partials<1>(hv_part, hv_nb, 0u, t);
  const double pq = t[0];
  // (brk: this step breaks down as if p.Hp <= 0, a host-forced test of the
  // branch; -1 otherwise)
  if (!(pq > 0.0) || it == brk) {
    if (blk.id == 0 && threadIdx.x == 0) {
      sc->pq = pq;
      sc->done = 2;
    }
    if (FIRST) cg_zero_x<D>(x, g, md, blk);
    // the previous (even) step left its term to this one
    else if (it & 1) cg_fold_x<D>(x, p_prev, a_prev, it == 1, g, md, blk);
    return;
  }
  const double alpha = rz_it / pq;
  if (blk.id == 0 && threadIdx.x == 0) {
    sc->pq = pq;
    sc->a = alpha;
    sc->ah[it & 1] = alpha;
    sc->iters = it + 1;
  }
  double rz = 0.0, rr = 0.0;
  for (int tt = 0;; ++tt) {
    long long tile = xcd_tile(ntiles, tt, blk);
    if (tile < 0) break;
    long long xv = tile * kWave + lane;
    bool valid = xv < N;
    Pos<D> pos = make_pos<D>(g, valid ? xv : N - 1);
    const double rest = jacobi_rest<D>(pos, g, md);
    double s = 0.0, v[D];
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = 0.0;
    auto frame = [&](size_t base, const Fr& f) {
#pragma unroll
      for (int a = 0; a < D; ++a) {
        size_t o = base + (size_t)a * N;
        const double d = (double)f.d[a];
        if (XM == kXOne)
          x[o] = FIRST ? (float)(alpha * (double)f.p[a])
                       : (float)((double)f.x[a] + alpha * (double)f.p[a]);
        else if (XM == kXTwo)
          x[o] = (float)(((double)f.x[a] + a_prev * (double)f.pp[a]) +
                         alpha * (double)f.p[a]);
        else if (XM == kXTwoFirst)
          x[o] = (float)(a_prev * (double)f.pp[a] + alpha * (double)f.p[a]);
        float rv = (float)((double)f.r[a] - alpha * (double)f.q[a]);
        float zv = (float)((double)rv / (md.mdiag_c * d * d + rest));
        r[o] = rv;
        z[o] = zv;
        rz += (double)rv * (double)zv;
        rr += (double)rv * (double)rv;
        s += d * (double)zv;
        v[a] += (double)zv;
      }
    };
    if (valid && PRE) {
      // small grids (a wave's frames in turn are the latency): after the
      // frame requested ahead, two frames per pass, whose loads issue
      // together (an odd last frame loads its own values twice); frames
      // are accumulated in order, as one at a time
      int j = j0;
      if (tt == 0 && j < j1) {
        frame((size_t)j * D * N + pos.idx, f0);
        ++j;
      }
#pragma unroll 1
      for (; j < j1; j += 2) {
        const int jb = j + 1 < j1 ? j + 1 : j;
        const size_t b0 = (size_t)j * D * N + pos.idx;
        const size_t b1 = (size_t)jb * D * N + pos.idx;
        Fr fa, fb;
        load(b0, fa);
        load(b1, fb);
        frame(b0, fa);
        if (jb != j) frame(b1, fb);
      }
    } else if (valid && D == 3) {
      // volumes on large grids: one component at a time, which keeps the
      // form limited to 64 registers free of spills (issuing all 15 loads
      // of a frame first spilled 52 B per lane and streamed 8% slower)
#pragma unroll 1
      for (int j = j0; j < j1; ++j) {
        const size_t base = (size_t)j * D * N + pos.idx;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const size_t o = base + (size_t)a * N;
          const float pv = kP ? p[o] : 0.f, ppv = kPP ? p_prev[o] : 0.f,
                      dv = dW[o], xv2 = kXR ? x[o] : 0.f, rv0 = r[o],
                      qv = q[o];
          const double d = (double)dv;
          if (XM == kXOne)
            x[o] = FIRST ? (float)(alpha * (double)pv)
                         : (float)((double)xv2 + alpha * (double)pv);
          else if (XM == kXTwo)
            x[o] = (float)(((double)xv2 + a_prev * (double)ppv) +
                           alpha * (double)pv);
          else if (XM == kXTwoFirst)
            x[o] = (float)(a_prev * (double)ppv + alpha * (double)pv);
          float rv = (float)((double)rv0 - alpha * (double)qv);
          float zv = (float)((double)rv / (md.mdiag_c * d * d + rest));
          r[o] = rv;
          z[o] = zv;
          rz += (double)rv * (double)zv;
          rr += (double)rv * (double)rv;
          s += d * (double)zv;
          v[a] += (double)zv;
        }
      }
    } else if (valid) {
#pragma unroll 1
      for (int j = j0; j < j1; ++j) {
        const size_t base = (size_t)j * D * N + pos.idx;
        Fr f;
        load(base, f);
        frame(base, f);
      }
    }
    store_voxel_sums<D>(s, v, xv, valid, N, Sz, Vz);
  }
  double vals[2] = {rz, rr};
  block_partials<2>(vals, 0u, part, blk);
}

// OCC: two blocks per compute unit (at most 64 registers per lane), so that
// while one block combines its per-voxel sums the other streams; for grids
// with more blocks than compute units.  Small grids (latency-bound levels)
// run faster with the registers unconstrained.  Same arithmetic either way.
template <int D, bool OCC, bool FIRST, int XM>
__global__ __launch_bounds__(1024, OCC ? 8 : 1) void cgv_update_kernel(
    int it, const float* __restrict__ p, const float* __restrict__ p_prev,
    const float* __restrict__ q, const float* __restrict__ dW, Geom g,
    Model md, float* __restrict__ x, float* __restrict__ r,
    float* __restrict__ z, double* __restrict__ Sz, float* __restrict__ Vz,
    const double* __restrict__ hv_part, int hv_nb, double* __restrict__ part,
    Scal* __restrict__ sc, int gn_it, const double* __restrict__ ev_part,
    int ev_nb, GNLog* __restrict__ log, int brk) {
  cgv_update_body<D, FIRST, !OCC, XM>(it, p, p_prev, q, dW, g, md, x, r, z,
                                      Sz, Vz, hv_part, hv_nb, part, sc, gn_it,
                                      ev_part, ev_nb, log, brk, grid_blk());
}

// Per-voxel S and V of a stored field v (Hessian product test entry).
template <int D>
__global__ __launch_bounds__(1024) void cgv_sums_kernel(
    const float* __restrict__ v, const float* __restrict__ dW, Geom g,
    Model md, double* __restrict__ S, float* __restrict__ V) {
  int j0, j1;
  wave_frames(md.nK, j0, j1);
  const int lane = threadIdx.x & (kWave - 1);
  const long long N = g.N;
  const long long ntiles = (N + kWave - 1) / kWave;
  for (int it = 0;; ++it) {
    long long tile = xcd_tile(ntiles, it);
    if (tile < 0) break;
    long long x = tile * kWave + lane;
    bool valid = x < N;
    double s = 0.0, vs[D];
#pragma unroll
    for (int a = 0; a < D; ++a) vs[a] = 0.0;
    if (valid) {
      for (int j = j0; j < j1; ++j) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          size_t o = ((size_t)j * D + a) * N + x;
          double vv = (double)v[o];
          s += (double)dW[o] * vv;
          vs[a] += vv;
        }
      }
    }
    store_voxel_sums<D>(s, vs, x, valid, N, S, V);
  }
}

// Hessian product on p = z + beta p_old (it > 0) or p = z (it = 0: FIRST,
// a form of its own, so that no load waits behind a branch on it) for one
// 64 x 4 tile of a group of frames; stores p and q = H p, partial p.q.
// For it > 0 it first finishes the previous update: beta and the
// convergence test from the update's partials.
template <int REG, bool FIRST>
__device__ __forceinline__ void cgt_hvp2_body(
    int it, const float* __restrict__ zv, const float* __restrict__ p_old,
    float* __restrict__ p_new, const float* __restrict__ dW, const Geom& g,
    const Model& md, float* __restrict__ q, float* __restrict__ x,
    const double* __restrict__ Sz,
    const float* __restrict__ Vz, const double* __restrict__ Sp_old,
    const float* __restrict__ Vp_old, double* __restrict__ Sp_new,
    float* __restrict__ Vp_new, int nreal, int nfg, int fpg,
    const double* __restrict__ up_part, int up_nb, int fixed, double rtol,
    double* __restrict__ part, Scal* __restrict__ sc, int gn_it, Blk blk) {
  constexpr int D = 2;
  __shared__ double P[D][kHY][kHX];
  __shared__ double L[REG ? D : 1][REG ? kLY : 1][REG ? kLX : 1];
  // Everything this block reads is requested before it waits for the
  // control scalars and the update's partials: the per-voxel sums and the
  // first frame's halo tile are in flight meanwhile (on the coarse levels
  // these round trips are most of a launch's time).
  const int done = sc->done, stop = sc->gn_stop;
  const double rz_old = FIRST ? 0.0 : sc->rzh[(it - 1) & 1];
  const double r0 = sc->r0;
  // block -> (tile, frame group), XCD-chunked
  const int per_xcd = blk.n / kXCD;
  const int bb = (blk.id % kXCD) * per_xcd + blk.id / kXCD;
  const int m0 = g.m[0], m1 = g.m[1];
  const long long N = g.N;
  const bool has = bb < nreal;
  const int tile = has ? bb / nfg : 0, fg = has ? bb - (bb / nfg) * nfg : 0;
  const int ntx = (m1 + kTX - 1) / kTX;
  const int y0 = (tile / ntx) * kTY, x0 = (tile % ntx) * kTX;
  const int ty = threadIdx.x / kTX, tx = threadIdx.x % kTX;
  const int y = y0 + ty, xx = x0 + tx;
  const bool valid = has && y < m0 && xx < m1;
  const unsigned vox = valid ? (unsigned)(y * m1 + xx) : 0u;
  const int jbeg = fg * fpg;
  const int jend = !has ? jbeg : (jbeg + fpg < md.nK ? jbeg + fpg : md.nK);
  double S = 0.0, V0 = 0.0, V1 = 0.0, So = 0.0, Vo0 = 0.0, Vo1 = 0.0;
  if (valid) {
    S = Sz[vox];
    V0 = Vz[vox];
    V1 = Vz[N + vox];
    if (!FIRST) {
      So = Sp_old[vox];
      Vo0 = Vp_old[vox];
      Vo1 = Vp_old[N + vox];
    }
  }
  // p of the halo tile, staged through registers one frame ahead: the
  // loads of frame j + 1 are in flight while frame j is computed
  // (replicate padding at the grid edge = clamped loads)
  constexpr int kSt = (kHY * kHX + kTX * kTY - 1) / (kTX * kTY);
  unsigned so[kSt];
#pragma unroll
  for (int s = 0; s < kSt; ++s) {
    const int i = threadIdx.x + s * kTX * kTY;
    const int hy = i / kHX, hx = i - (i / kHX) * kHX;
    const int gy = min(max(y0 - 2 + hy, 0), m0 - 1);
    const int gx = min(max(x0 - 2 + hx, 0), m1 - 1);
    so[s] = (unsigned)(gy * m1 + gx);
  }
  float sz[kSt][D], sp[kSt][D];
  auto fetch = [&](int j) {
#pragma unroll
    for (int s = 0; s < kSt; ++s) {
      if (threadIdx.x + s * kTX * kTY < kHY * kHX) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const size_t plane = ((size_t)j * D + a) * N;
          sz[s][a] = zv[plane + so[s]];
          sp[s][a] = !FIRST ? p_old[plane + so[s]] : 0.f;
        }
      }
    }
  };
  if (jbeg < jend) fetch(jbeg);
  // at CG step 0 the done flag is the previous iteration's (the update of
  // this step forms the new one)
  if ((!FIRST && done) || gn_it >= stop) return;
  double beta = 0.0;
  if (!FIRST) {
    double t[2];
    reduce_partials<2>(up_part, up_nb, 0u, t);
    bool conv = (!fixed && sqrt(t[1]) <= rtol * r0) || t[0] == 0.0;
    if (conv) {
      if (blk.id == 0 && threadIdx.x == 0) sc->done = 1;
      // converged after an even step: its term of x is still pending
      if ((it & 1) && valid) {
        const double a_prev = sc->ah[(it - 1) & 1];
        for (int j = jbeg; j < jend; ++j)
#pragma unroll
          for (int a = 0; a < D; ++a) {
            const size_t o = ((size_t)j * D + a) * N + vox;
            x[o] = (float)((it == 1 ? 0.0 : (double)x[o]) +
                           a_prev * (double)p_old[o]);
          }
      }
      return;
    }
    beta = t[0] / rz_old;
    if (blk.id == 0 && threadIdx.x == 0) {
      sc->rzh[it & 1] = t[0];
      sc->rr = t[1];
      sc->beta = beta;
    }
  }
  const float bf = (float)beta;
  double acc = 0.0;
  if (has) {
    double sbar = 0.0, vbar[D] = {0.0, 0.0};
    if (valid) {
      if (!FIRST) {
        S += beta * So;
        V0 += beta * Vo0;
        V1 += beta * Vo1;
      }
      if (fg == 0) {
        Sp_new[vox] = S;
        Vp_new[vox] = V0;
        Vp_new[N + vox] = V1;
      }
      sbar = S * md.inv_nK;
      vbar[0] = V0 * md.inv_nK;
      vbar[1] = V1 * md.inv_nK;
    }
    for (int j = jbeg; j < jend; ++j) {
#pragma unroll
      for (int s = 0; s < kSt; ++s) {
        const int i = threadIdx.x + s * kTX * kTY;
        if (i < kHY * kHX) {
          const int hy = i / kHX, hx = i - (i / kHX) * kHX;
#pragma unroll
          for (int a = 0; a < D; ++a)
            P[a][hy][hx] = (double)(!FIRST ? __builtin_fmaf(bf, sp[s][a],
                                                            sz[s][a])
                                           : sz[s][a]);
        }
      }
      __syncthreads();
      if (j + 1 < jend) fetch(j + 1);
      if (REG) {
        // L p on the 1-cell halo; outside the grid it replicates the edge
        for (int i = threadIdx.x; i < kLY * kLX; i += blockDim.x) {
          int ly = i / kLX, lx = i - (i / kLX) * kLX;
          int gy = min(max(y0 - 1 + ly, 0), m0 - 1);
          int gx = min(max(x0 - 1 + lx, 0), m1 - 1);
          int cy = gy - y0 + 2, cx = gx - x0 + 2;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            double c = P[a][cy][cx];
            L[a][ly][lx] = (P[a][cy - 1][cx] - c) + (P[a][cy + 1][cx] - c) +
                           (P[a][cy][cx - 1] - c) + (P[a][cy][cx + 1] - c);
          }
        }
        __syncthreads();
      }
      if (valid) {
        const int py = ty + 2, px = tx + 2;
        double pc[D], d[D], s = 0.0;
        const size_t jb = (size_t)j * D * N + vox;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          pc[a] = P[a][py][px];
          d[a] = (double)dW[jb + (size_t)a * N];
          s += d[a] * pc[a];
        }
        const double ds = md.data_c * (s - sbar);
        // neighbours that leave the grid replicate this voxel: zero terms
        const bool hn = y > 0, hs = y < m0 - 1, hw = xx > 0, he = xx < m1 - 1;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double btb;
          if (REG) {
            const int ly = ty + 1, lx = tx + 1;
            double c = L[a][ly][lx];
            btb = (hn ? L[a][ly - 1][lx] - c : 0.0) +
                  (hs ? L[a][ly + 1][lx] - c : 0.0) +
                  (hw ? L[a][ly][lx - 1] - c : 0.0) +
                  (he ? L[a][ly][lx + 1] - c : 0.0);
          } else {
            double c = pc[a];
            btb = -((P[a][py - 1][px] - c) + (P[a][py + 1][px] - c) +
                    (P[a][py][px - 1] - c) + (P[a][py][px + 1] - c));
          }
          double h = ds * d[a] + md.alpha_hd * md.reg_scale * btb +
                     md.lam_c * vbar[a];
          float hf = (float)h;
          q[jb + (size_t)a * N] = hf;
          p_new[jb + (size_t)a * N] = (float)pc[a];
          acc += pc[a] * (double)hf;
        }
      }
      __syncthreads();
    }
  }
  double vals[1] = {acc};
  block_partials<1>(vals, 0u, part, blk);
}

// Seven blocks per compute unit (at most 72 registers per lane) keep enough
// tile loads in flight without the spill that eight (64 registers) cost
// (the diffusion form needs more registers: five).
template <int REG, bool FIRST>
__global__ __launch_bounds__(kHv2Threads, REG ? 7 : 5) void cgt_hvp2_kernel(
    int it, const float* __restrict__ zv, const float* __restrict__ p_old,
    float* __restrict__ p_new, const float* __restrict__ dW, Geom g,
    Model md, float* __restrict__ q, float* __restrict__ x,
    const double* __restrict__ Sz,
    const float* __restrict__ Vz, const double* __restrict__ Sp_old,
    const float* __restrict__ Vp_old, double* __restrict__ Sp_new,
    float* __restrict__ Vp_new, int nreal, int nfg, int fpg,
    const double* __restrict__ up_part, int up_nb, int fixed, double rtol,
    double* __restrict__ part, Scal* __restrict__ sc, int gn_it) {
  cgt_hvp2_body<REG, FIRST>(it, zv, p_old, p_new, dW, g, md, q, x, Sz, Vz,
                            Sp_old, Vp_old, Sp_new, Vp_new, nreal, nfg, fpg,
                            up_part, up_nb, fixed, rtol, part, sc, gn_it,
                            grid_blk());
}

// CG step, part 0 for volumes (it > 0): beta = r.z / r.z_old from the
// update's partials (stop on convergence), and the voxel sums of the new
// direction, S_p = S_z + beta S_pold and V_p = V_z + beta V_pold, formed once
// per voxel.  The 3-D Hessian product reads the per-voxel sums once per frame
// (they do not stay in the L2 across a column's frames), so it reads these
// four values instead of eight.
__device__ __forceinline__ void cg_psums_body(
    int it, const double* __restrict__ Sz, const float* __restrict__ Vz,
    const double* __restrict__ Sp_old, const float* __restrict__ Vp_old,
    double* __restrict__ Sp_new, float* __restrict__ Vp_new, long long N,
    const double* __restrict__ up_part, int up_nb, int fixed, double rtol,
    Scal* __restrict__ sc, int gn_it, Blk blk) {
  constexpr int D = 3;
  if (sc->done || gn_it >= sc->gn_stop) return;
  double t[2];
  reduce_partials<2>(up_part, up_nb, 0u, t);
  const double rz_old = sc->rzh[(it - 1) & 1];
  bool conv = (!fixed && sqrt(t[1]) <= rtol * sc->r0) || t[0] == 0.0;
  if (conv) {
    if (blk.id == 0 && threadIdx.x == 0) sc->done = 1;
    return;
  }
  const double beta = t[0] / rz_old;
  if (blk.id == 0 && threadIdx.x == 0) {
    sc->rzh[it & 1] = t[0];
    sc->rr = t[1];
    sc->beta = beta;
  }
  const long long stride = (long long)blk.n * blockDim.x;
  for (long long v = (long long)blk.id * blockDim.x + threadIdx.x; v < N;
       v += stride) {
    Sp_new[v] = Sz[v] + beta * Sp_old[v];
#pragma unroll
    for (int a = 0; a < D; ++a)
      Vp_new[a * N + v] = Vz[a * N + v] + beta * Vp_old[a * N + v];
  }
}

__global__ __launch_bounds__(1024) void cg_psums_kernel(
    int it, const double* __restrict__ Sz, const float* __restrict__ Vz,
    const double* __restrict__ Sp_old, const float* __restrict__ Vp_old,
    double* __restrict__ Sp_new, float* __restrict__ Vp_new, long long N,
    const double* __restrict__ up_part, int up_nb, int fixed, double rtol,
    Scal* __restrict__ sc, int gn_it) {
  cg_psums_body(it, Sz, Vz, Sp_old, Vp_old, Sp_new, Vp_new, N, up_part, up_nb,
                fixed, rtol, sc, gn_it, grid_blk());
}

// 3-D Hessian product on p = z + beta p_old (it > 0) or p = z for one
// column of a group of frames: a 32 x 16 tile in (x, y) marched through
// kT3Z planes in z.  For each frame the block keeps a ring of five planes of
// p (2-cell halo, float32: exactly the values the kernel stores) and three
// planes of L p (1-cell halo; formed in float64 and kept as float32, which
// lets two 512-thread blocks share a compute unit) in LDS; every step stages
// one new plane of p (its loads issued one step ahead, into registers), forms one
// plane of L p and finishes one plane of q = H p.  The halo overhead per
// step is that of a 2-D tile (36 x 20 loads for 32 x 16 outputs) instead of
// a 3-D one.  The voxel sums of p are read per frame: at CG step 0 those of
// z (which the product keeps for the next step), later the ones
// cg_psums_kernel formed together with beta.
template <int REG, bool FIRST>
__device__ __forceinline__ void cgt_hvp3_body(
    int it, const float* __restrict__ zv, const float* __restrict__ p_old,
    float* __restrict__ p_new, const float* __restrict__ dW, const Geom& g,
    const Model& md, float* __restrict__ q, float* __restrict__ x,
    const double* __restrict__ Sz,
    const float* __restrict__ Vz, const double* __restrict__ Sp_old,
    const float* __restrict__ Vp_old, double* __restrict__ Sp_new,
    float* __restrict__ Vp_new, int nreal, int nfg, int fpg,
    const double* __restrict__ up_part, int up_nb, int fixed, double rtol,
    double* __restrict__ part, Scal* __restrict__ sc, int gn_it, Blk blk) {
  constexpr int D = 3;
  constexpr int HX = kT3X + 4, HY = kT3Y + 4;   // p plane with halo
  constexpr int LX = kT3X + 2, LY = kT3Y + 2;   // L p plane with halo
  constexpr int NT = kT3X * kT3Y;               // threads = tile points
  constexpr int kPS = (HX * HY + NT - 1) / NT;  // p points per thread
  constexpr int kLS = (LX * LY + NT - 1) / NT;  // L points per thread
  __shared__ float P[D][5][HY][HX];
  __shared__ float L[REG ? D : 1][REG ? 3 : 1][REG ? LY : 1][REG ? LX : 1];
  (void)up_part;
  (void)up_nb;
  (void)fixed;
  (void)rtol;
  (void)Sp_old;
  (void)Vp_old;
  // at CG step 0 the done flag is the previous iteration's (the update of
  // this step forms the new one)
  if (gn_it >= sc->gn_stop) return;
  const int per_xcd = blk.n / kXCD;
  const int bb = (blk.id % kXCD) * per_xcd + blk.id / kXCD;
  if (!FIRST && sc->done) {
    // converged at this step (the sums kernel found it) after an even step:
    // that step's term of x is still pending
    if ((it & 1) && sc->iters == it && bb < nreal) {
      const double a_prev = sc->ah[(it - 1) & 1];
      const int m0 = g.m[0], m1 = g.m[1], m2 = g.m[2];
      const long long N = g.N;
      const long long plane_n = (long long)m1 * m2;
      const int tile = bb / nfg, fg = bb - (bb / nfg) * nfg;
      const int ntx = (m2 + kT3X - 1) / kT3X, nty = (m1 + kT3Y - 1) / kT3Y;
      const int xx = (tile % ntx) * kT3X + (int)threadIdx.x % kT3X;
      const int yy = ((tile / ntx) % nty) * kT3Y + (int)threadIdx.x / kT3X;
      const int z0 = (tile / ntx / nty) * kT3Z;
      const int z1 = z0 + kT3Z < m0 ? z0 + kT3Z : m0;
      const int jbeg = fg * fpg;
      const int jend = jbeg + fpg < md.nK ? jbeg + fpg : md.nK;
      if (xx < m2 && yy < m1)
        for (int j = jbeg; j < jend; ++j)
          for (int zz = z0; zz < z1; ++zz)
#pragma unroll
            for (int a = 0; a < D; ++a) {
              const size_t o = ((size_t)j * D + a) * N +
                               (size_t)zz * plane_n + (size_t)(yy * m2 + xx);
              x[o] = (float)((it == 1 ? 0.0 : (double)x[o]) +
                             a_prev * (double)p_old[o]);
            }
    }
    return;
  }
  // it > 0: beta and the sums of p come from cg_psums_kernel (launched just
  // before); it = 0: p = z, whose sums this kernel keeps for the next step
  const double beta = FIRST ? 0.0 : sc->beta;
  const double* Sc = FIRST ? Sz : Sp_new;
  const float* Vc = FIRST ? Vz : Vp_new;
  const float bf = (float)beta;
  double acc = 0.0;
  if (bb < nreal) {
    const int m0 = g.m[0], m1 = g.m[1], m2 = g.m[2];
    const long long N = g.N;
    const long long plane_n = (long long)m1 * m2;
    const int tile = bb / nfg, fg = bb - (bb / nfg) * nfg;
    const int ntx = (m2 + kT3X - 1) / kT3X, nty = (m1 + kT3Y - 1) / kT3Y;
    const int x0 = (tile % ntx) * kT3X;
    const int y0 = ((tile / ntx) % nty) * kT3Y;
    const int z0 = (tile / ntx / nty) * kT3Z;
    const int z1 = z0 + kT3Z < m0 ? z0 + kT3Z : m0;
    const int lx = threadIdx.x % kT3X, ly = threadIdx.x / kT3X;
    const int x = x0 + lx, y = y0 + ly;
    const bool inplane = x < m2 && y < m1;
    const unsigned vxy = inplane ? (unsigned)(y * m2 + x) : 0u;
    // in-plane offsets of this thread's halo points (clamped: replicate)
    unsigned po[kPS];
    int pi[kPS];
#pragma unroll
    for (int s = 0; s < kPS; ++s) {
      const int i = threadIdx.x + s * NT;
      pi[s] = i < HX * HY ? i : -1;
      const int hy = i / HX, hx = i - (i / HX) * HX;
      const int gy = min(max(y0 - 2 + hy, 0), m1 - 1);
      const int gx = min(max(x0 - 2 + hx, 0), m2 - 1);
      po[s] = (unsigned)(gy * m2 + gx);
    }
    const bool hn = y > 0, hs = y < m1 - 1, hw = x > 0, he = x < m2 - 1;
    const int jbeg = fg * fpg;
    const int jend = jbeg + fpg < md.nK ? jbeg + fpg : md.nK;
    float rz[kPS][D], rp[kPS][D];
    // loads of p plane pz (clamped) of frame j into registers
    auto fetch = [&](int j, int pz) {
      const int gz = min(max(pz, 0), m0 - 1);
#pragma unroll
      for (int s = 0; s < kPS; ++s) {
        if (pi[s] >= 0) {
#pragma unroll
          for (int a = 0; a < D; ++a) {
            const size_t o =
                ((size_t)j * D + a) * N + (size_t)gz * plane_n + po[s];
            rz[s][a] = zv[o];
            rp[s][a] = !FIRST ? p_old[o] : 0.f;
          }
        }
      }
    };
    auto put = [&](int pz) {
      const int slot = (pz - z0 + 2) % 5;
#pragma unroll
      for (int s = 0; s < kPS; ++s) {
        if (pi[s] >= 0) {
          const int hy = pi[s] / HX, hx = pi[s] - (pi[s] / HX) * HX;
#pragma unroll
          for (int a = 0; a < D; ++a)
            P[a][slot][hy][hx] =
                !FIRST ? __builtin_fmaf(bf, rp[s][a], rz[s][a]) : rz[s][a];
        }
      }
    };
    // L p on plane lz (1-cell halo in x, y) from the p planes lz - 1..lz + 1
    auto lplane = [&](int lz) {
      const int c = (lz - z0 + 2) % 5, dn = (lz - 1 - z0 + 2) % 5,
                up = (lz + 1 - z0 + 2) % 5, sl = (lz - z0 + 1) % 3;
#pragma unroll
      for (int s = 0; s < kLS; ++s) {
        const int i = threadIdx.x + s * NT;
        if (i < LX * LY) {
          const int qy = i / LX, qx = i - (i / LX) * LX;
          const int cy = qy + 1, cx = qx + 1;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            const double v = P[a][c][cy][cx];
            L[a][sl][qy][qx] = ((double)P[a][dn][cy][cx] - v) +
                               ((double)P[a][up][cy][cx] - v) +
                               ((double)P[a][c][cy - 1][cx] - v) +
                               ((double)P[a][c][cy + 1][cx] - v) +
                               ((double)P[a][c][cy][cx - 1] - v) +
                               ((double)P[a][c][cy][cx + 1] - v);
          }
        }
      }
    };
    for (int j = jbeg; j < jend; ++j) {
      // prologue: p planes z0 - 2 .. z0 + 1, then L planes z0 - 1, z0
      for (int pz = z0 - 2; pz <= z0 + 1; ++pz) {
        fetch(j, pz);
        put(pz);
      }
      fetch(j, z0 + 2);
      __syncthreads();
      if (REG) {
        lplane(z0 - 1);
        lplane(z0);
      }
      for (int zz = z0; zz < z1; ++zz) {
        put(zz + 2);                  // staged one step ahead
        __syncthreads();
        if (zz + 3 <= z1 + 1) fetch(j, zz + 3);
        if (REG) {
          lplane(zz + 1);
          __syncthreads();
        }
        if (inplane) {
          const unsigned vox = (unsigned)((size_t)zz * plane_n + vxy);
          double S = Sc[vox], V[D];
#pragma unroll
          for (int a = 0; a < D; ++a) V[a] = Vc[(size_t)a * N + vox];
          if (FIRST && fg == 0 && j == jbeg) {
            Sp_new[vox] = S;
#pragma unroll
            for (int a = 0; a < D; ++a) Vp_new[(size_t)a * N + vox] = V[a];
          }
          const double sbar = S * md.inv_nK;
          double vbar[D];
#pragma unroll
          for (int a = 0; a < D; ++a) vbar[a] = V[a] * md.inv_nK;
          const int c = (zz - z0 + 2) % 5, py = ly + 2, px = lx + 2;
          double pc[D], d[D], sum = 0.0;
          const size_t jb = (size_t)j * D * N + vox;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            pc[a] = P[a][c][py][px];
            d[a] = (double)dW[jb + (size_t)a * N];
            sum += d[a] * pc[a];
          }
          const double ds = md.data_c * (sum - sbar);
          // neighbours that leave the grid replicate this voxel: zero terms
          const bool hd = zz > 0, hu = zz < m0 - 1;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            double btb;
            if (REG) {
              const int sm = (zz - 1 - z0 + 1) % 3, s0 = (zz - z0 + 1) % 3,
                        sp = (zz + 1 - z0 + 1) % 3;
              const int qy = ly + 1, qx = lx + 1;
              const double cc = L[a][s0][qy][qx];
              btb = (hd ? L[a][sm][qy][qx] - cc : 0.0) +
                    (hu ? L[a][sp][qy][qx] - cc : 0.0) +
                    (hn ? L[a][s0][qy - 1][qx] - cc : 0.0) +
                    (hs ? L[a][s0][qy + 1][qx] - cc : 0.0) +
                    (hw ? L[a][s0][qy][qx - 1] - cc : 0.0) +
                    (he ? L[a][s0][qy][qx + 1] - cc : 0.0);
            } else {
              const int dn = (zz - 1 - z0 + 2) % 5, up = (zz + 1 - z0 + 2) % 5;
              const double cc = pc[a];
              btb = -(((double)P[a][dn][py][px] - cc) +
                      ((double)P[a][up][py][px] - cc) +
                      ((double)P[a][c][py - 1][px] - cc) +
                      ((double)P[a][c][py + 1][px] - cc) +
                      ((double)P[a][c][py][px - 1] - cc) +
                      ((double)P[a][c][py][px + 1] - cc));
            }
            const double h = ds * d[a] + md.alpha_hd * md.reg_scale * btb +
                             md.lam_c * vbar[a];
            const float hf = (float)h;
            q[jb + (size_t)a * N] = hf;
            p_new[jb + (size_t)a * N] = (float)pc[a];
            acc += pc[a] * (double)hf;
          }
        }
      }
      __syncthreads();
    }
  }
  double vals[1] = {acc};
  block_partials<1>(vals, 0u, part, blk);
}

// Two 512-thread blocks per compute unit (at most 128 registers per lane;
// the LDS rings take 64 KB).  Columns of 32 x 16 measured 15% faster than
// 16 x 16 ones (less halo per output), and than 64 x 16, 32 x 32 and 32 x 8.
template <int REG, bool FIRST>
__global__ __launch_bounds__(kHv3Threads, 4) void cgt_hvp3_kernel(
    int it, const float* __restrict__ zv, const float* __restrict__ p_old,
    float* __restrict__ p_new, const float* __restrict__ dW, Geom g,
    Model md, float* __restrict__ q, float* __restrict__ x,
    const double* __restrict__ Sz,
    const float* __restrict__ Vz, const double* __restrict__ Sp_old,
    const float* __restrict__ Vp_old, double* __restrict__ Sp_new,
    float* __restrict__ Vp_new, int nreal, int nfg, int fpg,
    const double* __restrict__ up_part, int up_nb, int fixed, double rtol,
    double* __restrict__ part, Scal* __restrict__ sc, int gn_it) {
  cgt_hvp3_body<REG, FIRST>(it, zv, p_old, p_new, dW, g, md, q, x, Sz, Vz,
                            Sp_old, Vp_old, Sp_new, Vp_new, nreal, nfg, fpg,
                            up_part, up_nb, fixed, rtol, part, sc, gn_it,
                            grid_blk());
}

// ------------------------------------------------------------ launchers

static int cgv_blocks(const Geom& g) {
  long long ntiles = (g.N + kWave - 1) / kWave;
  long long nb = ntiles < g.vox_cap ? ntiles : g.vox_cap;
  return (int)((nb + kXCD - 1) / kXCD * kXCD);
}

// A fixed block size (waves without frames idle), so that a problem gets
// the same blocks, and the same rounding, alone and batched.
static int cgv_threads(int dim, int nK) {
  (void)dim;
  (void)nK;
  return kMaxChunks * kWave;
}

int cg_tile_count(const Geom& g, int dim) {
  if (dim == 2)
    return ((g.m[1] + kTX - 1) / kTX) * ((g.m[0] + kTY - 1) / kTY);
  return ((g.m[2] + kT3X - 1) / kT3X) * ((g.m[1] + kT3Y - 1) / kT3Y) *
         ((g.m[0] + kT3Z - 1) / kT3Z);
}

CgTiles cg_tiles(const Geom& g, int nK, int dim) {
  CgTiles t;
  int ntiles = cg_tile_count(g, dim);
  int nfg = (g.hv_target + ntiles - 1) / ntiles;
  if (nfg > nK) nfg = nK;
  if (nfg < 1) nfg = 1;
  t.fpg = (nK + nfg - 1) / nfg;
  t.nfg = (nK + t.fpg - 1) / t.fpg;
  t.nreal = ntiles * t.nfg;
  t.grid = (t.nreal + kXCD - 1) / kXCD * kXCD;
  t.vox_grid = cgv_blocks(g);
  return t;
}

hipError_t launch_cgt_hvp(int it, const float* z, const float* p_old,
                          float* p_new, const float* dW, const Geom& g,
                          const Model& md, float* q, float* x, CgSums sums,
                          int fixed,
                          double rtol, RedBuf rb, Scal* sc, hipStream_t s,
                          int gn_it, hipEvent_t ev0, hipEvent_t ev1) {
  const int dim = geom_dim(g);
  CgTiles t = cg_tiles(g, md.nK, dim);
  const double* Sp_old = sums.Sp[(it + 1) & 1];
  const float* Vp_old = sums.Vp[(it + 1) & 1];
  double* Sp_new = sums.Sp[it & 1];
  float* Vp_new = sums.Vp[it & 1];
  // with events: the dispatch records its own start and end
  decltype(&cgt_hvp2_kernel<0, true>) kern;
  if (it == 0)
    kern = dim == 2 ? (md.reg == 0 ? cgt_hvp2_kernel<0, true>
                                   : cgt_hvp2_kernel<1, true>)
                    : (md.reg == 0 ? cgt_hvp3_kernel<0, true>
                                   : cgt_hvp3_kernel<1, true>);
  else
    kern = dim == 2 ? (md.reg == 0 ? cgt_hvp2_kernel<0, false>
                                   : cgt_hvp2_kernel<1, false>)
                    : (md.reg == 0 ? cgt_hvp3_kernel<0, false>
                                   : cgt_hvp3_kernel<1, false>);
  if (dim == 3 && it > 0) {
    // the sums of p first (timed with the product: start event here)
    hipExtLaunchKernelGGL(cg_psums_kernel, dim3(cgv_blocks(g)),
                          dim3(cgv_threads(dim, md.nK)), 0, s, ev0, nullptr,
                          0, it, sums.Sz, sums.Vz, Sp_old, Vp_old, Sp_new,
                          Vp_new, g.N, (const double*)rb.region(kRegUpdate),
                          t.vox_grid, fixed, rtol, sc, gn_it);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ev0 = nullptr;
  }
  hipExtLaunchKernelGGL(kern, dim3(t.grid),
                        dim3(dim == 2 ? kHv2Threads : kHv3Threads), 0, s, ev0,
                        ev1, 0, it, z, p_old, p_new, dW, g, md, q, x, sums.Sz,
                        sums.Vz, Sp_old, Vp_old, Sp_new, Vp_new, t.nreal,
                        t.nfg, t.fpg, (const double*)rb.region(kRegUpdate),
                        t.vox_grid, fixed, rtol, rb.region(kRegHv), sc, gn_it);
  return hipGetLastError();
}

// The update's forms: (dimension, two blocks per compute unit, CG step 0,
// x mode).
#define STML_CGV_FORMS(D, OCC)                                              \
  {cgv_update_kernel<D, OCC, true, kXNone>,                                 \
   cgv_update_kernel<D, OCC, true, kXOne>,                                  \
   cgv_update_kernel<D, OCC, false, kXNone>,                                \
   cgv_update_kernel<D, OCC, false, kXOne>,                                 \
   cgv_update_kernel<D, OCC, false, kXTwo>,                                 \
   cgv_update_kernel<D, OCC, false, kXTwoFirst>}

// index of the form for step it of cg_max: step 0 (x untouched or x = a p),
// then the four modes of later steps
static int cgv_form(int it, int cg_max) {
  const int xm = cg_x_mode(it, cg_max);
  return it == 0 ? (xm == kXOne ? 1 : 0) : 2 + xm;
}

hipError_t launch_cgv_update(int dim, int it, int cg_max, int brk,
                             const float* p,
                             const float* p_prev, const float* q,
                             const float* dW, const Geom& g, const Model& md,
                             float* x, float* r, float* z, CgSums sums,
                             RedBuf rb, Scal* sc, hipStream_t s, int gn_it,
                             GNLog* log, hipEvent_t ev0, hipEvent_t ev1) {
  int nb = cgv_blocks(g), nt = cgv_threads(dim, md.nK);
  int hv_nb = cg_tiles(g, md.nK, dim).grid;
  const bool occ = nb > kCUs;
  using Kern = decltype(&cgv_update_kernel<2, true, true, kXNone>);
  static const Kern forms[2][2][6] = {
      {STML_CGV_FORMS(2, false), STML_CGV_FORMS(2, true)},
      {STML_CGV_FORMS(3, false), STML_CGV_FORMS(3, true)}};
  const Kern kern = forms[dim == 3][occ][cgv_form(it, cg_max)];
  hipExtLaunchKernelGGL(kern, dim3(nb), dim3(nt), 0, s, ev0, ev1, 0, it, p,
                        p_prev, q, dW, g, md, x, r, z, sums.Sz, sums.Vz,
                        (const double*)rb.region(kRegHv), hv_nb,
                        rb.region(kRegUpdate), sc, gn_it,
                        (const double*)rb.region(kRegEval), tile_blocks(g),
                        log, brk);
  return hipGetLastError();
}

// ------------------------------------------------------ batched iteration

__device__ __forceinline__ int cg_job_index(const int* __restrict__ f, int n,
                                            int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (f[mid] <= b) lo = mid;
    else hi = mid;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

__device__ __forceinline__ const Job& cg_job_of(const JobSet& js, int c,
                                                Blk& blk) {
  const int* f = js.first + (size_t)c * (js.n + 1);
  const int b = blockIdx.x;
  const int j = cg_job_index(f, js.n, b);
  blk = Blk{b - f[j], f[j + 1] - f[j]};
  return js.jobs[j];
}

template <int D, int REG, bool FIRST>
__global__ __launch_bounds__(D == 2 ? kHv2Threads : kHv3Threads,
                             D == 3 ? 4 : (REG ? 7 : 5)) void cg_hvp_batch_kernel(
    JobSet js, int it, int fixed, double rtol) {
  Blk blk;
  const Job& J = cg_job_of(js, kClsHv, blk);
  const Geom g = J.g;
  const Model md = J.md;
  Scal* sc = J.sc;
  float* pn = (it & 1) ? J.P1 : J.P0;
  const float* po = (it & 1) ? J.P0 : J.P1;
  if constexpr (D == 2)
    cgt_hvp2_body<REG, FIRST>(it, J.z, po, pn, J.dW, g, md, J.q, J.x, J.sums.Sz,
                       J.sums.Vz, J.sums.Sp[(it + 1) & 1],
                       J.sums.Vp[(it + 1) & 1], J.sums.Sp[it & 1],
                       J.sums.Vp[it & 1], J.ct.nreal, J.ct.nfg, J.ct.fpg,
                       J.rb.region(kRegUpdate), J.nb_vox, fixed, rtol,
                       J.rb.region(kRegHv), sc, sc->gn_cur, blk);
  else
    cgt_hvp3_body<REG, FIRST>(it, J.z, po, pn, J.dW, g, md, J.q, J.x, J.sums.Sz,
                       J.sums.Vz, J.sums.Sp[(it + 1) & 1],
                       J.sums.Vp[(it + 1) & 1], J.sums.Sp[it & 1],
                       J.sums.Vp[it & 1], J.ct.nreal, J.ct.nfg, J.ct.fpg,
                       J.rb.region(kRegUpdate), J.nb_vox, fixed, rtol,
                       J.rb.region(kRegHv), sc, sc->gn_cur, blk);
}

__global__ __launch_bounds__(1024) void cg_psums_batch_kernel(JobSet js, int it,
                                                             int fixed,
                                                             double rtol) {
  Blk blk;
  const Job& J = cg_job_of(js, kClsVox, blk);
  Scal* sc = J.sc;
  cg_psums_body(it, J.sums.Sz, J.sums.Vz, J.sums.Sp[(it + 1) & 1],
                J.sums.Vp[(it + 1) & 1], J.sums.Sp[it & 1], J.sums.Vp[it & 1],
                J.g.N, J.rb.region(kRegUpdate), J.nb_vox, fixed, rtol, sc,
                sc->gn_cur, blk);
}

template <int D, bool FIRST, int XM>
__global__ __launch_bounds__(1024, 8) void cg_update_batch_kernel(JobSet js,
                                                               int it) {
  Blk blk;
  const Job& J = cg_job_of(js, kClsVox, blk);
  const Geom g = J.g;
  const Model md = J.md;
  Scal* sc = J.sc;
  const float* pn = (it & 1) ? J.P1 : J.P0;
  const float* po = (it & 1) ? J.P0 : J.P1;
  cgv_update_body<D, FIRST, false, XM>(
      it, pn, po, J.q, J.dW, g, md, J.x, J.r, J.z, J.sums.Sz, J.sums.Vz,
      J.rb.region(kRegHv), J.ct.grid, J.rb.region(kRegUpdate), sc,
      sc->gn_cur, J.rb.region(kRegEval), J.nb_tile, J.log, -1, blk);
}

template <int D>
__global__ __launch_bounds__(1024) void cg_zero_x_batch_kernel(JobSet js) {
  Blk blk;
  const Job& J = cg_job_of(js, kClsVox, blk);
  const Scal* sc = J.sc;
  if (sc->gn_cur >= sc->gn_stop) return;
  cg_zero_x<D>(J.x, J.g, J.md, blk);
}

void job_shape(Job* job) {
  const int dim = geom_dim(job->g);
  job->ct = cg_tiles(job->g, job->md.nK, dim);
  job->nb_tile = tile_blocks(job->g);
  job->nb_vox = job->ct.vox_grid;
  job->count = (long long)job->md.nK * dim * job->g.N;
  job->nb_elem = elem_grid(job->count);
}

hipError_t batch_zero_x(const JobSet& js, int nvox, int dim, hipStream_t s) {
  if (dim == 2)
    cg_zero_x_batch_kernel<2><<<nvox, cgv_threads(2, 0), 0, s>>>(js);
  else
    cg_zero_x_batch_kernel<3><<<nvox, cgv_threads(3, 0), 0, s>>>(js);
  return hipGetLastError();
}

hipError_t batch_cg_hvp(const JobSet& js, int nhv, int nvox, int dim, int reg,
                        int it, int fixed, double rtol, hipStream_t s) {
  if (dim == 3 && it > 0) {
    cg_psums_batch_kernel<<<nvox, cgv_threads(3, 0), 0, s>>>(js, it, fixed,
                                                             rtol);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  decltype(&cg_hvp_batch_kernel<2, 0, true>) kern;
  if (it == 0)
    kern = dim == 2 ? (reg == 0 ? cg_hvp_batch_kernel<2, 0, true>
                                : cg_hvp_batch_kernel<2, 1, true>)
                    : (reg == 0 ? cg_hvp_batch_kernel<3, 0, true>
                                : cg_hvp_batch_kernel<3, 1, true>);
  else
    kern = dim == 2 ? (reg == 0 ? cg_hvp_batch_kernel<2, 0, false>
                                : cg_hvp_batch_kernel<2, 1, false>)
                    : (reg == 0 ? cg_hvp_batch_kernel<3, 0, false>
                                : cg_hvp_batch_kernel<3, 1, false>);
  kern<<<nhv, dim == 2 ? kHv2Threads : kHv3Threads, 0, s>>>(js, it, fixed,
                                                            rtol);
  return hipGetLastError();
}

#define STML_CGV_BATCH_FORMS(D)                                             \
  {cg_update_batch_kernel<D, true, kXNone>,                                 \
   cg_update_batch_kernel<D, true, kXOne>,                                  \
   cg_update_batch_kernel<D, false, kXNone>,                                \
   cg_update_batch_kernel<D, false, kXOne>,                                 \
   cg_update_batch_kernel<D, false, kXTwo>,                                 \
   cg_update_batch_kernel<D, false, kXTwoFirst>}

hipError_t batch_cg_update(const JobSet& js, int nvox, int dim, int it,
                           int cg_max, hipStream_t s) {
  using Kern = decltype(&cg_update_batch_kernel<2, true, kXNone>);
  static const Kern forms[2][6] = {STML_CGV_BATCH_FORMS(2),
                                   STML_CGV_BATCH_FORMS(3)};
  forms[dim == 3][cgv_form(it, cg_max)]<<<nvox, cgv_threads(dim, 0), 0, s>>>(
      js, it);
  return hipGetLastError();
}

hipError_t launch_hessvec_tiled(const float* v, const float* dW,
                                const Geom& g, const Model& md, float* hv,
                                float* vcopy, CgSums sums, RedBuf rb,
                                Scal* sc, hipStream_t s) {
  const int dim = geom_dim(g);
  int nb = cgv_blocks(g), nt = cgv_threads(dim, md.nK);
  if (dim == 2)
    cgv_sums_kernel<2><<<nb, nt, 0, s>>>(v, dW, g, md, sums.Sz, sums.Vz);
  else
    cgv_sums_kernel<3><<<nb, nt, 0, s>>>(v, dW, g, md, sums.Sz, sums.Vz);
  hipError_t e = launch_gn_reset(sc, nullptr, 0, s);
  if (e != hipSuccess) return e;
  e = launch_cgt_hvp(0, v, nullptr, vcopy, dW, g, md, hv, nullptr, sums, 1,
                     0.0, rb, sc, s, 0);
  if (e != hipSuccess) return e;
  return launch_finalize_vhv(rb.region(kRegHv), cg_tiles(g, md.nK, dim).grid,
                             sc, s);
}

}  // namespace stml
