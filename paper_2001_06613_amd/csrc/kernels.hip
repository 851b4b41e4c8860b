// HIP kernels of the STML registration path for gfx950 (CDNA4, wave64).
//
// Tile kernels (evaluation, trial steps) give every block one or more
// 64-voxel tiles; the waves of a block split the frames of the subset K
// between them, so each voxel's cross-frame means (mean warped image, mean
// displacement) are combined through LDS; the evaluation keeps W and dW/du
// of a wave's first frames in LDS for its second sweep.  All warp and residual
// arithmetic is float64 from float32 loads; every reduction is float64 and
// deterministic.
#include <math.h>

#include "launch.h"
#include "reduce.h"

namespace stml {

// ------------------------------------------------------------------ setup

Geom make_geom(int dim, const int* ext, double h) {
  Geom g;
  g.m[0] = ext[0];
  g.m[1] = ext[1];
  g.m[2] = dim == 3 ? ext[2] : 1;
  if (dim == 2) {
    g.s[1] = 1;
    g.s[0] = g.m[1];
    g.s[2] = 0;
    g.N = (long long)g.m[0] * g.m[1];
  } else {
    g.s[2] = 1;
    g.s[1] = g.m[2];
    g.s[0] = (long long)g.m[1] * g.m[2];
    g.N = (long long)g.m[0] * g.m[1] * g.m[2];
  }
  g.inv_h = 1.0 / h;
  g.tile_cap = kMaxTileBlocks;
  g.vox_cap = kMaxTileBlocks;
  g.hv_target = kHvBlocks;
  return g;
}

Model make_model(int dim, double h, int nK, double alpha, double lambda,
                 int reg) {
  Model md;
  double hd = dim == 3 ? h * h * h : h * h;
  md.hd = hd;
  md.data_c = 2.0 * hd;
  md.mdiag_c = 2.0 * hd * (1.0 - 1.0 / nK);
  md.alpha_hd = alpha * hd;
  md.half_alpha_hd = 0.5 * alpha * hd;
  md.lam_hd = lambda * hd;
  md.lam_c = 2.0 * lambda * hd / nK;
  md.pen_diag = 2.0 * lambda * hd / ((double)nK * nK);
  md.reg_scale = reg == 0 ? 1.0 / (h * h) : 1.0 / (h * h * h * h);
  md.inv_nK = 1.0 / nK;
  md.reg = reg;
  md.nK = nK;
  return md;
}

static int round_up(long long v, int m) { return (int)((v + m - 1) / m * m); }

int tile_blocks(const Geom& g) {
  long long ntiles = (g.N + kWave - 1) / kWave;
  long long nb = ntiles < g.tile_cap ? ntiles : g.tile_cap;
  return round_up(nb, kXCD);
}

// Waves per block split the frames of K; more waves shorten the per-wave
// frame loops (latency) at the cost of registers and LDS: 8 for the 2-D
// evaluation and trial sweeps, 4 in 3-D.  The block size does not depend on
// |K| (waves without frames idle), so that a problem gets the same blocks,
// and the same rounding, alone and batched.
int tile_threads(int dim, int nK) {
  (void)nK;
  return (dim == 2 ? 8 : 4) * kWave;
}
int eval_threads(int dim, int nK) {
  (void)nK;
  return (dim == 2 ? 8 : 4) * kWave;
}

#define STML_DIM_DISPATCH(dim, KERNEL, GRID, BLOCK, STREAM, ...)          \
  do {                                                                    \
    if ((dim) == 2)                                                       \
      KERNEL<2><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);                 \
    else                                                                  \
      KERNEL<3><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);                 \
  } while (0)

// (dimension, regulariser) specialisations of the tile kernels.
#define STML_TILE_DISPATCH(dim, reg, KERNEL, GRID, BLOCK, STREAM, ...)     \
  do {                                                                    \
    if ((dim) == 2 && (reg) == 0)                                         \
      KERNEL<2, 0><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);              \
    else if ((dim) == 2)                                                  \
      KERNEL<2, 1><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);              \
    else if ((reg) == 0)                                                  \
      KERNEL<3, 0><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);              \
    else                                                                  \
      KERNEL<3, 1><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);              \
  } while (0)

static int elem_blocks(size_t count, int per_thread = 4) {
  size_t nb = (count + 256 * per_thread - 1) / (256 * per_thread);
  if (nb < 1) nb = 1;
  if (nb > kMaxElemBlocks) nb = kMaxElemBlocks;
  return (int)nb;
}

// --------------------------------------------------------- simple kernels

__global__ void fill_kernel(float* __restrict__ p, size_t count, float v) {
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += stride)
    p[i] = v;
}

__global__ void check_finite_kernel(const float* __restrict__ p, size_t count,
                                    Scal* sc) {
  size_t stride = (size_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += stride)
    bad += !isfinite(p[i]);
  if (bad) atomicAdd(&sc->bad, bad);
}

// One spatial restriction step: coarse cell = mean of the existing fine
// cells 2I + {0,1}^D (extents halve rounding up).
template <int D>
__global__ void restrict_kernel(const float* __restrict__ fine,
                                float* __restrict__ coarse, int n, Geom gf,
                                Geom gc) {
  long long total = (long long)n * gc.N;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
       e < total; e += stride) {
    int k = (int)(e / gc.N);
    long long xc = e - (long long)k * gc.N;
    Pos<D> pc = make_pos<D>(gc, xc);
    const float* f = fine + (size_t)k * gf.N;
    double sum = 0.0;
    int cnt = 0;
#pragma unroll
    for (int o = 0; o < (1 << D); ++o) {
      long long idx = 0;
      bool ok = true;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        int c = 2 * pc.c[a] + ((o >> (D - 1 - a)) & 1);
        ok = ok && (c < gf.m[a]);
        idx += (long long)c * gf.s[a];
      }
      if (ok) {
        sum += (double)f[idx];
        ++cnt;
      }
    }
    coarse[e] = (float)(sum / cnt);
  }
}

// Prolongation: the coarse cell-centred linear interpolant (edge clamp)
// sampled at fine cell centres; fine index i sits at coarse coordinate
// i/2 - 1/4.  Blocks in y split the fields (frames x components), so that a
// thread interpolates a few fields of its voxel rather than all of them.
template <int D>
__global__ void prolong_kernel(const float* __restrict__ coarse,
                               float* __restrict__ fine, int fields, Geom gc,
                               Geom gf) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
       x < gf.N; x += stride) {
    Pos<D> pf = make_pos<D>(gf, x);
    int i0[D], i1[D];
    double f[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      int M = gc.m[a];
      double q = 0.5 * (double)pf.c[a] - 0.25;
      q = fmin(fmax(q, 0.0), (double)(M - 1));
      if (M >= 2) {
        int fl = (int)floor(q);
        i0[a] = fl < M - 2 ? fl : M - 2;
        f[a] = q - i0[a];
        i1[a] = i0[a] + 1;
      } else {
        i0[a] = i1[a] = 0;
        f[a] = 0.0;
      }
    }
    for (int fi = blockIdx.y; fi < fields; fi += gridDim.y) {
      const float* c = coarse + (size_t)fi * gc.N;
      double v = 0.0;
#pragma unroll
      for (int o = 0; o < (1 << D); ++o) {
        double w = 1.0;
        long long idx = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          int bit = (o >> (D - 1 - a)) & 1;
          w *= bit ? f[a] : 1.0 - f[a];
          idx += (long long)(bit ? i1[a] : i0[a]) * gc.s[a];
        }
        v += w * (double)c[idx];
      }
      fine[(size_t)fi * gf.N + x] = (float)v;
    }
  }
}

// ---------------------------------------------------------- tile kernels

// Split of the frames 0..nK-1 between the waves of a block.
struct Chunk {
  int j0, j1;
};
__device__ __forceinline__ Chunk frame_chunk(int nK) {
  int G = blockDim.x / kWave;
  int w = wave_id();
  int per = (nK + G - 1) / G;
  int j0 = w * per;
  int j1 = j0 + per < nK ? j0 + per : nK;
  return {j0, j1};
}

// Objective (D, S, P), gradient and dW/du at u for the frames K.
// Sweep 1 over the wave's frames warps every frame, stores dW/du and sums
// W and u per voxel; after the LDS combine, sweep 2 forms r = W - mean W and
// writes the gradient, taking W and dW/du of a wave's first frames from LDS
// and warping the rest again.  The gradient uses dW/du rounded to float32,
// the values the Hessian product uses.  Block partials of D, S, P go to
// `part` (3 x gridDim slots).
// INIT: sweep 2 also starts the Jacobi-PCG of the Gauss-Newton step from
// the float32 gradient just written: r = -g, z = r / M with M recomputed
// from the float32 dW/du, per-voxel S_z = sum_k dW_k . z_k and V_z =
// sum_k z_k (combined over the waves in LDS), and partials of r.z and r.r
// after those of D, S, P (5 x gridDim slots).
// PAIR (grids of at most one block per compute unit, where a wave's frames
// in turn are the latency): both sweeps take two frames per pass, whose
// loads issue together (in sweep 2 all stencils of both frames before any
// arithmetic); every value is formed and accumulated as one frame at a time,
// in the same order, so the results are bitwise those of the plain form.
template <int D, int REG, bool INIT, bool PAIR = false>
__device__ __forceinline__ void eval_body(
    const float* __restrict__ T, const float* __restrict__ u,
    const int* __restrict__ K, const Geom& g, const Model& md,
    float* __restrict__ grad, float* __restrict__ dWo,
    double* __restrict__ part, int gn_it, const Scal* __restrict__ sc,
    CgStart cs, Blk blk) {
  if (sc && gn_it >= sc->gn_stop) return;
  constexpr int G_ = D == 2 ? 8 : 4;   // waves per block (eval_threads)
  // W and dW/du (rounded to float32, as stored) of a wave's first kWF frames
  // stay in LDS between the sweeps: the second sweep needs neither the
  // displacement nor the frame again for them
  constexpr int kWF = 8;
  __shared__ double xs[G_][kWave][1 + D];
  __shared__ double wc[G_][kWF][kWave];
  __shared__ float dc[G_][kWF][D][kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = wave_id();
  const int G = blockDim.x / kWave;
  const Chunk ch = frame_chunk(md.nK);
  const long long N = g.N;
  const long long ntiles = (N + kWave - 1) / kWave;
  double accD = 0.0, accS = 0.0, accP = 0.0, rz = 0.0, rr = 0.0;
  for (int it = 0;; ++it) {
    long long tile = xcd_tile(ntiles, it, blk);
    if (tile < 0) break;
    tile = stencil_tile<D>(g, tile);
    long long x = tile * kWave + lane;
    bool valid = x < N;
    Pos<D> p = make_pos<D>(g, valid ? x : N - 1);
    double sz = 0.0, vz[D];
#pragma unroll
    for (int a = 0; a < D; ++a) vz[a] = 0.0;
    double sW = 0.0, sU[D];
#pragma unroll
    for (int a = 0; a < D; ++a) sU[a] = 0.0;
    // sweep 1, one frame: displacement, then the warp's gathers
    auto s1_load = [&](int j, double* uv) {
      const float* uk = u + (size_t)K[j] * D * N;
#pragma unroll
      for (int a = 0; a < D; ++a) uv[a] = (double)uk[(size_t)a * N + p.idx];
    };
    auto s1_frame = [&](int j, const double* uv, double W, const double* dw) {
      sW += W;
      if (j - ch.j0 < kWF) {
        wc[w][j - ch.j0][lane] = W;
#pragma unroll
        for (int a = 0; a < D; ++a) dc[w][j - ch.j0][a][lane] = (float)dw[a];
      }
      float* dj = dWo ? dWo + (size_t)j * D * N : nullptr;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        sU[a] += uv[a];
        if (valid && dj) dj[(size_t)a * N + p.idx] = (float)dw[a];
      }
    };
    if (PAIR) {
      for (int j = ch.j0; j < ch.j1; j += 2) {
        const int jb = j + 1 < ch.j1 ? j + 1 : j;
        double u0[D], u1[D], dw0[D], dw1[D], W0, W1;
        s1_load(j, u0);
        s1_load(jb, u1);
        warp_sample<D>(T + (size_t)K[j] * N, g, p, u0, W0, dw0);
        warp_sample<D>(T + (size_t)K[jb] * N, g, p, u1, W1, dw1);
        s1_frame(j, u0, W0, dw0);
        if (jb != j) s1_frame(jb, u1, W1, dw1);
      }
    } else {
      for (int j = ch.j0; j < ch.j1; ++j) {
        double uv[D], dw[D], W;
        s1_load(j, uv);
        warp_sample<D>(T + (size_t)K[j] * N, g, p, uv, W, dw);
        s1_frame(j, uv, W, dw);
      }
    }
    xs[w][lane][0] = sW;
#pragma unroll
    for (int a = 0; a < D; ++a) xs[w][lane][1 + a] = sU[a];
    __syncthreads();
    double Wb = 0.0, ub[D];
#pragma unroll
    for (int a = 0; a < D; ++a) ub[a] = 0.0;
    for (int c = 0; c < G; ++c) {
      Wb += xs[c][lane][0];
#pragma unroll
      for (int a = 0; a < D; ++a) ub[a] += xs[c][lane][1 + a];
    }
    __syncthreads();
    Wb *= md.inv_nK;
#pragma unroll
    for (int a = 0; a < D; ++a) ub[a] *= md.inv_nK;
    if (valid) {
      const double rest = INIT ? jacobi_rest<D>(p, g, md) : 0.0;
      const Nbr<D> nbr = neighbours<D>(p, g);
      constexpr int NP = RegPts<D, REG>::kN;
      // sweep 2, one frame: W and dW/du (from LDS, or warped again)
      auto s2_wd = [&](int j, double& W, double* dw) {
        if (j - ch.j0 < kWF) {
          W = wc[w][j - ch.j0][lane];
#pragma unroll
          for (int a = 0; a < D; ++a) dw[a] = (double)dc[w][j - ch.j0][a][lane];
        } else {
          const float* uk = u + (size_t)K[j] * D * N;
          double uv[D];
#pragma unroll
          for (int a = 0; a < D; ++a)
            uv[a] = (double)uk[(size_t)a * N + p.idx];
          warp_sample<D>(T + (size_t)K[j] * N, g, p, uv, W, dw);
#pragma unroll
          for (int a = 0; a < D; ++a) dw[a] = (double)(float)dw[a];
        }
      };
      // ... then the residual, the regulariser terms from the loaded
      // stencils of its components, the gradient and the PCG start
      auto s2_comp = [&](int j, int a, double r, const double* dw,
                         const float (&va)[NP]) {
        float* gj = grad ? grad + (size_t)j * D * N : nullptr;
        {
          double btb, e, cen;
          reg_eval<D, REG>(va, nbr, btb, e, cen);
          accS += e;
          if (gj) {
            double gv = md.data_c * r * dw[a] +
                        md.alpha_hd * md.reg_scale * btb + md.lam_c * ub[a];
            const float gf = (float)gv;
            gj[(size_t)a * N + p.idx] = gf;
            if (INIT) {
              const size_t o = ((size_t)j * D + a) * N + p.idx;
              const float rv = -gf;
              const float zv =
                  (float)((double)rv / (md.mdiag_c * dw[a] * dw[a] + rest));
              cs.r[o] = rv;
              cs.z[o] = zv;
              rz += (double)rv * (double)zv;
              rr += (double)rv * (double)rv;
              sz += dw[a] * (double)zv;
              vz[a] += (double)zv;
            }
          }
        }
      };
      auto s2_frame = [&](int j, double W, const double* dw,
                          const float (*v)[NP]) {
        const double r = W - Wb;
        accD += r * r;
#pragma unroll
        for (int a = 0; a < D; ++a) s2_comp(j, a, r, dw, v[a]);
      };
      auto s2_load = [&](int j, float (*v)[NP]) {
        const float* uk = u + (size_t)K[j] * D * N;
#pragma unroll
        for (int a = 0; a < D; ++a)
          reg_load<D, REG>(Src1{uk + (size_t)a * N}, p, nbr, v[a]);
      };
      if (PAIR) {
        for (int j = ch.j0; j < ch.j1; j += 2) {
          const int jb = j + 1 < ch.j1 ? j + 1 : j;
          double W0, W1, dw0[D], dw1[D];
          float v0[D][NP], v1[D][NP];
          s2_wd(j, W0, dw0);
          s2_wd(jb, W1, dw1);
          s2_load(j, v0);
          s2_load(jb, v1);
          // keep the stencil loads of both frames together
          __builtin_amdgcn_sched_barrier(0);
          s2_frame(j, W0, dw0, v0);
          if (jb != j) s2_frame(jb, W1, dw1, v1);
        }
      } else {
        for (int j = ch.j0; j < ch.j1; ++j) {
          double W, dw[D];
          s2_wd(j, W, dw);
          if (D == 3) {
            // volumes (no register cap): the stencils of all components
            // before any arithmetic
            float v[D][NP];
            s2_load(j, v);
            __builtin_amdgcn_sched_barrier(0);
            s2_frame(j, W, dw, v);
            continue;
          }
          const double r = W - Wb;
          accD += r * r;
          // one component's stencil at a time: its loads, then its terms
#pragma unroll
          for (int a = 0; a < D; ++a) {
            float va[NP];
            reg_load<D, REG>(Src1{u + ((size_t)K[j] * D + a) * N}, p, nbr,
                             va);
            __builtin_amdgcn_sched_barrier(0);
            s2_comp(j, a, r, dw, va);
          }
        }
      }
      if (w == 0) {
#pragma unroll
        for (int a = 0; a < D; ++a) accP += ub[a] * ub[a];
      }
    }
    if (INIT) {
      // per-voxel S_z and V_z over the waves' frames: wave c sums value c
      xs[w][lane][0] = sz;
#pragma unroll
      for (int a = 0; a < D; ++a) xs[w][lane][1 + a] = vz[a];
      __syncthreads();
      if (w <= D && valid) {
        double t = 0.0;
        for (int c = 0; c < G; ++c) t += xs[c][lane][w];
        if (w == 0) cs.Sz[x] = t;
        else cs.Vz[(size_t)(w - 1) * N + x] = t;
      }
      __syncthreads();
    }
  }
  if (INIT) {
    double vals[5] = {accD, accS, accP, rz, rr};
    block_partials<5>(vals, 0u, part, blk);
  } else {
    double vals[3] = {accD, accS, accP};
    block_partials<3>(vals, 0u, part, blk);
  }
}

// Two 8-wave blocks per compute unit in 2-D (LDS allows two): at most 128
// registers per lane.  The paired form runs on grids of at most one block
// per compute unit: at most 256.
template <int D, int REG, bool INIT, bool PAIR = false>
__global__ __launch_bounds__(D == 2 ? 512 : 256,
                             D == 2 ? (PAIR ? 2 : 4) : 1) void eval_kernel(
    const float* __restrict__ T, const float* __restrict__ u,
    const int* __restrict__ K, Geom g, Model md, float* __restrict__ grad,
    float* __restrict__ dWo, double* __restrict__ part, int gn_it,
    const Scal* __restrict__ sc, CgStart cs) {
  eval_body<D, REG, INIT, PAIR>(T, u, K, g, md, grad, dWo, part, gn_it, sc,
                                cs, grid_blk());
}

// One block: the objective of the evaluation and the CG start scalars (the
// five partials of an evaluation that formed the CG start).
__device__ __forceinline__ void finalize_start_body(
    const double* __restrict__ ev_part, int ev_nb, const Model& md,
    Scal* __restrict__ sc, int gn_it, GNLog* __restrict__ log) {
  if (gn_it >= sc->gn_stop) return;
  double e[5];
  reduce_partials<5>(ev_part, ev_nb, 0u, e);
  const double i2[2] = {e[3], e[4]};
  if (threadIdx.x == 0) {
    double Dv = md.hd * e[0];
    double Sv = md.half_alpha_hd * md.reg_scale * e[1];
    double Pv = md.lam_hd * e[2];
    sc->D = Dv;
    sc->S = Sv;
    sc->P = Pv;
    sc->J = Dv + Sv + Pv;
    sc->rzh[0] = i2[0];
    sc->r0 = sqrt(i2[1]);
    sc->rr = i2[1];
    sc->iters = 0;
    sc->done = i2[0] == 0.0 ? 1 : 0;
    if (log) log[gn_it].J = Dv + Sv + Pv;
    // a start at or below the target takes no step (the stop tests of the
    // accept kernel run only where a step was taken)
    if (gn_it == 0 && Dv + Sv + Pv <= sc->J_target) sc->gn_stop = 0;
  }
}

__global__ __launch_bounds__(256) void finalize_start_kernel(
    const double* __restrict__ ev_part, int ev_nb, Model md,
    Scal* __restrict__ sc, int gn_it, GNLog* __restrict__ log) {
  finalize_start_body(ev_part, ev_nb, md, sc, gn_it, log);
}

// Totals of line-search sweep q (its objective values Jt at its steps, by
// the exact quadratic expansion of S and P) and of sweep 0 (the reference
// J0t = J(t = 0), the slope g.delta, max |delta| and sum delta^2).
struct SweepTotals {
  double Jt[kTrialSteps];
  double J0t, slope, maxd, ssqd;
};

template <int NT>
__device__ __forceinline__ void sweep_objectives(const double (&out)[NT + 9],
                                                 int q, int ls_max,
                                                 const Model& md,
                                                 double (&Jt)[kTrialSteps]) {
  const double sA = md.half_alpha_hd * md.reg_scale;
#pragma unroll
  for (int s = 0; s < NT; ++s) {
    const double t = sweep_t(q, s, ls_max);
    const double Dv = md.hd * out[s];
    const double Sv =
        sA * (out[NT] + 2.0 * t * out[NT + 1] + t * t * out[NT + 2]);
    const double Pv = md.lam_hd * (out[NT + 3] + 2.0 * t * out[NT + 4] +
                                   t * t * out[NT + 5]);
    Jt[s] = Dv + Sv + Pv;
  }
}

// LDS of sweep_totals (reused by the two reductions in turn)
constexpr int kSweepLds = reduce_lds_doubles<kTrialSteps + 9>();

__device__ SweepTotals sweep_totals(RedBuf rb, int nb, int q, int ls_max,
                                    const Model& md, double* lds) {
  constexpr int N0 = kSweep0Steps, N1 = kTrialSteps;
  SweepTotals st;
  double o0[N0 + 9];
  reduce_partials_in<N0 + 9>(rb.region(kRegTrial), nb, 1u << (N0 + 7), o0,
                             lds);
  double J0[kTrialSteps];
  sweep_objectives<N0>(o0, 0, ls_max, md, J0);
  st.J0t = J0[0];
  st.slope = o0[N0 + 6];
  st.maxd = o0[N0 + 7];
  st.ssqd = o0[N0 + 8];
  if (q == 0) {
#pragma unroll
    for (int s = 0; s < kTrialSteps; ++s) st.Jt[s] = s < N0 ? J0[s] : 0.0;
  } else {
    double o1[N1 + 9];
    reduce_partials_in<N1 + 9>(rb.region(trial_region(q)), nb,
                               1u << (N1 + 7), o1, lds);
    sweep_objectives<N1>(o1, q, ls_max, md, st.Jt);
  }
  return st;
}

// Armijo test J(t) <= J(0) + c1 t g.delta over the steps of sweep q in
// order: the first accepted step's index (and its objective), or -1.
__device__ __forceinline__ int sweep_decision(const SweepTotals& st, int q,
                                              int ls_max, double c1,
                                              double& Jacc) {
  const int ns = sweep_steps(q);
  int acc = -1;
  // unrolled with constant indices: the totals stay in registers
#pragma unroll
  for (int s = 0; s < kTrialSteps; ++s) {
    const double t = sweep_t(q, s, ls_max);
    if (acc < 0 && s < ns && sweep_tests(q, s, ls_max) &&
        st.Jt[s] <= st.J0t + c1 * t * st.slope) {
      acc = s;
      Jacc = st.Jt[s];
    }
  }
  return acc;
}

__device__ __forceinline__ int sweep_accepts(RedBuf rb, int nb, int q,
                                             int ls_max, double c1,
                                             const Model& md, double& Jacc,
                                             double* lds) {
  const SweepTotals st = sweep_totals(rb, nb, q, ls_max, md, lds);
  return sweep_decision(st, q, ls_max, c1, Jacc);
}

// Objective at u + t delta for the NT steps of line-search sweep `sweep`
// (sweep 0: t = 0 and t = 1, one dependent round of gathers per image
// frame).  The data term per voxel is sum (W - c)^2 - (sum (W - c))^2 / |K|
// with c the voxel's value in the first frame of K (a shift against
// cancellation); S and P are quadratic in t and are expanded exactly.  The
// per-step sums live in LDS (one slot row per thread), which keeps register
// use low.  A frame's loads (u, delta, g and both stencils) issue together,
// and in 2-D the gathers of up to three steps at a time, so that an image
// frame of a later sweep costs four dependent memory round trips instead of
// ten.
template <int D, int REG, int NT>
__device__ __forceinline__ void trial_body(
    const float* __restrict__ T, const float* __restrict__ u,
    const float* __restrict__ dl, const float* __restrict__ gr,
    const int* __restrict__ K, const Geom& g, const Model& md, int sweep,
    int ls_max, double c1, RedBuf rb, int nb, int gn_it,
    const Scal* __restrict__ sc, GNLog* __restrict__ log, Blk blk) {
  constexpr int NV = 2 * NT + 2 * D;
  __shared__ double xs[D == 2 ? 8 : 4][kWave][NV];
  if (gn_it >= sc->gn_stop) return;
  if constexpr (NT == kTrialSteps) {
    // a sweep >= 1 runs only after its predecessor ran and accepted no step
    static_assert(sizeof(xs) / sizeof(double) >= kSweepLds, "LDS");
    if (sweep >= 2 && log[gn_it].next_pass < sweep - 1) return;
    double Jacc;
    if (sweep_accepts(rb, nb, sweep - 1, ls_max, c1, md, Jacc,
                      &xs[0][0][0]) >= 0)
      return;
    if (blk.id == 0 && threadIdx.x == 0) log[gn_it].next_pass = sweep;
  }
  double* __restrict__ part = rb.region(trial_region(sweep));
  const int lane = threadIdx.x & (kWave - 1);
  const int w = wave_id();
  const int G = blockDim.x / kWave;
  const Chunk ch = frame_chunk(md.nK);
  const long long N = g.N;
  const long long ntiles = (N + kWave - 1) / kWave;
  double* my = xs[w][lane];
  double accD[NT];
#pragma unroll
  for (int s = 0; s < NT; ++s) accD[s] = 0.0;
  double rA = 0, rB = 0, rC = 0, pA = 0, pB = 0, pC = 0, slope = 0, mx = 0,
         sq = 0;
  for (int it = 0;; ++it) {
    long long tile = xcd_tile(ntiles, it, blk);
    if (tile < 0) break;
    tile = stencil_tile<D>(g, tile);
    long long x = tile * kWave + lane;
    bool valid = x < N;
    Pos<D> p = make_pos<D>(g, valid ? x : N - 1);
    const double c = (double)T[(size_t)K[0] * N + p.idx];
    for (int v = 0; v < NV; ++v) my[v] = 0.0;
    for (int j = ch.j0; j < ch.j1; ++j) {
      int k = K[j];
      double uv[D], dv[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        uv[a] = (double)u[((size_t)k * D + a) * N + p.idx];
        size_t o = ((size_t)j * D + a) * N + p.idx;
        dv[a] = (double)dl[o];
        my[2 * NT + a] += uv[a];
        my[2 * NT + D + a] += dv[a];
        // every lane loads (a lane past the end at the clamped last voxel),
        // so that the loads issue together; only valid lanes count
        const double gv = (double)gr[o];
        double uu, uw, ww;
        reg_cross<D, REG>(u + ((size_t)k * D + a) * N,
                          dl + ((size_t)j * D + a) * N, p, g, uu, uw, ww);
        slope = valid ? slope + gv * dv[a] : slope;
        mx = valid ? fmax(mx, fabs(dv[a])) : mx;
        sq = valid ? sq + dv[a] * dv[a] : sq;
        rA = valid ? rA + uu : rA;
        rB = valid ? rB + uw : rB;
        rC = valid ? rC + ww : rC;
      }
      const float* Tk = T + (size_t)k * N;
      // steps whose loads issue together: three in a later image sweep;
      // one at a time in the two-step image sweep (two in flight measured
      // slower under the register cap); both steps of the two-step volume
      // sweep (no register cap), one at a time in a later one
      constexpr int TG = D == 2 ? (NT < 3 ? 1 : 3) : (NT < 3 ? NT : 1);
#pragma unroll 1
      for (int s0 = 0; s0 < NT; s0 += TG) {
        double wvs[TG];
#pragma unroll
        for (int kk = 0; kk < TG; ++kk) {
          const int s = s0 + kk < NT ? s0 + kk : NT - 1;
          const double ts = sweep_t(sweep, s, ls_max);
          double ut[D];
#pragma unroll
          for (int a = 0; a < D; ++a) ut[a] = uv[a] + ts * dv[a];
          wvs[kk] = warp_value<D>(Tk, g, p, ut) - c;
        }
#pragma unroll
        for (int kk = 0; kk < TG; ++kk) {
          if (s0 + kk < NT) {
            my[s0 + kk] += wvs[kk];
            my[NT + s0 + kk] += wvs[kk] * wvs[kk];
          }
        }
      }
    }
    __syncthreads();
    if (w == 0 && valid) {
      double t1[NT], t2[NT], tu[D], tl[D];
#pragma unroll
      for (int s = 0; s < NT; ++s) t1[s] = t2[s] = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) tu[a] = tl[a] = 0.0;
      for (int cw = 0; cw < G; ++cw) {
#pragma unroll
        for (int s = 0; s < NT; ++s) {
          t1[s] += xs[cw][lane][s];
          t2[s] += xs[cw][lane][NT + s];
        }
#pragma unroll
        for (int a = 0; a < D; ++a) {
          tu[a] += xs[cw][lane][2 * NT + a];
          tl[a] += xs[cw][lane][2 * NT + D + a];
        }
      }
#pragma unroll
      for (int s = 0; s < NT; ++s) accD[s] += t2[s] - t1[s] * t1[s] * md.inv_nK;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double ub = tu[a] * md.inv_nK, lb = tl[a] * md.inv_nK;
        pA += ub * ub;
        pB += ub * lb;
        pC += lb * lb;
      }
    }
    __syncthreads();
  }
  double vals[NT + 9];
#pragma unroll
  for (int s = 0; s < NT; ++s) vals[s] = accD[s];
  vals[NT + 0] = rA;
  vals[NT + 1] = rB;
  vals[NT + 2] = rC;
  vals[NT + 3] = pA;
  vals[NT + 4] = pB;
  vals[NT + 5] = pC;
  vals[NT + 6] = slope;
  vals[NT + 7] = mx;
  vals[NT + 8] = sq;
  block_partials<NT + 9>(vals, 1u << (NT + 7), part, blk);
}

// Two 8-wave blocks per compute unit in 2-D: at most 128 registers.
template <int D, int REG, int NT>
__global__ __launch_bounds__(D == 2 ? 512 : 256, D == 2 ? 4 : 1) void trial_kernel(
    const float* __restrict__ T, const float* __restrict__ u,
    const float* __restrict__ dl, const float* __restrict__ gr,
    const int* __restrict__ K, Geom g, Model md, int p, int ls_max, double c1,
    RedBuf rb, int nb, int gn_it, const Scal* __restrict__ sc,
    GNLog* __restrict__ log) {
  trial_body<D, REG, NT>(T, u, dl, gr, K, g, md, p, ls_max, c1, rb, nb, gn_it,
                         sc, log, grid_blk());
}

// Armijo decision after the sweeps and, if a step passes, u[K[j]] +=
// t delta_j.  The last sweep that ran is the one whose predecessors all
// failed; every block totals its partials (and those of sweep 0) itself
// and so takes the same decision from the same values; block 0 records
// them.  The flag a later block of this kernel might read (gn_stop) is only
// written in a way that leaves such a block's work unchanged; each block
// reads it once, so that its threads agree.
__device__ __forceinline__ void ls_accept_body(
    float* __restrict__ u, const float* __restrict__ dl,
    const int* __restrict__ K, int nK, int dim, long long N, int ls_max,
    double c1, int fixed, double tol_J, double tol_u, RedBuf rb, int tnb,
    const Model& md, int gn_it, Scal* __restrict__ sc,
    GNLog* __restrict__ log, Blk blk) {
  __shared__ int skip, q;
  __shared__ double lds[kSweepLds];
  GNLog* L = log + gn_it;
  if (threadIdx.x == 0) {
    skip = gn_it >= sc->gn_stop;
    q = L->next_pass;
  }
  __syncthreads();
  if (skip) return;
  const int qs = q;
  const SweepTotals st = sweep_totals(rb, tnb, qs, ls_max, md, lds);
  double Jacc = 0.0;
  const int sacc = sweep_decision(st, qs, ls_max, c1, Jacc);
  if (blk.id == 0 && threadIdx.x == 0) {
    L->J0t = st.J0t;
    L->slope = st.slope;
    L->maxd = st.maxd;
    L->ssqd = st.ssqd;
  }
  if (sacc < 0) {
    // the last sweep failed too: no step
    if (blk.id == 0 && threadIdx.x == 0) {
      L->status = 1;
      L->t = 0.0;
      L->cg = sc->iters;
      sc->gn_stop = gn_it;
    }
    return;
  }
  const double tacc = sweep_t(qs, sacc, ls_max);
  // |K| D N < 2^31 (a context checks it): 32-bit index arithmetic, whose
  // divisions cost a fraction of 64-bit ones
  const unsigned DN = (unsigned)dim * (unsigned)N;
  const size_t count = (size_t)nK * DN;
  const unsigned stride = (unsigned)blk.n * blockDim.x;
  // element e = j DN + i of delta (frame j of K), (j, i) advanced by the
  // stride without a division.  K is read from LDS, and in the passes where
  // all four of a thread's elements exist their loads issue together with
  // no branch between them; the rest go one at a time.
  __shared__ int Ks[kMaxFrames];
  for (int t = threadIdx.x; t < nK; t += blockDim.x) Ks[t] = K[t];
  __syncthreads();
  unsigned e = (unsigned)blk.id * blockDim.x + threadIdx.x;
  unsigned j = e / DN, i = e - (e / DN) * DN;
  constexpr int kU = 4;
  auto advance = [&]() {
    e += stride;
    i += stride;
    while (i >= DN && j < (unsigned)nK) {
      i -= DN;
      ++j;
    }
  };
  while (e + (kU - 1) * stride < count) {
    size_t o[kU], d[kU];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      o[k] = (size_t)Ks[j] * DN + i;
      d[k] = e;
      advance();
    }
    float uv[kU], dv[kU];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      uv[k] = u[o[k]];
      dv[k] = dl[d[k]];
    }
#pragma unroll
    for (int k = 0; k < kU; ++k)
      u[o[k]] = (float)((double)uv[k] + tacc * (double)dv[k]);
  }
  while (e < count) {
    const size_t o = (size_t)Ks[j] * DN + i;
    u[o] = (float)((double)u[o] + tacc * (double)dl[e]);
    advance();
  }
  if (blk.id == 0 && threadIdx.x == 0) {
    bool breakdown = sc->done == 2;
    L->t = tacc;
    L->Jacc = Jacc;
    L->cg = sc->iters;
    L->status = breakdown ? 2 : 0;
    const double rms = sqrt(st.ssqd / (double)count);
    bool stop = breakdown ||
                (!fixed && (((L->J - Jacc) <= tol_J * fabs(L->J) &&
                             tacc * rms <= tol_u) ||
                            Jacc <= sc->J_target));
    if (stop) sc->gn_stop = gn_it + 1;
  }
}

__global__ __launch_bounds__(256) void ls_accept_kernel(
    float* __restrict__ u, const float* __restrict__ dl,
    const int* __restrict__ K, int nK, int dim, long long N, int ls_max,
    double c1, int fixed, double tol_J, double tol_u, RedBuf rb, int tnb,
    Model md, int gn_it, Scal* __restrict__ sc, GNLog* __restrict__ log) {
  ls_accept_body(u, dl, K, nK, dim, N, ls_max, c1, fixed, tol_J, tol_u, rb,
                 tnb, md, gn_it, sc, log, grid_blk());
}

// Start of a registration: every Gauss-Newton iteration enabled, logs
// cleared.
__global__ void gn_reset_kernel(Scal* __restrict__ sc,
                                GNLog* __restrict__ log, int n,
                                double J_target) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    GNLog L = {};
    L.status = -1;
    L.next_pass = 0;
    log[i] = L;
  }
  if (i == 0) {
    sc->gn_stop = 0x7fffffff;
    sc->done = 0;
    sc->gn_cur = 0;
    sc->J_target = J_target;
  }
}

// One block: objective only (no CG start) and v.Hv of the test entry.
__global__ __launch_bounds__(256) void finalize_eval_kernel(
    const double* __restrict__ ev_part, int ev_nb, Model md,
    Scal* __restrict__ sc) {
  double e[3];
  reduce_partials<3>(ev_part, ev_nb, 0u, e);
  if (threadIdx.x == 0) {
    double Dv = md.hd * e[0];
    double Sv = md.half_alpha_hd * md.reg_scale * e[1];
    double Pv = md.lam_hd * e[2];
    sc->D = Dv;
    sc->S = Sv;
    sc->P = Pv;
    sc->J = Dv + Sv + Pv;
  }
}

__global__ __launch_bounds__(256) void finalize_vhv_kernel(
    const double* __restrict__ part, int nb, Scal* __restrict__ sc) {
  double t[1];
  reduce_partials<1>(part, nb, 0u, t);
  if (threadIdx.x == 0) sc->vHv = t[0];
}

// Linear temporal interpolation of all frames from the frames of K_q.
__global__ void linear_predict_kernel(const float* Y, float* __restrict__ Z,
                                      float* Yout, LinTab tab,
                                      int n, int dim, long long N) {
  size_t per = (size_t)dim * N;
  size_t count = (size_t)n * per;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += stride) {
    int k = (int)(e / per);
    size_t off = e - (size_t)k * per;
    int l = tab.left[k], r = tab.right[k];
    double v = tab.wl[k] * (double)Y[(size_t)l * per + off] +
               tab.wr[k] * (double)Y[(size_t)r * per + off];
    float fv = (float)v;
    Z[e] = fv;
    if (l != k || r != k) Yout[e] = fv;
  }
}

// Eq. (2) for every (component, voxel): zeta = omega + xi with
// (M + beta D^T D) xi = M (eta - omega); Thomas sweep with the shared
// factorisation, d' kept in LDS (64 systems per block).
__global__ __launch_bounds__(64) void ls_predict_kernel(
    float* __restrict__ Y, float* __restrict__ Z, ThomasTab tab, int n,
    int dim, long long N, double beta) {
  extern __shared__ double dp[];   // [n][blockDim.x]
  const int B = blockDim.x;
  const size_t per = (size_t)dim * N;
  const size_t sys = (size_t)blockIdx.x * B + threadIdx.x;
  const bool valid = sys < per;
  double prev = 0.0;
  // unrolled, so that the loads of several frames are in flight (only the
  // recurrence is sequential)
#pragma unroll 8
  for (int k = 0; k < n; ++k) {
    double rhs = 0.0;
    if (valid && tab.mask[k]) {
      size_t o = (size_t)k * per + sys;
      rhs = (double)Y[o] - (double)Z[o];
    }
    prev = (rhs + beta * prev) * tab.invp[k];
    dp[k * B + threadIdx.x] = prev;
  }
  double xi = 0.0;
#pragma unroll 8
  for (int k = n - 1; k >= 0; --k) {
    xi = (k == n - 1) ? dp[k * B + threadIdx.x]
                      : dp[k * B + threadIdx.x] - tab.cp[k] * xi;
    if (valid) {
      size_t o = (size_t)k * per + sys;
      float zv = (float)((double)Z[o] + xi);
      Z[o] = zv;
      Y[o] = zv;
    }
  }
}

// The same sweep for a sequence of exactly NF frames with d' in registers
// (fully unrolled): the LDS form holds n doubles per system and so admits
// few waves per compute unit; this one is limited by registers only.  Same
// arithmetic in the same order.
template <int NF>
__global__ __launch_bounds__(64) void ls_predict_reg_kernel(
    float* __restrict__ Y, float* __restrict__ Z, ThomasTab tab, int dim,
    long long N, double beta) {
  const size_t per = (size_t)dim * N;
  const size_t sys = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = sys < per;
  double dp[NF];
  double prev = 0.0;
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    double rhs = 0.0;
    if (valid && tab.mask[k]) {
      size_t o = (size_t)k * per + sys;
      rhs = (double)Y[o] - (double)Z[o];
    }
    prev = (rhs + beta * prev) * tab.invp[k];
    dp[k] = prev;
  }
  double xi = 0.0;
#pragma unroll
  for (int k = NF - 1; k >= 0; --k) {
    xi = (k == NF - 1) ? dp[k] : dp[k] - tab.cp[k] * xi;
    if (valid) {
      size_t o = (size_t)k * per + sys;
      float zv = (float)((double)Z[o] + xi);
      Z[o] = zv;
      Y[o] = zv;
    }
  }
}

// ------------------------------------------------------ batched iteration

// Problem of block b: the j with first[j] <= b < first[j + 1].
__device__ __forceinline__ int job_index(const int* __restrict__ f, int n,
                                         int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (f[mid] <= b) lo = mid;
    else hi = mid;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// This block's problem in kernel class c and its block context there.
__device__ __forceinline__ const Job& job_of(const JobSet& js, int c,
                                             Blk& blk) {
  const int* f = js.first + (size_t)c * (js.n + 1);
  const int b = blockIdx.x;
  const int j = job_index(f, js.n, b);
  blk = Blk{b - f[j], f[j + 1] - f[j]};
  return js.jobs[j];
}

template <int D, int REG>
__global__ __launch_bounds__(D == 2 ? 512 : 256, D == 2 ? 4 : 1) void eval_batch_kernel(
    JobSet js) {
  Blk blk;
  const Job& J = job_of(js, kClsTile, blk);
  const Geom g = J.g;
  const Model md = J.md;
  Scal* sc = J.sc;
  eval_body<D, REG, true>(J.T, J.u, J.K, g, md, J.grad, J.dW,
                          J.rb.region(kRegEval), sc->gn_cur, sc,
                          CgStart{J.r, J.z, J.sums.Sz, J.sums.Vz}, blk);
}

__global__ __launch_bounds__(256) void start_batch_kernel(JobSet js) {
  const Job& J = js.jobs[blockIdx.x];
  const Model md = J.md;
  Scal* sc = J.sc;
  finalize_start_body(J.rb.region(kRegEval), J.nb_tile, md, sc, sc->gn_cur,
                      J.log);
}

template <int D, int REG, int NT>
__global__ __launch_bounds__(D == 2 ? 512 : 256, D == 2 ? 4 : 1) void trial_batch_kernel(
    JobSet js, int p, int ls_max, double c1) {
  Blk blk;
  const Job& J = job_of(js, kClsTile, blk);
  const Geom g = J.g;
  const Model md = J.md;
  Scal* sc = J.sc;
  trial_body<D, REG, NT>(J.T, J.u, J.x, J.grad, J.K, g, md, p, ls_max, c1,
                         J.rb, J.nb_tile, sc->gn_cur, sc, J.log, blk);
}

__global__ __launch_bounds__(256) void accept_batch_kernel(
    JobSet js, int ls_max, double c1, int fixed, double tol_J, double tol_u) {
  Blk blk;
  const Job& J = job_of(js, kClsElem, blk);
  Scal* sc = J.sc;
  const Model md = J.md;
  ls_accept_body(J.u, J.x, J.K, md.nK, geom_dim(J.g), J.g.N, ls_max, c1,
                 fixed, tol_J, tol_u, J.rb, J.nb_tile, md, sc->gn_cur, sc,
                 J.log, blk);
}

// Start of a batched registration: per problem, every iteration enabled,
// logs cleared, iteration counter 0.
__global__ __launch_bounds__(256) void reset_batch_kernel(JobSet js,
                                                          int gn_max) {
  const Job& J = js.jobs[blockIdx.x];
  for (int i = threadIdx.x; i < gn_max; i += blockDim.x) {
    GNLog L = {};
    L.status = -1;
    L.next_pass = 0;
    J.log[i] = L;
  }
  if (threadIdx.x == 0) {
    J.sc->gn_stop = 0x7fffffff;
    J.sc->done = 0;
    J.sc->gn_cur = 0;
    J.sc->J_target = -INFINITY;
  }
}

// End of a batched iteration: stop flag per problem, counter advanced.
__global__ void advance_batch_kernel(JobSet js, int* __restrict__ stop) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= js.n) return;
  Scal* sc = js.jobs[j].sc;
  const int it = sc->gn_cur;
  stop[j] = sc->gn_stop <= it + 1 ? 1 : 0;
  sc->gn_cur = it + 1;
}

int elem_grid(long long count) { return elem_blocks((size_t)count); }

hipError_t batch_gn_reset(const JobSet& js, int gn_max, hipStream_t s) {
  reset_batch_kernel<<<js.n, 256, 0, s>>>(js, gn_max);
  return hipGetLastError();
}

hipError_t batch_eval(const JobSet& js, int nblocks, int dim, int reg,
                      hipStream_t s) {
  STML_TILE_DISPATCH(dim, reg, eval_batch_kernel, nblocks,
                     eval_threads(dim, 0), s, js);
  return hipGetLastError();
}

hipError_t batch_finalize_start(const JobSet& js, hipStream_t s) {
  start_batch_kernel<<<js.n, 256, 0, s>>>(js);
  return hipGetLastError();
}

// (dimension, regulariser, steps of the sweep) specialisations of the
// trial sweep kernels.
#define STML_TRIAL_DISPATCH(dim, reg, p, KERNEL, GRID, BLOCK, STREAM, ...)   \
  do {                                                                    \
    if ((p) == 0)                                                         \
      STML_TRIAL_DISPATCH_NT(dim, reg, kSweep0Steps, KERNEL, GRID, BLOCK, \
                             STREAM, __VA_ARGS__);                        \
    else                                                                  \
      STML_TRIAL_DISPATCH_NT(dim, reg, kTrialSteps, KERNEL, GRID, BLOCK,  \
                             STREAM, __VA_ARGS__);                        \
  } while (0)
#define STML_TRIAL_DISPATCH_NT(dim, reg, NT, KERNEL, GRID, BLOCK, STREAM, ...) \
  do {                                                                    \
    if ((dim) == 2 && (reg) == 0)                                         \
      KERNEL<2, 0, NT><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);          \
    else if ((dim) == 2)                                                  \
      KERNEL<2, 1, NT><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);          \
    else if ((reg) == 0)                                                  \
      KERNEL<3, 0, NT><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);          \
    else                                                                  \
      KERNEL<3, 1, NT><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);          \
  } while (0)

hipError_t batch_trial(const JobSet& js, int ntile, int dim, int reg, int p,
                       int ls_max, double c1, hipStream_t s) {
  STML_TRIAL_DISPATCH(dim, reg, p, trial_batch_kernel, ntile,
                      tile_threads(dim, 0), s, js, p, ls_max, c1);
  return hipGetLastError();
}

hipError_t batch_accept(const JobSet& js, int nelem, int ls_max, double c1,
                        int fixed, double tol_J, double tol_u,
                        hipStream_t s) {
  accept_batch_kernel<<<nelem, 256, 0, s>>>(js, ls_max, c1, fixed, tol_J,
                                            tol_u);
  return hipGetLastError();
}

hipError_t batch_advance(const JobSet& js, int* stop_out, hipStream_t s) {
  advance_batch_kernel<<<(js.n + 63) / 64, 64, 0, s>>>(js, stop_out);
  return hipGetLastError();
}

// ------------------------------------------------------------- launchers

hipError_t launch_fill(float* p, size_t count, float v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  fill_kernel<<<elem_blocks(count), 256, 0, s>>>(p, count, v);
  return hipGetLastError();
}

hipError_t launch_check_finite(const float* p, size_t count, Scal* sc,
                               hipStream_t s) {
  check_finite_kernel<<<elem_blocks(count), 256, 0, s>>>(p, count, sc);
  return hipGetLastError();
}

hipError_t launch_restrict(int dim, const float* fine, float* coarse, int n,
                           const Geom& gf, const Geom& gc, hipStream_t s) {
  int nb = elem_blocks((size_t)n * gc.N, 1);
  if (dim == 2)
    restrict_kernel<2><<<nb, 256, 0, s>>>(fine, coarse, n, gf, gc);
  else
    restrict_kernel<3><<<nb, 256, 0, s>>>(fine, coarse, n, gf, gc);
  return hipGetLastError();
}

hipError_t launch_prolong(int dim, const float* coarse, float* fine,
                          int fields, const Geom& gc, const Geom& gf,
                          hipStream_t s) {
  const int nb = elem_blocks((size_t)gf.N, 1);
  // about 4096 blocks in all, each field group at least one
  int fy = (4096 + nb - 1) / nb;
  if (fy > fields) fy = fields;
  if (fy < 1) fy = 1;
  const dim3 grid(nb, fy);
  if (dim == 2)
    prolong_kernel<2><<<grid, 256, 0, s>>>(coarse, fine, fields, gc, gf);
  else
    prolong_kernel<3><<<grid, 256, 0, s>>>(coarse, fine, fields, gc, gf);
  return hipGetLastError();
}

hipError_t launch_linear_predict(const float* Y, float* Z, float* Yout,
                                 LinTab tab, int n, int dim, long long N,
                                 hipStream_t s) {
  size_t count = (size_t)n * dim * N;
  linear_predict_kernel<<<elem_blocks(count), 256, 0, s>>>(Y, Z, Yout, tab, n,
                                                           dim, N);
  return hipGetLastError();
}

hipError_t launch_ls_predict(float* Y, float* Z, ThomasTab tab, int n,
                             int dim, long long N, double beta,
                             hipStream_t s) {
  size_t systems = (size_t)dim * N;
  if (n == 64 || n == 32) {
    // d' in registers (the frame counts of the image and volume workloads)
    const int nb = (int)((systems + 63) / 64);
    if (n == 64)
      ls_predict_reg_kernel<64><<<nb, 64, 0, s>>>(Y, Z, tab, dim, N, beta);
    else
      ls_predict_reg_kernel<32><<<nb, 64, 0, s>>>(Y, Z, tab, dim, N, beta);
    return hipGetLastError();
  }
  // d' of every system stays in LDS: n * B doubles <= 64 KiB.
  int B = n <= 128 ? 64 : 32;
  int nb = (int)((systems + B - 1) / B);
  size_t lds = (size_t)n * B * sizeof(double);
  ls_predict_kernel<<<nb, B, lds, s>>>(Y, Z, tab, n, dim, N, beta);
  return hipGetLastError();
}

hipError_t launch_eval(int dim, const float* T, const float* u, const int* K,
                       const Geom& g, const Model& md, float* grad,
                       float* dW, RedBuf rb, Scal* sc, hipStream_t s,
                       bool finalize, int gn_it, const CgStart* cs) {
  int nb = tile_blocks(g), nt = eval_threads(dim, md.nK);
  double* part = rb.region(kRegEval);
  const Scal* gate = finalize ? nullptr : sc;
  if (cs && !grad) return hipErrorInvalidValue;
  const CgStart none{nullptr, nullptr, nullptr, nullptr};
  const CgStart c0 = cs ? *cs : none;
  decltype(&eval_kernel<2, 0, false>) kern;
  // images on grids of at most one block per compute unit: the paired form
  // (the same results)
  if (dim == 2 && nb <= kCUs)
    kern = md.reg == 0
               ? (cs ? eval_kernel<2, 0, true, true>
                     : eval_kernel<2, 0, false, true>)
               : (cs ? eval_kernel<2, 1, true, true>
                     : eval_kernel<2, 1, false, true>);
  else if (dim == 2)
    kern = md.reg == 0 ? (cs ? eval_kernel<2, 0, true> : eval_kernel<2, 0, false>)
                       : (cs ? eval_kernel<2, 1, true> : eval_kernel<2, 1, false>);
  else
    kern = md.reg == 0 ? (cs ? eval_kernel<3, 0, true> : eval_kernel<3, 0, false>)
                       : (cs ? eval_kernel<3, 1, true> : eval_kernel<3, 1, false>);
  kern<<<nb, nt, 0, s>>>(T, u, K, g, md, grad, dW, part, gn_it, gate, c0);
  if (finalize)
    finalize_eval_kernel<<<1, 256, 0, s>>>(part, nb, md, sc);
  return hipGetLastError();
}

hipError_t launch_trial(int dim, const float* T, const float* u,
                        const float* delta, const float* grad, const int* K,
                        const Geom& g, const Model& md, int p, int ls_max,
                        double c1, RedBuf rb, Scal* sc, hipStream_t s,
                        int gn_it, GNLog* log) {
  int nb = tile_blocks(g);
  int nt = tile_threads(dim, md.nK);
  STML_TRIAL_DISPATCH(dim, md.reg, p, trial_kernel, nb, nt, s, T, u, delta,
                      grad, K, g, md, p, ls_max, c1, rb, nb, gn_it, sc, log);
  return hipGetLastError();
}

hipError_t launch_ls_accept(float* u, const float* delta, const int* K,
                            const Geom& g, const Model& md, int ls_max,
                            double c1, int fixed, double tol_J, double tol_u,
                            RedBuf rb, int gn_it, Scal* sc, GNLog* log,
                            hipStream_t s) {
  const int dim = geom_dim(g);
  size_t count = (size_t)md.nK * dim * g.N;
  ls_accept_kernel<<<elem_blocks(count), 256, 0, s>>>(
      u, delta, K, md.nK, dim, g.N, ls_max, c1, fixed, tol_J, tol_u, rb,
      tile_blocks(g), md, gn_it, sc, log);
  return hipGetLastError();
}

hipError_t launch_finalize_start(RedBuf rb, int ev_nb, const Model& md,
                                 Scal* sc, int gn_it, GNLog* log,
                                 hipStream_t s) {
  finalize_start_kernel<<<1, 256, 0, s>>>(rb.region(kRegEval), ev_nb, md, sc,
                                          gn_it, log);
  return hipGetLastError();
}

hipError_t launch_finalize_vhv(const double* part, int nb, Scal* sc,
                               hipStream_t s) {
  finalize_vhv_kernel<<<1, 256, 0, s>>>(part, nb, sc);
  return hipGetLastError();
}

hipError_t launch_gn_reset(Scal* sc, GNLog* log, int n, hipStream_t s,
                           double J_target) {
  int nb = (n + 255) / 256;
  gn_reset_kernel<<<nb < 1 ? 1 : nb, 256, 0, s>>>(sc, log, n, J_target);
  return hipGetLastError();
}

}  // namespace stml
