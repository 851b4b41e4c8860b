// Affine-linear groupwise registration with the correlation-based SqN
// distance and L-BFGS: the paper's experimental model (Sec. 2, eq. (1);
// Sec. 4).
//
// Frame k moves by u_k(x) = B_k xi(x) + b_k, xi(x) = (x - c) / R (c the
// centre of the finest grid, R half its largest side), so the parameters
// theta_k = (B_k row-major, b_k) are pixels and mean the same map on every
// level.  The distance is the pair sum of eq. (1) with 1 - rho_ij^2:
//     D = sum_{i,j in K} (1 - rho_ij^2),   rho_ij = C_ij / (s_i s_j),
// C the covariance of the warped frames over the grid and s_i = sqrt(C_ii)
// (the Schatten 4-norm SqN measure of the centred, normalised frames), plus
// the penalty P = lambda h^d sum_x |mean_k u_k(x)|^2.
//
// One evaluation is three passes over the voxels:
//   gram   : warp every frame of K, stage the warped values of 32 voxels
//            (and a row of ones) in LDS, and accumulate the raw Gram matrix
//            sum_x W_i W_j (its ones row gives sum_x W_i and N) in 16 x 16
//            float64 tiles on the matrix cores; one partial per block;
//   (sum, finalize: totals in block order; covariance, rho, D, P, and the
//            coefficients Rc of dD/dW_i = sum_b Rc_ib (W_b - mu_b))
//   resid  : r_i(x) = sum_b Rc_ib (W_b(x) - mu_b) from the warped frames
//            pass 1 kept (float32), as a GEMM on the matrix cores, stored
//            float32 [|K|][N];
//   pgrad  : per frame, sum_x r_i(x) dW_i/du(x) (xi(x), 1) -> the p
//            parameter partials per block; summed in block order together
//            with the penalty's gradient.
// The line search needs only the first pass.  L-BFGS (two-loop recursion),
// the Armijo decision and the pair update run in single-block kernels on
// the device; all sums are in fixed order, so repeated runs agree bit for
// bit.
#include <hip/hip_runtime.h>

#include "../../include/stml.h"
#include "launch.h"
#include "reduce.h"

namespace stml {

constexpr int kAffV = 32;          // voxels per staged tile
constexpr int kAffThreads = 256;
constexpr int kAffMaxP = 12;

__device__ __forceinline__ int aff_tri_index(int r, int c, int K1) {
  return r * K1 - (r * (r - 1)) / 2 + (c - r);
}

template <int D>
__device__ __forceinline__ void aff_xi(const AffGeom& ag, const Pos<D>& pos,
                                       double* xi) {
#pragma unroll
  for (int e = 0; e < D; ++e)
    xi[e] = (((double)pos.c[e] + 0.5) * ag.h - ag.c[e]) * ag.inv_R;
}

// Warped value (and dW/du) of frame plane T at voxel pos for parameters th.
template <int D>
__device__ __forceinline__ void aff_warp(const float* __restrict__ T,
                                         const AffGeom& ag, const Pos<D>& pos,
                                         const double* th, double& W,
                                         double* dW) {
  double xi[D], uv[D];
  aff_xi<D>(ag, pos, xi);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < D; ++e) s += th[a * D + e] * xi[e];
    uv[a] = s + th[D * D + a];
  }
  warp_sample<D>(T, ag.g, pos, uv, W, dW);
}

// Parameters of the frames of K at the trial point x + t d, into LDS.
__device__ __forceinline__ void aff_stage_params(const double* __restrict__ x,
                                                 const double* __restrict__ dv,
                                                 double t, int nP,
                                                 double* th) {
  for (int i = threadIdx.x; i < nP; i += blockDim.x)
    th[i] = dv ? x[i] + t * dv[i] : x[i];
}

// Voxel geometry of one tile (cell indices and xi), once per tile in LDS,
// so that the warps of the tile's frames do not redo the index division.
template <int D>
struct AffTileGeo {
  int c[D][kAffV];
  double xi[D][kAffV];
};

template <int D>
__device__ __forceinline__ void aff_tile_geo(const AffGeom& ag, long long v0,
                                             AffTileGeo<D>& tg) {
  if (threadIdx.x < kAffV) {
    const long long vox = v0 + threadIdx.x;
    Pos<D> pos = make_pos<D>(ag.g, vox < ag.g.N ? vox : ag.g.N - 1);
    double xi[D];
    aff_xi<D>(ag, pos, xi);
#pragma unroll
    for (int e = 0; e < D; ++e) {
      tg.c[e][threadIdx.x] = pos.c[e];
      tg.xi[e][threadIdx.x] = xi[e];
    }
  }
}

// Warped frames of one tile into Ws[row][kAffV + 1] (float64): rows of K,
// then (ones) a row of ones over the valid voxels; invalid voxels hold 0.
// Wout (optional) receives the warped values as float32 [|K|][N].  The
// tile's geometry must be in tg (and visible: after a barrier).
template <int D>
__device__ __forceinline__ void aff_stage_tile(
    const float* __restrict__ T, const int* __restrict__ K, int nk,
    bool ones, const AffGeom& ag, const double* th, const double* mu,
    long long v0, const AffTileGeo<D>& tg, double* Ws,
    float* __restrict__ Wout) {
  constexpr int P = D * D + D;
  const int rows = nk + (ones ? 1 : 0);
  const long long N = ag.g.N;
  for (int idx = threadIdx.x; idx < rows * kAffV; idx += blockDim.x) {
    const int k = idx / kAffV, v = idx - k * kAffV;
    const long long vox = v0 + v;
    double val = 0.0;
    if (vox < N) {
      if (k < nk) {
        Pos<D> pos;
        double xi[D], uv[D], dW[D];
#pragma unroll
        for (int e = 0; e < D; ++e) {
          pos.c[e] = tg.c[e][v];
          xi[e] = tg.xi[e][v];
        }
        const double* t = th + (size_t)k * P;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double s = 0.0;
#pragma unroll
          for (int e = 0; e < D; ++e) s += t[a * D + e] * xi[e];
          uv[a] = s + t[D * D + a];
        }
        warp_sample<D>(T + (size_t)K[k] * N, ag.g, pos, uv, val, dW);
        if (Wout) Wout[(size_t)k * N + vox] = (float)val;
        if (mu) val -= mu[k];
      } else {
        val = 1.0;
      }
    }
    Ws[k * (kAffV + 1) + v] = val;
  }
}

// Upper-triangle tile tau of a TI x TI tile grid -> (I, J), I <= J.
__device__ __forceinline__ void aff_tile_of(int tau, int TI, int& I, int& J) {
  I = 0;
  while (tau >= TI - I) {
    tau -= TI - I;
    ++I;
  }
  J = I + tau;
}

typedef double aff_d4 __attribute__((ext_vector_type(4)));

// Pass 1: raw Gram matrix G = A A^T of A = [W_K; 1] (rows padded with zeros
// to a multiple of 16) over this block's voxels, on the float64 matrix
// cores.  Per 32-voxel tile the warped rows are staged in LDS; the upper
// triangle of 16 x 16 output tiles is dealt round-robin to the block's
// four waves (blockIdx.y selects a group of kAffGramTiles tiles per wave
// when there are more), and each wave accumulates its tiles with
// v_mfma_f64_16x16x4f64 over the tile's voxels in steps of four: lane l
// supplies A[16 I + l % 16][v + l / 16] and A[16 J + l % 16][v + l / 16]
// and holds G[16 I + l / 16 + 4 r][16 J + l % 16] in register r.  The
// voxels are summed in a fixed order, so repeated runs agree bit for bit.
template <int D>
__global__ __launch_bounds__(kAffThreads) void aff_gram_kernel(
    const float* __restrict__ T, const int* __restrict__ K, int nk,
    const double* __restrict__ x, const double* __restrict__ dv, double t,
    AffGeom ag, double* __restrict__ part, int E, float* __restrict__ Wout) {
  extern __shared__ double lds[];
  __shared__ AffTileGeo<D> tg;
  constexpr int P = D * D + D;
  constexpr int MT = kAffGramTiles;
  const int K1 = nk + 1;
  const int Kt = (K1 + 15) / 16;
  const int NTt = Kt * (Kt + 1) / 2;
  double* th = lds;                                   // [nk][P]
  double* Ws = lds + ((nk * P + 1) & ~1);             // [16 Kt][kAffV + 1]
  aff_stage_params(x, dv, t, nk * P, th);
  for (int i = threadIdx.x + K1 * (kAffV + 1); i < 16 * Kt * (kAffV + 1);
       i += blockDim.x)
    Ws[i] = 0.0;                                      // padding rows
  const int w = wave_id();
  const int lane = threadIdx.x & (kWave - 1);
  const int r16 = lane & 15, k4 = lane >> 4;
  int ra[MT], rb[MT];                                 // LDS row offsets
  bool act[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int tau = (blockIdx.y * MT + m) * (kAffThreads / kWave) + w;
    act[m] = tau < NTt;
    int I = 0, J = 0;
    if (act[m]) aff_tile_of(tau, Kt, I, J);
    ra[m] = (16 * I + r16) * (kAffV + 1) + k4;
    rb[m] = (16 * J + r16) * (kAffV + 1) + k4;
  }
  aff_d4 acc[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) acc[m] = aff_d4{0.0, 0.0, 0.0, 0.0};
  const long long nch = (ag.g.N + kAffV - 1) / kAffV;
  for (long long ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    aff_tile_geo<D>(ag, ch * kAffV, tg);
    __syncthreads();
    // the first tile group also keeps the warped frames for pass 2
    aff_stage_tile<D>(T, K, nk, true, ag, th, nullptr, ch * kAffV, tg, Ws,
                      blockIdx.y == 0 ? Wout : nullptr);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kAffV; ks += 4) {
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        if (!act[m]) continue;          // wave-uniform
        const double a = Ws[ra[m] + ks];
        const double b = Ws[rb[m] + ks];
        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[m], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * E;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    if (!act[m]) continue;
    const int I = (ra[m] / (kAffV + 1) - r16) / 16;
    const int J = (rb[m] / (kAffV + 1) - r16) / 16;
    const int c = 16 * J + r16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // tiles with I < J lie above the diagonal; a diagonal tile keeps its
      // upper triangle (its mirror entries are the same sums)
      const int r = 16 * I + k4 + 4 * q;
      if (r < K1 && c < K1 && r <= c) out[aff_tri_index(r, c, K1)] = acc[m][q];
    }
  }
}

// Totals of E values over nb partials, in block order.
__global__ void aff_sum_kernel(const double* __restrict__ part, int nb,
                               int E, double* __restrict__ tot) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * E + e];
  tot[e] = s;
}

// Block-wide float64 sum in fixed order (every thread gets the total).
__device__ __forceinline__ double aff_block_sum(double v) {
  __shared__ double red[kAffThreads / kWave];
  __shared__ double total;
  v = wave_sum(v);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) s += red[i];
    total = s;
  }
  __syncthreads();
  double r = total;
  __syncthreads();
  return r;
}

__device__ __forceinline__ double aff_block_max(double v) {
  __shared__ double red[kAffThreads / kWave];
  __shared__ double total;
  v = wave_max(v);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = red[0];
    for (int i = 1; i < (int)(blockDim.x / kWave); ++i) s = fmax(s, red[i]);
    total = s;
  }
  __syncthreads();
  double r = total;
  __syncthreads();
  return r;
}

// Covariance, rho, D, the pass-2 coefficients, and the penalty with its
// gradient (closed form from the per-axis moments of xi over the grid).
__global__ __launch_bounds__(kAffThreads) void aff_finalize_kernel(
    const double* __restrict__ tot, int nk, AffGeom ag,
    const double* __restrict__ x, const double* __restrict__ dv, double t,
    double lam, AffScal* __restrict__ sc, double* __restrict__ mu,
    double* __restrict__ Rc, double* __restrict__ gpen, int grad) {
  __shared__ double s_sd[STML_MAX_FRAMES];
  __shared__ double s_mu[STML_MAX_FRAMES];
  __shared__ double tbar[kAffMaxP];
  __shared__ double mom1[3], mom2[3][3];
  const int d = ag.d, P = d * d + d;
  const int K1 = nk + 1;
  const double Nv = tot[aff_tri_index(nk, nk, K1)];
  int bad = 0;
  for (int i = threadIdx.x; i < nk; i += blockDim.x) {
    const double m = tot[aff_tri_index(i, nk, K1)] / Nv;
    const double c = tot[aff_tri_index(i, i, K1)] - Nv * m * m;
    s_mu[i] = m;
    s_sd[i] = c > 0.0 ? sqrt(c) : 0.0;
    if (!(c > 0.0)) bad = 1;
    if (mu) mu[i] = m;
  }
  __syncthreads();
  // rows: sum_b (1 - rho_ib^2) and G2_i = sum_b rho_ib^2
  double dsum = 0.0;
  for (int i = threadIdx.x; i < nk; i += blockDim.x) {
    double g2 = 0.0, row = 0.0;
    for (int b = 0; b < nk; ++b) {
      const int r = i < b ? i : b, c = i < b ? b : i;
      const double cov = tot[aff_tri_index(r, c, K1)] - Nv * s_mu[i] * s_mu[b];
      const double rho = cov / (s_sd[i] * s_sd[b]);
      row += 1.0 - rho * rho;
      g2 += rho * rho;
    }
    dsum += row;
    if (grad) {
      for (int b = 0; b < nk; ++b) {
        const int r = i < b ? i : b, c = i < b ? b : i;
        const double cov =
            tot[aff_tri_index(r, c, K1)] - Nv * s_mu[i] * s_mu[b];
        const double rho = cov / (s_sd[i] * s_sd[b]);
        Rc[(size_t)i * nk + b] =
            -4.0 * (rho - (i == b ? g2 : 0.0)) / (s_sd[i] * s_sd[b]);
      }
    }
  }
  const double Dv = aff_block_sum(dsum);
  const int any_bad = (int)aff_block_max((double)bad);
  // penalty: mean parameters over K at x + t d
  if (threadIdx.x < P) {
    double s = 0.0;
    for (int k = 0; k < nk; ++k) {
      const size_t o = (size_t)k * P + threadIdx.x;
      s += dv ? x[o] + t * dv[o] : x[o];
    }
    tbar[threadIdx.x] = s / nk;
  }
  // per-axis sums of xi and xi^2 over one axis' cells
  if (threadIdx.x < 32 && threadIdx.x / 2 < d) {
    const int a = threadIdx.x / 2;
    const bool sq = threadIdx.x & 1;
    double s = 0.0;
    for (int i = 0; i < ag.g.m[a]; ++i) {
      const double xi = (((double)i + 0.5) * ag.h - ag.c[a]) * ag.inv_R;
      s += sq ? xi * xi : xi;
    }
    if (sq) mom2[a][a] = s;
    else mom1[a] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double N = (double)ag.g.N;
    double m1[3], m2[3][3];
    for (int a = 0; a < d; ++a) m1[a] = mom1[a] * (N / ag.g.m[a]);
    for (int a = 0; a < d; ++a)
      for (int e = 0; e < d; ++e)
        m2[a][e] = a == e ? mom2[a][a] * (N / ag.g.m[a])
                          : mom1[a] * mom1[e] * (N / ((double)ag.g.m[a] *
                                                      ag.g.m[e]));
    const double lhd = lam * ag.hd;
    double pv = 0.0;
    for (int a = 0; a < d; ++a) {
      const double* Ba = tbar + a * d;
      const double ba = tbar[d * d + a];
      double quad = 0.0, lin = 0.0;
      for (int e = 0; e < d; ++e) {
        for (int f = 0; f < d; ++f) quad += Ba[e] * Ba[f] * m2[e][f];
        lin += Ba[e] * m1[e];
      }
      pv += quad + 2.0 * ba * lin + N * ba * ba;
      if (grad) {
        for (int e = 0; e < d; ++e) {
          double s = ba * m1[e];
          for (int f = 0; f < d; ++f) s += Ba[f] * m2[e][f];
          gpen[a * d + e] = 2.0 * lhd * s;
        }
        gpen[d * d + a] = 2.0 * lhd * (lin + N * ba);
      }
    }
    const double Pv = lhd * pv;
    sc->D = Dv;
    sc->P = Pv;
    sc->J = Dv + Pv;
    sc->bad = any_bad;
  }
}

// Pass 2: r_i(x) = sum_b Rc_ib (W_b(x) - mu_b) for the frames of K from the
// warped frames pass 1 stored (float32), as a GEMM on the float64 matrix
// cores.  A wave owns one 16-row tile I = blockIdx.y * (waves per block) +
// wave of the output and keeps its rows of Rc as MFMA operands in
// registers for the whole kernel (KS steps of four columns: lane l holds
// Rc[16 I + l % 16][4 s + l / 16] in a[s]); blocks of up to MAXT threads.
// Per 32-voxel tile the centred values are staged in LDS (rows padded with
// zeros to a multiple of 16) and each wave forms its two 16 x 16 output
// tiles (register q of lane l: r[16 I + l / 16 + 4 q][16 V + l % 16]).
template <int KS, int MAXT>
__global__ __launch_bounds__(MAXT) void aff_resid_kernel(
    const float* __restrict__ W, int nk, long long N,
    const double* __restrict__ mu, const double* __restrict__ Rc,
    float* __restrict__ r) {
  extern __shared__ double Ws[];                      // [16 Kt][kAffV + 1]
  constexpr int NV = kAffV / 16;
  const int Kt = (nk + 15) / 16;
  const int nks = 4 * Kt;                             // steps used (<= KS)
  const int I = blockIdx.y * (blockDim.x / kWave) + wave_id();
  const bool act = I < Kt;                            // wave-uniform
  const int lane = threadIdx.x & (kWave - 1);
  const int r16 = lane & 15, k4 = lane >> 4;
  for (int i = threadIdx.x + nk * (kAffV + 1); i < 16 * Kt * (kAffV + 1);
       i += blockDim.x)
    Ws[i] = 0.0;                                      // padding rows
  // rows past nk read row nk - 1 (their outputs are dropped); columns past
  // nk are zero
  const int row = min(16 * (act ? I : 0) + r16, nk - 1);
  double a[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int b = 4 * s + k4;
    a[s] = (s < nks && b < nk) ? Rc[(size_t)row * nk + b] : 0.0;
  }
  const long long nch = (N + kAffV - 1) / kAffV;
  for (long long ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < nk * kAffV; idx += blockDim.x) {
      const int b = idx / kAffV, v = idx - b * kAffV;
      const long long vox = ch * kAffV + v;
      Ws[b * (kAffV + 1) + v] =
          vox < N ? (double)W[(size_t)b * N + vox] - mu[b] : 0.0;
    }
    __syncthreads();
    aff_d4 acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = aff_d4{0.0, 0.0, 0.0, 0.0};
    if (!act) continue;                 // after the barriers of this tile
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      if (s < nks) {                    // block-uniform
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double bv = Ws[(4 * s + k4) * (kAffV + 1) + 16 * v + r16];
          acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bv, acc[v], 0,
                                                        0, 0);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const long long vox = ch * kAffV + 16 * v + r16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * I + k4 + 4 * q;
        if (i < nk && vox < N) r[(size_t)i * N + vox] = (float)acc[v][q];
      }
    }
  }
}

// Pass 3: per frame j of K (grid y), sum_x r_j(x) dW_j/du_a(x) xi_e(x) and
// sum_x r_j(x) dW_j/du_a(x) over this block's voxels; block partials.
template <int D>
__global__ __launch_bounds__(kAffThreads) void aff_pgrad_kernel(
    const float* __restrict__ T, const int* __restrict__ K,
    const double* __restrict__ x, const double* __restrict__ dv, double t,
    AffGeom ag, const float* __restrict__ r, double* __restrict__ part) {
  constexpr int P = D * D + D;
  const int j = blockIdx.y;
  double th[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const size_t o = (size_t)j * P + i;
    th[i] = dv ? x[o] + t * dv[o] : x[o];
  }
  const long long N = ag.g.N;
  const float* Tj = T + (size_t)K[j] * N;
  const float* rj = r + (size_t)j * N;
  double acc[P];
#pragma unroll
  for (int i = 0; i < P; ++i) acc[i] = 0.0;
  for (long long vox = (long long)blockIdx.x * blockDim.x + threadIdx.x;
       vox < N; vox += (long long)gridDim.x * blockDim.x) {
    Pos<D> pos = make_pos<D>(ag.g, vox);
    double W, dW[D], xi[D];
    aff_warp<D>(Tj, ag, pos, th, W, dW);
    aff_xi<D>(ag, pos, xi);
    const double rv = (double)rj[vox];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double q = rv * dW[a];
#pragma unroll
      for (int e = 0; e < D; ++e) acc[a * D + e] += q * xi[e];
      acc[D * D + a] += q;
    }
  }
  Blk blk{(int)blockIdx.x, (int)gridDim.x};
  block_partials<P>(acc, 0u, part + (size_t)j * P * gridDim.x, blk);
}

// g[j][i] = sum of the partials in block order + the penalty's share.
__global__ void aff_pgrad_sum_kernel(const double* __restrict__ part, int nb,
                                     int nk, int P,
                                     const double* __restrict__ gpen,
                                     double* __restrict__ g) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nk * P) return;
  const int j = e / P, i = e - j * P;
  const double* pj = part + (size_t)j * P * nb + (size_t)i * nb;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += pj[b];
  g[e] = s + gpen[i] / nk;
}

// ------------------------------------------------------------------ L-BFGS
// Pairs live in a ring of `mem` slots: slot (head + i) % mem is the i-th
// oldest of npairs.

__device__ __forceinline__ double aff_dot(const double* a, const double* b,
                                          int n) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += a[i] * b[i];
  return aff_block_sum(s);
}

// d = -H g by the two-loop recursion (gamma = s.y / y.y of the newest
// pair), or -g / max|g| without pairs; slope = g.d.  A direction that is
// not a descent direction drops the pairs and restarts from -g / max|g|.
__global__ __launch_bounds__(kAffThreads) void aff_lbfgs_dir_kernel(
    AffState* __restrict__ st, const double* __restrict__ g,
    double* __restrict__ d, const double* __restrict__ S,
    const double* __restrict__ Y, int nP, int mem) {
  __shared__ double alpha[16];
  __shared__ int s_np;
  if (threadIdx.x == 0) s_np = st->npairs;
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    const int np = s_np;
    if (np > 0) {
      for (int i = threadIdx.x; i < nP; i += blockDim.x) d[i] = g[i];
      __syncthreads();
      for (int m = np - 1; m >= 0; --m) {
        const int slot = (st->head + m) % mem;
        const double* s = S + (size_t)slot * nP;
        const double* y = Y + (size_t)slot * nP;
        const double a = st->rho[slot] * aff_dot(s, d, nP);
        if (threadIdx.x == 0) alpha[m] = a;
        for (int i = threadIdx.x; i < nP; i += blockDim.x) d[i] -= a * y[i];
        __syncthreads();
      }
      const int newest = (st->head + np - 1) % mem;
      const double* sn = S + (size_t)newest * nP;
      const double* yn = Y + (size_t)newest * nP;
      const double gamma = aff_dot(sn, yn, nP) / aff_dot(yn, yn, nP);
      for (int i = threadIdx.x; i < nP; i += blockDim.x) d[i] *= gamma;
      __syncthreads();
      for (int m = 0; m < np; ++m) {
        const int slot = (st->head + m) % mem;
        const double* s = S + (size_t)slot * nP;
        const double* y = Y + (size_t)slot * nP;
        const double b = st->rho[slot] * aff_dot(y, d, nP);
        const double am = alpha[m];
        for (int i = threadIdx.x; i < nP; i += blockDim.x)
          d[i] += (am - b) * s[i];
        __syncthreads();
      }
      for (int i = threadIdx.x; i < nP; i += blockDim.x) d[i] = -d[i];
    } else {
      double mx = 0.0;
      for (int i = threadIdx.x; i < nP; i += blockDim.x)
        mx = fmax(mx, fabs(g[i]));
      const double gmax = aff_block_max(mx);
      for (int i = threadIdx.x; i < nP; i += blockDim.x)
        d[i] = gmax == 0.0 ? 0.0 : -g[i] / gmax;
    }
    __syncthreads();
    const double slope = aff_dot(g, d, nP);
    if (slope < 0.0 || np == 0) {
      if (threadIdx.x == 0) st->slope = slope;
      break;
    }
    if (threadIdx.x == 0) {                      // restart
      st->npairs = 0;
      s_np = 0;
    }
    __syncthreads();
  }
}

// Armijo test of the trial t whose objective the finalize kernel just
// wrote: J_t <= J + c1 t slope.
__global__ void aff_accept_kernel(AffState* __restrict__ st,
                                  const AffScal* __restrict__ sc, double t,
                                  double c1) {
  if (threadIdx.x != 0) return;
  const double Jt = sc->J;
  st->Jt = Jt;
  st->bad = sc->bad;
  st->accepted = (Jt <= st->J + c1 * t * st->slope) ? 1 : 0;
  if (st->accepted) st->t = t;
}

// After the gradient at x_new = x + t d: keep the pair (s, y) if
// s.y > 1e-10 |s| |y|, move x and g, and evaluate the stop test.
__global__ __launch_bounds__(kAffThreads) void aff_update_kernel(
    AffState* __restrict__ st, double* __restrict__ x,
    const double* __restrict__ d, double* __restrict__ g,
    const double* __restrict__ gn, double* __restrict__ S,
    double* __restrict__ Y, int nP, int mem, double tol_J, double tol_u) {
  const double t = st->t;
  const int np = st->npairs;
  const int slot = np < mem ? (st->head + np) % mem : st->head;
  double* s = S + (size_t)slot * nP;
  double* y = Y + (size_t)slot * nP;
  double ss = 0.0, yy = 0.0, sy = 0.0, dd = 0.0;
  for (int i = threadIdx.x; i < nP; i += blockDim.x) {
    const double xn = x[i] + t * d[i];
    const double si = xn - x[i], yi = gn[i] - g[i];
    ss += si * si;
    yy += yi * yi;
    sy += si * yi;
    dd += d[i] * d[i];
  }
  ss = aff_block_sum(ss);
  yy = aff_block_sum(yy);
  sy = aff_block_sum(sy);
  dd = aff_block_sum(dd);
  const bool keep = sy > 1e-10 * sqrt(ss) * sqrt(yy);
  for (int i = threadIdx.x; i < nP; i += blockDim.x) {
    const double xn = x[i] + t * d[i];
    if (keep) {
      s[i] = xn - x[i];
      y[i] = gn[i] - g[i];
    }
    x[i] = xn;
    g[i] = gn[i];
  }
  if (threadIdx.x == 0) {
    if (keep) {
      st->rho[slot] = 1.0 / sy;
      if (np < mem) st->npairs = np + 1;
      else st->head = (st->head + 1) % mem;
    }
    const double Jp = st->J;
    st->J = st->Jt;
    st->iters += 1;
    const double rms = t * sqrt(dd / nP);
    st->stop = ((Jp - st->Jt) <= tol_J * fabs(Jp) && rms <= tol_u) ? 1 : 0;
  }
}

// x = theta[K] (gather), or theta[K] = x (scatter).
__global__ void aff_gather_kernel(double* __restrict__ x,
                                  const double* __restrict__ theta,
                                  const int* __restrict__ K, int nk, int P,
                                  int scatter) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nk * P) return;
  const int j = e / P, i = e - j * P;
  double* th = const_cast<double*>(theta) + (size_t)K[j] * P + i;
  if (scatter) *th = x[e];
  else x[e] = *th;
}

// Temporal predictors on parameters [n][P] (float64): the linear
// interpolation of the coarsest level, and eq. (2) (zeta = omega + xi,
// (M + beta D^T D) xi = M (eta - omega), shared factorisation) on finer
// levels; Y and Z receive the prediction.
__global__ void aff_linear_predict_kernel(double* __restrict__ Y,
                                          double* __restrict__ Z, LinTab tab,
                                          int n, int P) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * P) return;
  const int k = e / P, i = e - k * P;
  const double v = tab.wl[k] * Y[(size_t)tab.left[k] * P + i] +
                   tab.wr[k] * Y[(size_t)tab.right[k] * P + i];
  Z[e] = v;
}

__global__ void aff_ls_predict_kernel(double* __restrict__ Y,
                                      double* __restrict__ Z, ThomasTab tab,
                                      int n, int P, double beta,
                                      double* __restrict__ dp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  double prev = 0.0;
  for (int k = 0; k < n; ++k) {
    const double rhs = tab.mask[k] ? Y[(size_t)k * P + i] - Z[(size_t)k * P + i]
                                   : 0.0;
    prev = (rhs + beta * prev) * tab.invp[k];
    dp[(size_t)k * P + i] = prev;
  }
  double xi = 0.0;
  for (int k = n - 1; k >= 0; --k) {
    xi = (k == n - 1) ? dp[(size_t)k * P + i]
                      : dp[(size_t)k * P + i] - tab.cp[k] * xi;
    const double z = Z[(size_t)k * P + i] + xi;
    Z[(size_t)k * P + i] = z;
    Y[(size_t)k * P + i] = z;
  }
}

// u_k(x) = B_k xi(x) + b_k of every frame into a float32 field [n][D][N].
template <int D>
__global__ void aff_field_kernel(const double* __restrict__ theta, int n,
                                 AffGeom ag, float* __restrict__ u) {
  constexpr int P = D * D + D;
  const long long N = ag.g.N;
  const long long total = (long long)n * N;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
       e < total; e += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(e / N);
    const long long vox = e - (long long)k * N;
    Pos<D> pos = make_pos<D>(ag.g, vox);
    double xi[D];
    aff_xi<D>(ag, pos, xi);
    const double* th = theta + (size_t)k * P;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double s = 0.0;
#pragma unroll
      for (int f = 0; f < D; ++f) s += th[a * D + f] * xi[f];
      u[((size_t)k * D + a) * N + vox] = (float)(s + th[D * D + a]);
    }
  }
}

// ------------------------------------------------------------ launchers

AffShape aff_shape(const AffGeom& ag, int nk) {
  AffShape sh;
  const int K1 = nk + 1;
  const int Kt = (K1 + 15) / 16;
  const int NTt = Kt * (Kt + 1) / 2;
  const long long nch = (ag.g.N + kAffV - 1) / kAffV;
  // kAffGramTiles 16 x 16 tiles per wave before the tiles are spread over
  // groups that each warp the frames again
  const int per_group = kAffGramTiles * (kAffThreads / kWave);
  sh.groups = (NTt + per_group - 1) / per_group;
  sh.E = K1 * (K1 + 1) / 2;
  sh.nb_gram = (int)(nch < kAffGramBlocks ? nch : kAffGramBlocks);
  sh.nb_resid = (int)(nch < 2 * kCUs ? nch : 2 * kCUs);
  const long long per = (ag.g.N + kAffThreads - 1) / kAffThreads;
  sh.nb_pgrad = (int)(per < kAffPgradBlocks ? per : kAffPgradBlocks);
  const int P = ag.d * ag.d + ag.d;
  sh.lds_gram = (size_t)(((nk * P + 1) & ~1) + 16 * Kt * (kAffV + 1)) *
                sizeof(double);
  const int Ktr = (nk + 15) / 16;
  sh.lds_resid = (size_t)(16 * Ktr * (kAffV + 1)) * sizeof(double);
  return sh;
}

// Dynamic LDS above 64 KiB has to be allowed per kernel.
static hipError_t aff_allow_lds() {
  static hipError_t e = [] {
    const int cap = 156 * 1024;    // 160 KiB per CU, less static LDS
    hipError_t r = hipSuccess;
    const void* ks[] = {(const void*)aff_gram_kernel<2>,
                        (const void*)aff_gram_kernel<3>,
                        (const void*)aff_resid_kernel<16, 256>,
                        (const void*)aff_resid_kernel<40, 640>,
                        (const void*)aff_resid_kernel<64, 512>};
    for (const void* k : ks) {
      hipError_t q = hipFuncSetAttribute(
          k, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
      if (q != hipSuccess) r = q;
    }
    return r;
  }();
  return e;
}

hipError_t launch_aff_objective(const float* T, const int* K, int nk,
                                const double* x, const double* dv, double t,
                                const AffGeom& ag, double lam, AffBufs b,
                                bool grad, bool reuse_gram, hipStream_t s) {
  const AffShape sh = aff_shape(ag, nk);
  hipError_t e = aff_allow_lds();
  if (e != hipSuccess) return e;
  if (!reuse_gram) {
    dim3 grid(sh.nb_gram, sh.groups);
    if (ag.d == 2)
      aff_gram_kernel<2><<<grid, kAffThreads, sh.lds_gram, s>>>(
          T, K, nk, x, dv, t, ag, b.part, sh.E, b.W);
    else
      aff_gram_kernel<3><<<grid, kAffThreads, sh.lds_gram, s>>>(
          T, K, nk, x, dv, t, ag, b.part, sh.E, b.W);
    aff_sum_kernel<<<(sh.E + 255) / 256, 256, 0, s>>>(b.part, sh.nb_gram,
                                                       sh.E, b.tot);
  }
  aff_finalize_kernel<<<1, kAffThreads, 0, s>>>(b.tot, nk, ag, x, dv, t, lam,
                                                b.sc, b.mu, b.Rc, b.gpen,
                                                grad ? 1 : 0);
  if (!grad) return hipGetLastError();
  {
    // one wave per 16-row tile: up to 10 tiles in one block (KS = 40,
    // 640 threads), else two block rows of at most 8 waves (|K| <= 256)
    const int Kt = (nk + 15) / 16;
    decltype(&aff_resid_kernel<16, 256>) rk;
    int rows = 1, waves = Kt;
    if (Kt <= 4) {
      rk = aff_resid_kernel<16, 256>;
    } else if (Kt <= 10) {
      rk = aff_resid_kernel<40, 640>;
    } else {
      rk = aff_resid_kernel<64, 512>;
      rows = 2;
      waves = (Kt + 1) / 2;
    }
    rk<<<dim3(sh.nb_resid, rows), waves * kWave, sh.lds_resid, s>>>(
        b.W, nk, ag.g.N, b.mu, b.Rc, b.r);
  }
  dim3 gp(sh.nb_pgrad, nk);
  if (ag.d == 2)
    aff_pgrad_kernel<2><<<gp, kAffThreads, 0, s>>>(T, K, x, dv, t, ag, b.r,
                                                   b.gpart);
  else
    aff_pgrad_kernel<3><<<gp, kAffThreads, 0, s>>>(T, K, x, dv, t, ag, b.r,
                                                   b.gpart);
  const int P = ag.d * ag.d + ag.d;
  aff_pgrad_sum_kernel<<<(nk * P + 255) / 256, 256, 0, s>>>(
      b.gpart, sh.nb_pgrad, nk, P, b.gpen, b.gout);
  return hipGetLastError();
}

__global__ void aff_state_init_kernel(AffState* __restrict__ st,
                                      const AffScal* __restrict__ sc) {
  if (threadIdx.x != 0) return;
  st->J = sc->J;
  st->Jt = sc->J;
  st->slope = 0.0;
  st->t = 0.0;
  st->npairs = 0;
  st->head = 0;
  st->iters = 0;
  st->accepted = 0;
  st->stop = 0;
  st->bad = sc->bad;
}

hipError_t launch_aff_state_init(AffState* st, const AffScal* sc,
                                 hipStream_t s) {
  aff_state_init_kernel<<<1, 64, 0, s>>>(st, sc);
  return hipGetLastError();
}

hipError_t launch_aff_direction(AffState* st, const double* g, double* d,
                                const double* S, const double* Y, int nP,
                                int mem, hipStream_t s) {
  aff_lbfgs_dir_kernel<<<1, kAffThreads, 0, s>>>(st, g, d, S, Y, nP, mem);
  return hipGetLastError();
}

hipError_t launch_aff_accept(AffState* st, const AffScal* sc, double t,
                             double c1, hipStream_t s) {
  aff_accept_kernel<<<1, 64, 0, s>>>(st, sc, t, c1);
  return hipGetLastError();
}

hipError_t launch_aff_update(AffState* st, double* x, const double* d,
                             double* g, const double* gn, double* S,
                             double* Y, int nP, int mem, double tol_J,
                             double tol_u, hipStream_t s) {
  aff_update_kernel<<<1, kAffThreads, 0, s>>>(st, x, d, g, gn, S, Y, nP, mem,
                                              tol_J, tol_u);
  return hipGetLastError();
}

hipError_t launch_aff_gather(double* x, const double* theta, const int* K,
                             int nk, int P, bool scatter, hipStream_t s) {
  aff_gather_kernel<<<(nk * P + 255) / 256, 256, 0, s>>>(x, theta, K, nk, P,
                                                         scatter ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_aff_linear_predict(double* Y, double* Z, LinTab tab, int n,
                                     int P, hipStream_t s) {
  aff_linear_predict_kernel<<<(n * P + 255) / 256, 256, 0, s>>>(Y, Z, tab, n,
                                                                P);
  // every frame takes the prediction (frames of K_q are kept: weight 1)
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(Y, Z, (size_t)n * P * sizeof(double),
                        hipMemcpyDeviceToDevice, s);
}

hipError_t launch_aff_ls_predict(double* Y, double* Z, ThomasTab tab, int n,
                                 int P, double beta, double* dp,
                                 hipStream_t s) {
  aff_ls_predict_kernel<<<1, 64, 0, s>>>(Y, Z, tab, n, P, beta, dp);
  return hipGetLastError();
}

hipError_t launch_aff_field(const double* theta, int n, const AffGeom& ag,
                            float* u, hipStream_t s) {
  const long long total = (long long)n * ag.g.N;
  const int nb = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  if (ag.d == 2)
    aff_field_kernel<2><<<nb, 256, 0, s>>>(theta, n, ag, u);
  else
    aff_field_kernel<3><<<nb, 256, 0, s>>>(theta, n, ag, u);
  return hipGetLastError();
}

}  // namespace stml
