// Deterministic float64 reductions without grid-wide fences.
//
// A producing kernel writes one partial per block into fixed slots
// (block_partials).  The kernel that needs the total reduces the slots in
// slot order at its start (reduce_partials): every block of the consumer
// computes the same value, and the kernel boundary makes the producer's
// stores visible on every XCD.  A per-block agent-scope fence would write
// back the whole L2 of a multi-XCD device once per block.  The order of
// every sum depends only on slot indices, so repeated runs are bitwise
// identical.
#pragma once

#include "stml_dev.h"

namespace stml {

// vals[v]: this thread's contribution to value v; bit v of maxmask selects
// max instead of sum.  Writes part[v * blk.n + blk.id].
template <int NV>
__device__ void block_partials(const double (&vals)[NV], unsigned maxmask,
                               double* __restrict__ part, Blk blk) {
  __shared__ double red[kMaxChunks][NV];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double x = ((maxmask >> v) & 1u) ? wave_max(vals[v]) : wave_sum(vals[v]);
    if (lane == 0) red[w][v] = x;
  }
  __syncthreads();
  if (NV <= 4) {
    // wave 0 combines the waves' values: lane i holds wave i's
    if (w == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const bool mx = (maxmask >> v) & 1u;
        const double id = mx ? -__builtin_inf() : 0.0;
        const double x = lane < nw ? red[lane][v] : id;
        const double s = mx ? wave_max(x) : wave_sum(x);
        if (lane == 0) part[(size_t)v * blk.n + blk.id] = s;
      }
    }
  } else if (threadIdx.x < NV) {
    // many values: one thread per value, in parallel
    int v = threadIdx.x;
    bool mx = (maxmask >> v) & 1u;
    double s = red[0][v];
    for (int i = 1; i < nw; ++i) s = mx ? fmax(s, red[i][v]) : s + red[i][v];
    part[(size_t)v * blk.n + blk.id] = s;
  }
}
template <int NV>
__device__ void block_partials(const double (&vals)[NV], unsigned maxmask,
                               double* __restrict__ part) {
  block_partials<NV>(vals, maxmask, part, grid_blk());
}

// Totals of NV values from nb partial slots each; every thread of the block
// receives them.  Up to 64 slots, every wave sums them by a wave reduction
// (lane l holds slot l); more slots are summed in 256
// fixed strands (strand v: slots v, v + 256, ...), whichever threads
// compute them, and the strands then in a fixed tree.  Either way the order
// depends on nb only, not on the block size.
// LDS a reduction of NV values needs beyond 64 slots (reduce_partials_in).
template <int NV>
constexpr int reduce_lds_doubles() {
  return NV * 4 * kWave + NV;
}

template <int NV>
__device__ void reduce_partials_in(const double* __restrict__ part, int nb,
                                   unsigned maxmask, double (&out)[NV],
                                   double* lds);

template <int NV>
__device__ void reduce_partials(const double* __restrict__ part, int nb,
                                unsigned maxmask, double (&out)[NV]) {
  __shared__ double lds[reduce_lds_doubles<NV>()];
  reduce_partials_in<NV>(part, nb, maxmask, out, lds);
}

// The same with the caller's LDS (reduce_lds_doubles<NV>() doubles), which
// it may reuse once this returns.
template <int NV>
__device__ void reduce_partials_in(const double* __restrict__ part, int nb,
                                   unsigned maxmask, double (&out)[NV],
                                   double* lds) {
  if (nb <= kWave) {
    // few slots: every wave sums them itself (lane l takes slot l), without
    // LDS or barriers; the order depends on nb only (more slots would be
    // read again by every wave of every block)
    const int lane = threadIdx.x & (kWave - 1);
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
      acc[v] = ((maxmask >> v) & 1u) ? -1.0e300 : 0.0;
    for (int i = lane; i < nb; i += kWave) {
      double x[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) x[v] = part[(size_t)v * nb + i];
#pragma unroll
      for (int v = 0; v < NV; ++v)
        acc[v] = ((maxmask >> v) & 1u) ? fmax(acc[v], x[v]) : acc[v] + x[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
      out[v] = ((maxmask >> v) & 1u) ? wave_max(acc[v]) : wave_sum(acc[v]);
    return;
  }
  constexpr int kStrands = 4 * kWave;
  double(*red)[kStrands] = reinterpret_cast<double(*)[kStrands]>(lds);
  double* tot = lds + NV * kStrands;
  for (int v0 = threadIdx.x; v0 < kStrands; v0 += blockDim.x) {
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
      acc[v] = ((maxmask >> v) & 1u) ? -1.0e300 : 0.0;
    for (int i = v0; i < nb; i += kStrands) {
      double x[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) x[v] = part[(size_t)v * nb + i];
#pragma unroll
      for (int v = 0; v < NV; ++v)
        acc[v] = ((maxmask >> v) & 1u) ? fmax(acc[v], x[v]) : acc[v] + x[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) red[v][v0] = acc[v];
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    const int l = threadIdx.x;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      bool mx = (maxmask >> v) & 1u;
      double s = red[v][l];
      for (int k = 1; k < 4; ++k)
        s = mx ? fmax(s, red[v][l + k * kWave]) : s + red[v][l + k * kWave];
      s = mx ? wave_max(s) : wave_sum(s);
      if (l == 0) tot[v] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = tot[v];
  __syncthreads();
}

}  // namespace stml
