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
// max instead of sum.  Writes part[v * gridDim.x + blockIdx.x].
template <int NV>
__device__ void block_partials(const double (&vals)[NV], unsigned maxmask,
                               double* __restrict__ part) {
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
  if (threadIdx.x < NV) {
    int v = threadIdx.x;
    bool mx = (maxmask >> v) & 1u;
    double s = red[0][v];
    for (int i = 1; i < nw; ++i) s = mx ? fmax(s, red[i][v]) : s + red[i][v];
    part[(size_t)v * gridDim.x + blockIdx.x] = s;
  }
}

// Totals of NV values from nb partial slots each; every thread of the block
// receives them.
template <int NV>
__device__ void reduce_partials(const double* __restrict__ part, int nb,
                                unsigned maxmask, double (&out)[NV]) {
  __shared__ double red[kMaxChunks][NV];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    acc[v] = ((maxmask >> v) & 1u) ? -1.0e300 : 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    double x[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) x[v] = part[(size_t)v * nb + i];
#pragma unroll
    for (int v = 0; v < NV; ++v)
      acc[v] = ((maxmask >> v) & 1u) ? fmax(acc[v], x[v]) : acc[v] + x[v];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    bool mx = (maxmask >> v) & 1u;
    double s = mx ? wave_max(acc[v]) : wave_sum(acc[v]);
    if (lane == 0) red[w][v] = s;
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    bool mx = (maxmask >> v) & 1u;
    double t = red[0][v];
    for (int i = 1; i < nw; ++i) t = mx ? fmax(t, red[i][v]) : t + red[i][v];
    out[v] = t;
  }
  __syncthreads();
}

}  // namespace stml
