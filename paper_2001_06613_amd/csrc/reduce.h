// Deterministic single-pass block reductions in float64.
//
// Every block writes its partial sums to fixed slots; the last block to
// finish (found with one agent-scope atomic counter per kernel) sums the
// slots in index order and publishes the scalars.  The order of the final
// sum depends only on the slot index, never on which block finished last,
// so repeated runs give bitwise-identical results.
#pragma once

#include "stml_dev.h"

namespace stml {

// vals[v] is this thread's contribution to value v.  maxmask bit v set means
// value v is reduced with max instead of sum.  On return, in the last block
// only, out[v] holds the grid-wide result for every thread and the function
// returns true.
template <int NV>
__device__ bool grid_reduce(const double (&vals)[NV], unsigned maxmask,
                            double* __restrict__ part,
                            unsigned* __restrict__ counter,
                            double (&out)[NV]) {
  __shared__ double red[kMaxChunks][NV > 0 ? NV : 1];
  __shared__ bool last;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int nb = gridDim.x;
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
    part[(size_t)v * nb + blockIdx.x] = s;
    __threadfence();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == (unsigned)(nb - 1));
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    bool mx = (maxmask >> v) & 1u;
    double s = mx ? -1.0e300 : 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
      double x = part[(size_t)v * nb + i];
      s = mx ? fmax(s, x) : s + x;
    }
    s = mx ? wave_max(s) : wave_sum(s);
    __syncthreads();
    if (lane == 0) red[w][v] = s;
    __syncthreads();
    double t = red[0][v];
    for (int i = 1; i < nw; ++i) t = mx ? fmax(t, red[i][v]) : t + red[i][v];
    out[v] = t;
  }
  if (threadIdx.x == 0) *counter = 0u;
  return true;
}

}  // namespace stml
