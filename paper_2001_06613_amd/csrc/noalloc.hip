// Objective entry point that allocates nothing: the evaluation kernels of
// stml_eval, with their scratch (reduction partials, scalars, frame list)
// in one static device array per GPU instead of a context workspace.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "../../include/stml.h"
#include "launch.h"

using namespace stml;

namespace {

// Scratch layout: [partials of the evaluation | Scal | frame list].  The
// evaluation writes at most 16 float64 values per block, for at most
// kMaxTileBlocks blocks (the default cap: the launch shape of stml_eval on a
// fresh context).
constexpr size_t kPartBytes = (size_t)16 * kMaxTileBlocks * sizeof(double);
constexpr size_t kScalOff = kPartBytes;
constexpr size_t kKOff = kScalOff + ((sizeof(Scal) + 255) / 256) * 256;
constexpr size_t kScratchBytes = kKOff + STML_MAX_FRAMES * sizeof(int);
static_assert(kScratchBytes == STML_NOALLOC_SCRATCH_BYTES,
              "header constant out of date");

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};          // device address of scratch, per GPU
thread_local std::string g_err;

int fail(int code, const char* msg) {
  g_err = msg;
  return code;
}

}  // namespace

// Each GPU the library runs on holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

const char* stml_noalloc_last_error(void) { return g_err.c_str(); }

int stml_eval_noalloc(const stml_opts* o, int n, const int* extent, double h,
                      const float* frames_dev, const int* frames, int nk,
                      const float* u_dev, double* out_JDSP, float* grad_dev,
                      float* dW_dev, void* hip_stream) {
  if (!o || !extent || !frames || !frames_dev || !u_dev || !out_JDSP ||
      !grad_dev || !dW_dev)
    return fail(STML_EINVAL, "null pointer");
  if ((o->dim != 2 && o->dim != 3) ||
      (o->regulariser != STML_REG_DIFFUSION &&
       o->regulariser != STML_REG_CURVATURE) ||
      !(o->alpha >= 0) || !(o->lambda >= 0) || !(h > 0))
    return fail(STML_EINVAL, "invalid options or spacing");
  const int dim = o->dim;
  long long N = 1;
  for (int a = 0; a < dim; ++a) {
    if (extent[a] < 1) return fail(STML_EINVAL, "extent must be >= 1");
    N *= extent[a];
  }
  if (n < 1 || n > STML_MAX_FRAMES)
    return fail(STML_ENOMEM, "n above the scratch maximum (STML_MAX_FRAMES)");
  if (N > (1LL << 30) || (long long)n * dim * N > 2000000000LL)
    return fail(STML_EINVAL, "frames above 2^30 voxels or 2e9 values");
  if (nk < 1 || nk > n) return fail(STML_EINVAL, "need 1..n frames in K");
  int hk[STML_MAX_FRAMES];
  for (int i = 0; i < nk; ++i) {
    if (frames[i] < 0 || frames[i] >= n || (i && frames[i] <= frames[i - 1]))
      return fail(STML_EINVAL, "frame list must be ascending in [0, n)");
    hk[i] = frames[i];
  }
  Geom g = make_geom(dim, extent, h);
  g.tile_cap = kMaxTileBlocks;
  g.vox_cap = kMaxTileBlocks;
  g.hv_target = kHvBlocks;
  if (tile_blocks(g) > kMaxTileBlocks)
    return fail(STML_ENOMEM, "evaluation grid above the scratch maximum");
  const Model md = make_model(dim, h, nk, o->alpha, o->lambda,
                              o->regulariser);

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(STML_EDEVICE, "no current HIP device");
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
      void* p = nullptr;
      hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(STML_EDEVICE, "hipGetSymbolAddress(scratch) failed");
      g_ptr[dev] = p;
    }
    base = static_cast<char*>(g_ptr[dev]);
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  RedBuf rb{reinterpret_cast<double*>(base)};     // only kRegEval is used
  double* part = rb.region(kRegEval);
  if ((char*)part != base) return fail(STML_EDEVICE, "scratch layout");
  Scal* sc = reinterpret_cast<Scal*>(base + kScalOff);
  int* Kd = reinterpret_cast<int*>(base + kKOff);

  if (hipMemcpyAsync(Kd, hk, nk * sizeof(int), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return fail(STML_EDEVICE, "frame list copy failed");
  if (launch_eval(dim, frames_dev, u_dev, Kd, g, md, grad_dev, dW_dev, rb,
                  sc, s, true, 0) != hipSuccess)
    return fail(STML_EDEVICE, "evaluation launch failed");
  Scal hs;
  if (hipMemcpyAsync(&hs, sc, sizeof(Scal), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(STML_EDEVICE, "reading the objective failed");
  out_JDSP[0] = hs.J;
  out_JDSP[1] = hs.D;
  out_JDSP[2] = hs.S;
  out_JDSP[3] = hs.P;
  g_err.clear();
  return STML_OK;
}
